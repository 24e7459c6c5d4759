// kernels_xdrop.hip -- X-drop seed extension on gfx950: sixteen extension
// sides per wavefront, four lanes per side, a persistent work queue.
//
// The rule (Sec. 2, Sec. 5.2, Sec. 7.2) evaluated antidiagonal by
// antidiagonal k = i + j in sheared coordinates d = j - i (Sec. 6.2): a
// candidate cell is removed when its H falls more than X below the best score
// of the earlier antidiagonals, and the next antidiagonal is evaluated from
// one step before the first survivor to one step after the last.
//
// Layout.  A side owns a window of 128 diagonals d = base + 2*pos + (k & 1),
// pos = 0..63: the 64 cells of one antidiagonal, sixteen per lane (lane g of
// the side's quad holds pos 16g .. 16g+15).  Per diagonal a lane keeps the
// latest H and the E / F values it passes right / down; E comes from d - 1
// and F from d + 1 of the previous antidiagonal (the other parity), H of the
// diagonal predecessor from the same slot, so one quad-DPP per antidiagonal
// moves a value across a lane boundary.
//
// Offset frame.  Every stored value of antidiagonal k is kept minus k*e (e
// the gap extension score), so a gap step adds nothing:
//   E'(k, d) = max(E'(k-1, d-1), H'(k-1, d-1) + o),  F' likewise from d+1,
//   H'(k, d) = max(H'(k-2, d) + s - 2e, E'(k, d), F'(k, d)),
// with o the gap open score.  Per cell: one add of the substitution byte
// (SDWA), a three-way max, the prune compare and select, the open add and
// two max.
//
// Pruning without range masks.  Only H of a removed cell is set to minus
// infinity.  Its E and F may keep values, but every such value is below the
// threshold of its antidiagonal, and thresholds (in the offset frame) never
// fall, so no later survivor's H, no prune decision and no survivor range
// can change.  A cell outside the candidate range inside the matrix can only
// be revived through its diagonal predecessor; its substitution score is
// replaced by -128, which keeps it below the threshold whenever
// X < 128 + 2|e| (the planner checks this).  Cells past the matrix's far
// edges (j > N or i > M) can hold values carried out of the last column or
// row; they never count as survivors, values never flow back from them, and
// with non-positive gap scores they never beat the cell they came from, so
// they never become the best cell either.
//
// Substitution scores come from one v_perm_b32 per four cells: the codes'
// XOR selects byte 0 (match) or 1..3 (mismatch) of a table, byte 4..7
// (-128) where the candidate range excludes the cell.  Codes are staged per
// side in LDS rings (query reversed) and read as one unaligned 16-byte run
// per lane and antidiagonal.
//
// Traceback codes (the form with CIGAR): per antidiagonal and side only the
// 8-cell groups (one code dword each) that hold candidate cells, packed one
// antidiagonal after the other; per antidiagonal a byte with its first and
// last group and the window base's step, per 64 antidiagonals the stream
// offset and the window base (the layout of xdl_tb_table / xdl_tb_stream).
// Lane gl's groups are 2gl and 2gl + 1; cell m of a lane sits in its group
// m >> 3 at nibble 7 - (m & 7);
// its bits, high to low: F passed down opened from H (F-open), E passed right
// opened from H (E-open), H not from E, H not from the diagonal -- so H takes
// the diagonal, then E, then F, and a gap opens before it extends.  The codes
// of a survivor are those of the pruned recurrence: every value compared on
// the optimal path is at or above its antidiagonal's threshold, hence not a
// stale one.
//
// Best cell: keys (H' << 6 | pos) give, per antidiagonal, the highest score
// and among equals the largest d (smallest i); the running best is the score
// with a key (-i, -j) for ties.  Survivor bounds come from per-lane survivor
// masks and quad DPP minima / maxima.  The window slides by one cell when the
// candidate range reaches an edge; a region wider than 64 cells goes to the
// widening queue (the one-side kernel with wider windows).
#include "internal.h"

#include <type_traits>

namespace alnk {

namespace {

constexpr int XC = 16;             // cells per lane per antidiagonal
constexpr int XNEG = -(1 << 22);   // minus infinity in the offset frame
constexpr int XBIG = (1 << 29);    // threshold of an idle side: nothing survives
constexpr int kRing = 128;         // codes per ring
constexpr int kRingMirror = 32;    // first bytes repeated after the ring
constexpr int kRingStride = kRing + kRingMirror;
constexpr int kSides = 16;         // sides per wavefront
constexpr int kZBias = 1 << 20;    // Z-drop: bias of diagonal differences

// quad DPP: lane l reads lane l-1 (shr) / l+1 (shl) of its quad; the quad's
// edge lane gets `edge`.  quad_perm always names a lane of the quad, so every
// lane reads a defined value and bound_ctrl changes nothing; with it and no
// old value the compiler folds the move into the instruction that uses it.
template <int CTRL> __device__ __forceinline__ int quad_dpp(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
__device__ __forceinline__ int quad_shr1(int v, int edge, bool first) {
  const int x = quad_dpp<0x90>(v); // quad_perm 0,0,1,2
  return first ? edge : x;
}
__device__ __forceinline__ int quad_shl1(int v, int edge, bool last) {
  const int x = quad_dpp<0xF9>(v); // quad_perm 1,2,3,3
  return last ? edge : x;
}
__device__ __forceinline__ int quad_max(int v) {
  v = max(v, quad_dpp<0xB1>(v)); // quad_perm 1,0,3,2
  v = max(v, quad_dpp<0x4E>(v)); // quad_perm 2,3,0,1
  return v;
}
__device__ __forceinline__ int quad_min(int v) {
  v = min(v, quad_dpp<0xB1>(v));
  v = min(v, quad_dpp<0x4E>(v));
  return v;
}
__device__ __forceinline__ int quad_bcast0(int v) {
  return quad_dpp<0x00>(v); // quad_perm 0,0,0,0
}

// 16 ring bytes from `addr` (any alignment; the mirror covers the wrap)
__device__ __forceinline__ void ring16(const uint8_t *ring, int addr, uint32_t (&w)[4]) {
  const uint32_t *d = reinterpret_cast<const uint32_t *>(ring + (addr & ~3));
  uint32_t x[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) x[k] = d[k];
  const uint32_t sh = (uint32_t)addr & 3u;
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = __builtin_amdgcn_alignbyte(x[k + 1], x[k], sh);
}

// v = 2 v + bit, the bit taken from a compare's lane mask as a carry
__device__ __forceinline__ void shift_in(uint32_t &v, bool bit) {
  const unsigned long long km = __builtin_amdgcn_ballot_w64(bit);
  unsigned long long cc;
  asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(v), "=s"(cc) : "v"(v), "s"(km));
  (void)cc;
}

// byte b of the result = byte 3 - b of x
__device__ __forceinline__ uint32_t byte_reverse(uint32_t x) {
  return __builtin_amdgcn_perm(0u, x, 0x00010203u);
}

} // namespace

// three wavefronts per SIMD: the form with traceback needs a few registers
// more than fit, and spills two of them on its task-start path
// ZD: Z-drop (Sec. 9.3) instead of X-drop: a candidate is kept when its H
// plus its distance |d - d_best| from the best cell's diagonal reaches the
// threshold.  The thresholds then differ between diagonals, so the pruning
// above is made explicit: H, E and F of a removed cell or of a cell outside
// the candidate range are minus infinity, and only kept cells enter the
// antidiagonal's best.
// Four wavefronts per SIMD for the X-drop score form (128 VGPRs, no spill in
// the step), three with codes or Z-drop (they need more registers)
template <bool TB, bool ZD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(TB || ZD ? 3 : 4))) void
xdrop_lanes_kernel(XdlArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int lane = threadIdx.x & 63;
  const int gl = lane & 3;        // lane within the side's quad
  const int side = lane >> 2;     // side slot of this wavefront
  const bool qfirst = gl == 0, qlast = gl == 3;
  uint8_t *qring = smem + side * 2 * kRingStride;
  uint8_t *rring = qring + kRingStride;

  const int X = a.xdrop, go = a.gap_open, ge = a.gap_extend;
  // substitution table in the offset frame: byte 0 match, 1..3 mismatch,
  // 4..7 the out-of-range penalty
  const uint32_t m8 = (uint32_t)(a.match - 2 * ge) & 0xffu;
  const uint32_t x8 = (uint32_t)(a.mismatch - 2 * ge) & 0xffu;
  const uint32_t tab_lo = m8 | (x8 << 8) | (x8 << 16) | (x8 << 24);
  const uint32_t tab_hi = 0x80808080u;

  int H0[XC], H1[XC], E0[XC], F0[XC], E1[XC], F1[XC];
#pragma unroll
  for (int m = 0; m < XC; ++m) H0[m] = H1[m] = E0[m] = F0[m] = E1[m] = F1[m] = XNEG;

  // side state, equal across the quad
  bool active = false, exhausted = false;
  int task = 0, pair = 0, M = 0, N = 0, base = 0, k = 0, kE = 0, T = XBIG;
  int plo = 1, phi = 0, qtop = 0, rtop = 0;
  int best = 0;         // best score so far
  uint32_t best_key = 0; // its cell: (0xffff - i) << 16 | (0xffff - j)
  long long cells = 0;
  const uint8_t *Q = nullptr, *R = nullptr;
  // traceback: one byte per antidiagonal, a table entry per 64, the codes
  uint8_t *tb_meta = nullptr; // the side's region
  int tcur = 0;               // byte offset in the region of the next code dword
  int bprev = 0;              // window base of the antidiagonal before
  uint32_t mlo = 0, mhi = 0;  // lane gl: bytes of antidiagonals 32n + 8gl .. + 7, newest on top

  // 32 codes per call into a ring (the query reversed), padding (4) past
  // the sequence; lane gl stages codes top + 8gl .. top + 8gl + 7
  auto stage = [&](const uint8_t *src, int len, uint8_t *ring, int top, bool rev) {
    const int c0 = top + 8 * gl;
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int c = c0 + b;
      const uint32_t raw = src[min(c, len - 1)]; // clamped: issued unconditionally
      const uint32_t v = (c < len) ? min(raw, 4u) : 4u;
      if (b < 4) lo |= v << (8 * b);
      else hi |= v << (8 * (b - 4));
    }
    int at;
    if (rev) { // code c lives at (127 - c) mod 128
      const uint32_t rl = byte_reverse(hi), rh = byte_reverse(lo);
      lo = rl;
      hi = rh;
      at = (kRing - 8 - (c0 & (kRing - 1))) & (kRing - 1);
    } else {
      at = c0 & (kRing - 1);
    }
    *reinterpret_cast<uint2 *>(ring + at) = make_uint2(lo, hi);
    if (at < kRingMirror) *reinterpret_cast<uint2 *>(ring + kRing + at) = make_uint2(lo, hi);
  };

  for (;;) {
    // ---- idle sides take the next task (the list is longest first)
    bool need = !active && !exhausted;
    bool fresh = false;
    while (__ballot(need)) {
      if (need) {
        int t = 0;
        if (qfirst) t = atomicAdd(a.queue, 1);
        t = quad_bcast0(t);
        if (t >= a.ntasks) {
          exhausted = true;
        } else {
          task = t;
          pair = a.tasks[t].pair;
          M = a.b.q_len[pair];
          N = a.b.r_len[pair];
          if (M == 0 || N == 0) {
            if (qfirst) {
              aln_result *res = a.res + pair;
              res->score = 0;
              res->q_end = 0;
              res->r_end = 0;
              res->cells = 0;
            }
          } else {
            Q = a.b.q + a.b.q_off[pair];
            R = a.b.r + a.b.r_off[pair];
            if (TB) {
              const int nb = (M + N + 1 + 63) / 64;
              uint8_t *tbp = a.tb + a.tasks[t].tb_off;
              tb_meta = tbp;
              tcur = (int)xdl_tb_stream(nb);
              bprev = -64; // the first window base, set below
              mlo = 0;
              mhi = 1u << 24; // antidiagonal 0: no groups (first 1, last 0)
              if (qfirst) *reinterpret_cast<int2 *>(tbp + xdl_tb_table(nb)) = make_int2(0, -64);
            }
            fresh = true; // arrays reset below, outside this loop
            base = -64;
            k = 1;
            kE = ge;
            best = 0; // score 0 at (0,0)
            best_key = 0xffffffffu;
            T = -X - kE;
            plo = 31; // candidates of k = 1: d = -1, 1
            phi = 32;
            cells = 0;
            qtop = 0;
            rtop = 0;
            // rings start as padding
            for (int e = gl * 4; e < 2 * kRingStride; e += 16)
              *reinterpret_cast<uint32_t *>(qring + e) = 0x04040404u;
            active = true;
          }
        }
      }
      need = !active && !exhausted;
    }
    if (!__ballot(active)) break;
    // new sides: every slot minus infinity but the cell (0,0) with H = 0 at
    // d = 0 (pos 32, parity 0), whose E and F outputs are the gap open in the
    // frame of k = 1
    if (__ballot(fresh)) {
      if (fresh) {
#pragma unroll
        for (int m = 0; m < XC; ++m) H0[m] = H1[m] = E0[m] = F0[m] = E1[m] = F1[m] = XNEG;
        if (gl == 2) {
          H0[0] = 0;
          E0[0] = go;
          F0[0] = go;
        }
      }
    }

    // one antidiagonal of parity P (P == k & 1 for every active side)
    auto step = [&](auto ptag) {
      constexpr int P = decltype(ptag)::value;
      // ---- keep the rings ahead of the window (26 codes of margin; the
      // window moves at most two codes per antidiagonal pair)
      for (; P == 1;) {
        const int topq = ((k - base - P) >> 1) - 1;  // query code of pos 0
        const int topr = ((k + base + P) >> 1) + 62; // reference code of pos 63
        const bool sq = active && qtop < topq + 26;
        const bool sr = active && rtop < topr + 26;
        if (!__ballot(sq || sr)) break;
        if (sq) {
          stage(Q, M, qring, qtop, true);
          qtop += 32;
        }
        if (sr) {
          stage(R, N, rring, rtop, false);
          rtop += 32;
        }
      }
      // ---- this lane's codes: query i - 1 (descending) and reference j - 1
      uint32_t qw[4], rw[4];
      {
        const int cq = ((k - base - P) >> 1) - 1 - XC * gl;
        const int cr = ((k + base + P) >> 1) - 1 + XC * gl;
        ring16(qring, (kRing - 1 - cq) & (kRing - 1), qw);
        ring16(rring, cr & (kRing - 1), rw);
      }
      // ---- substitution bytes; cells outside [plo, phi] get the penalty
      uint32_t sc[4], inr_rev; // inr_rev: bit 15 - m set for cells m in range
      {
        const int lo = min(max(plo - XC * gl, 0), XC);
        const int hi = min(max(phi - XC * gl + 1, 0), XC);
        // hi >= lo always (an idle side has plo = phi + 1)
        inr_rev = ((1u << (hi - lo)) - 1u) << (XC - hi);
        const uint32_t out = ~(((1u << (hi - lo)) - 1u) << lo);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t nib = (out >> (4 * w)) & 15u;
          const uint32_t spread = (nib * 0x00204081u) & 0x01010101u;
          const uint32_t x = (qw[w] ^ rw[w]) | (spread << 2);
          sc[w] = __builtin_amdgcn_perm(tab_hi, tab_lo, x);
        }
      }
      // ---- the cells
      int kmax = INT32_MIN;
      uint32_t sb = 0, code0 = 0, code1 = 0;
      // Z-drop: this lane's first cell's diagonal minus the best cell's,
      // biased so that the distance is one unsigned difference per cell
      uint32_t zlane = 0;
      if (ZD) {
        const int bi = 0xffff - (int)(best_key >> 16), bj = 0xffff - (int)(best_key & 0xffffu);
        zlane = (uint32_t)(base + P + 2 * XC * gl - (bj - bi) + kZBias);
      }
      const int xin = P == 0 ? quad_shr1(E1[XC - 1], XNEG, qfirst)
                             : quad_shl1(F0[0], XNEG, qlast);
#pragma unroll
      for (int m = 0; m < XC; ++m) {
        const int ein = P == 0 ? (m == 0 ? xin : E1[m - 1]) : E0[m];
        const int fin = P == 0 ? F1[m] : (m == XC - 1 ? xin : F0[m + 1]);
        const int hp = P == 0 ? H0[m] : H1[m];
        const int s = (int)(int8_t)(sc[m >> 2] >> (8 * (m & 3)));
        const int h = max(max(hp + s, ein), fin);
        bool keep = h >= T;
        if (ZD) {
          // h + |d - d_best|, d = (first cell's diagonal) + 2m
          const uint32_t zc = (uint32_t)(kZBias - 2 * m);
          const int hz = (int)((max(zlane, zc) - min(zlane, zc)) + (uint32_t)h);
          keep = hz >= T && ((inr_rev >> (XC - 1 - m)) & 1u);
        }
        const int hm = keep ? h : XNEG;
        // X-drop: E and F may take h of a removed cell, below the threshold
        // either way
        const int t = h + go;
        const int en = (ZD && !keep) ? XNEG : max(ein, t);
        const int fn = (ZD && !keep) ? XNEG : max(fin, t);
        if (P == 0) {
          H0[m] = hm;
          E0[m] = en;
          F0[m] = fn;
        } else {
          H1[m] = hm;
          E1[m] = en;
          F1[m] = fn;
        }
        // X-drop: a removed cell never beats a kept one
        kmax = max(kmax, (ZD && !keep) ? INT32_MIN : ((h << 6) | m));
        // shift the survivor bit in: sb = 2 sb + keep (cell m ends at bit 15 - m)
        shift_in(sb, keep);
        if (TB) { // the cell's code, high bit first
          uint32_t &c = m < 8 ? code0 : code1;
          shift_in(c, t >= fin);
          shift_in(c, t >= ein);
          shift_in(c, ein < h);
          shift_in(c, hp + s < h);
        }
      }
      if (TB && active) {
        // only the 8-cell groups g0 .. g1 that hold candidates are stored
        // (a walk reads survivors only), after the antidiagonal before's
        const int g0 = plo >> 3, span = (phi >> 3) - g0;
        const int e0 = 2 * gl - g0; // stream slot of this lane's first group
        uint32_t *dst = reinterpret_cast<uint32_t *>(tb_meta + (tcur + 4 * e0));
        if ((unsigned)e0 <= (unsigned)span) dst[0] = code0;
        if ((unsigned)(e0 + 1) <= (unsigned)span) dst[1] = code1;
        tcur += 4 * (span + 1);
        // the antidiagonal's byte: g0 (bits 0-2), g1 (3-5) and the window
        // base's step from the antidiagonal before, (base - bprev) / 2 in
        // two's complement (bits 6-7).  Lane gl collects those of its 8 of
        // every 32 antidiagonals, and the side's four lanes store the 32
        // bytes at once (one whole memory sector: smaller stores cost as
        // much each)
        const uint32_t mbyte = ((uint32_t)plo >> 3) | ((uint32_t)phi & 0x38u) |
                               (((uint32_t)(base - bprev) << 5) & 0xc0u);
        bprev = base;
        if (((k >> 3) & 3) == gl) {
          mlo = __builtin_amdgcn_alignbit(mhi, mlo, 8);
          mhi = __builtin_amdgcn_alignbit(mbyte, mhi, 8);
        }
        if ((k & 31) == 31) {
          *reinterpret_cast<uint2 *>(tb_meta + (k - 31) + 8 * gl) = make_uint2(mlo, mhi);
          if ((k & 63) == 63) {
            // the next block starts on a 16-byte boundary; its entry holds
            // the base of its antidiagonal before (the table has room for
            // one entry past the last block)
            tcur = (tcur + 15) & ~15;
            const int nb = (M + N + 64) >> 6;
            if (qfirst)
              reinterpret_cast<int2 *>(tb_meta + xdl_tb_table(nb))[(k + 1) >> 6] =
                  make_int2((tcur - (int)xdl_tb_stream(nb)) >> 2, base);
          }
        }
      }
      sb &= inr_rev;
      // ---- the antidiagonal's outcome per side
      kmax = quad_max(kmax | (XC * gl));
      const int fl = sb ? XC * gl + (int)__builtin_clz(sb) - 16 : 64;
      const int ll = sb ? XC * gl + 15 - (int)__builtin_ctz(sb) : -1;
      const int f = quad_min(fl), l = quad_max(ll);
      const bool surv = active && f <= l;
      if (surv) {
        const int hs = kmax >> 6, ps = kmax & 63;
        const int d = base + 2 * ps + P;
        const int bi = (k - d) >> 1, bj = k - bi;
        const uint32_t key = ((uint32_t)(0xffff - bi) << 16) | (uint32_t)(0xffff - bj);
        const int cs = hs + kE;
        if (cs > best || (cs == best && key > best_key)) {
          best = cs;
          best_key = key;
        }
      }
      // ---- next antidiagonal: candidates in the other parity's positions,
      // clipped to the matrix
      const int kn = k + 1;
      const int kEn = kE + ge;
      int nlo = P == 0 ? f - 1 : f, nhi = P == 0 ? l : l + 1;
      const int dlo = max(-kn, kn - 2 * M), dhi = min(kn, 2 * N - kn);
      nlo = max(nlo, (dlo - base - (1 - P)) >> 1);
      nhi = min(nhi, (dhi - base - (1 - P)) >> 1);
      const bool cont = surv && kn <= M + N && nlo <= nhi;
      const bool wide = cont && nhi - nlo > 63;
      if (active && (!cont || wide)) {
        // the extension ends here (or leaves for a wider window)
        if (TB && (k & 31) != 31 && 8 * gl <= (k & 31)) { // the bytes of the last, partial 32
          const int sh = 8 * gl + 7 > (k & 31) ? 8 * (7 - (k & 7)) : 0; // a partial 8
          const unsigned long long m8 = ((unsigned long long)mhi << 32 | mlo) >> sh;
          *reinterpret_cast<uint2 *>(tb_meta + (k & ~31) + 8 * gl) =
              make_uint2((uint32_t)m8, (uint32_t)(m8 >> 32));
        }
        if (qfirst) {
          aln_result *res = a.res + pair;
          if (wide) {
            // score only: the wider one-side kernel; with traceback: the
            // one-side pass that writes codes in its own layout (the walk of
            // this layout skips the pair, marked in its task)
            res->flags |= ALN_F_WIDENED;
            const int slot = atomicAdd(a.widen_count, 1);
            const PairTask *src = a.tasks + task;
            PairTask *dst = a.widen + slot;
            dst->pair = src->pair;
            dst->rows = a.widen_rows;
            dst->tb_off = src->tb_off;
            dst->cigar_off = src->cigar_off;
            dst->cigar_cap = src->cigar_cap;
            dst->aux = 0;
            if (TB) const_cast<PairTask *>(a.tasks)[task].aux = 1;
          } else {
            res->score = best;
            res->q_end = 0xffff - (int)(best_key >> 16);
            res->r_end = 0xffff - (int)(best_key & 0xffffu);
            res->cells = cells;
          }
        }
        active = false;
        T = XBIG;
        plo = 1;
        phi = 0;
      }
      if (active) {
        // interior cells (i, j >= 1) of the next antidiagonal
        const int clo = max(nlo, (2 - kn - base - (1 - P)) >> 1);
        const int chi = min(nhi, (kn - 2 - base - (1 - P)) >> 1);
        cells += chi >= clo ? chi - clo + 1 : 0;
        k = kn;
        kE = kEn;
        T = best - X - kEn;
        plo = nlo;
        phi = nhi;
      }
      // ---- keep the candidates inside the window: slide by one cell.  The
      // live arrays are both H and the E / F just written.
      const bool sup = active && plo < 0, sdn = active && phi > 63;
      // The shifts are selects in place under a wave-uniform branch: a
      // branch on the side's own flag made the compiler copy every array at
      // its join on every antidiagonal (about 100 moves per lane).
      if (__ballot(sup)) { // base -= 2: every pos moves up one
#define XD_SLIDE_UP(A)                                                                      \
  {                                                                                         \
    const int c = quad_shr1(A[XC - 1], XNEG, qfirst);                                       \
    _Pragma("unroll") for (int m = XC - 1; m > 0; --m) A[m] = sup ? A[m - 1] : A[m];        \
    A[0] = sup ? c : A[0];                                                                  \
  }
        XD_SLIDE_UP(H0)
        XD_SLIDE_UP(H1)
        if (P == 0) {
          XD_SLIDE_UP(E0)
          XD_SLIDE_UP(F0)
        } else {
          XD_SLIDE_UP(E1)
          XD_SLIDE_UP(F1)
        }
#undef XD_SLIDE_UP
        if (sup) {
          base -= 2;
          plo += 1;
          phi += 1;
        }
      }
      if (__ballot(sdn)) { // base += 2: every pos moves down one
#define XD_SLIDE_DOWN(A)                                                                    \
  {                                                                                         \
    const int c = quad_shl1(A[0], XNEG, qlast);                                             \
    _Pragma("unroll") for (int m = 0; m < XC - 1; ++m) A[m] = sdn ? A[m + 1] : A[m];        \
    A[XC - 1] = sdn ? c : A[XC - 1];                                                        \
  }
        XD_SLIDE_DOWN(H0)
        XD_SLIDE_DOWN(H1)
        if (P == 0) {
          XD_SLIDE_DOWN(E0)
          XD_SLIDE_DOWN(F0)
        } else {
          XD_SLIDE_DOWN(E1)
          XD_SLIDE_DOWN(F1)
        }
#undef XD_SLIDE_DOWN
        if (sdn) {
          base += 2;
          plo -= 1;
          phi -= 1;
        }
      }
    };
    step(std::integral_constant<int, 1>{});
    step(std::integral_constant<int, 0>{});
  }
  // the last wavefront out resets the queue for the next launch
  if (lane == 0 && atomicAdd(a.queue + 1, 1) == (int)gridDim.x - 1) {
    a.queue[0] = 0;
    a.queue[1] = 0;
  }
}

size_t xdrop_lanes_lds_bytes() { return (size_t)kSides * 2 * kRingStride; }

hipError_t launch_xdrop_lanes(bool tb, const XdlArgs &a, int waves, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (a.zdrop && tb) return hipErrorInvalidValue; // Z-drop codes: the one-side pass
  if (tb)
    hipLaunchKernelGGL((xdrop_lanes_kernel<true, false>), dim3(waves), dim3(64), xdrop_lanes_lds_bytes(), s, a);
  else if (a.zdrop)
    hipLaunchKernelGGL((xdrop_lanes_kernel<false, true>), dim3(waves), dim3(64), xdrop_lanes_lds_bytes(), s, a);
  else
    hipLaunchKernelGGL((xdrop_lanes_kernel<false, false>), dim3(waves), dim3(64), xdrop_lanes_lds_bytes(), s, a);
  return hipGetLastError();
}

int xdrop_lanes_waves_per_cu(bool tb) {
  int nb = 0;
  const hipError_t e =
      tb ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, xdrop_lanes_kernel<true, false>, 64,
                                                        xdrop_lanes_lds_bytes())
         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, xdrop_lanes_kernel<false, false>, 64,
                                                        xdrop_lanes_lds_bytes());
  if (e != hipSuccess) return 4;
  return nb > 0 ? nb : 1;
}

} // namespace alnk
