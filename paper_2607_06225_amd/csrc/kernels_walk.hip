// kernels_walk.hip -- traceback walks on gfx950: stored 4-bit codes -> CIGAR.
//
// One wavefront per pair.  The path from the end cell back to the start is
// inherently serial, so every lane runs the same walk (all control flow is
// wave-uniform) and lane 0 writes the CIGAR words.  What the wave adds is
// memory parallelism: the codes are read in an order that never goes
// forward -- the antidiagonal k = i + j never grows along the path, and in the
// strip layout neither does the skewed step t = j - 1 + lane -- so the codes
// are consumed block by block.  The wave copies the current block from HBM
// into LDS with coalesced 16-byte loads while the next block's loads are
// already in flight in registers; each step is then one LDS read instead of a
// dependent HBM read.  The sequence bytes needed for '=' / 'X' come from
// 256-byte LDS windows that slide down as i and j fall.
//
// Preferences are the ones the codes encode (traceback of Sec. 2): in state H
// (LOCAL: stop on a zero) diagonal, then E, then F; in E and F the opening
// bit decides between returning to H and extending the gap.
#include "internal.h"

namespace alnk {

namespace {

constexpr int kBlockBytes = 16384;  // one LDS code block

// The walk's state is the same in every lane; reading it through
// readfirstlane keeps it in scalar registers and its branches scalar.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
constexpr int kPre = kBlockBytes / 16 / 64; // uint4 per lane per block
constexpr int kLook = 32;                   // cells a walk step looks ahead

__device__ __forceinline__ int ctz64(unsigned long long v) { return v ? __ffsll((long long)v) - 1 : 64; }

// Run-length CIGAR written backwards from the end of the pair's slot.  The
// state is wave-uniform; lane 0 stores.
struct WaveCigar {
  uint32_t *out;
  int w, cur, run;
  bool overflow;
  __device__ void flush(int lane) {
    if (cur < 0) return;
    if (w > 0) {
      --w;
      if (lane == 0) out[w] = ((uint32_t)run << 4) | (uint32_t)cur;
    } else {
      overflow = true;
    }
  }
  // The '=' / 'X' ops of a diagonal run of L <= kLook cells, first step of
  // the walk first (bit p of mm: cell p mismatches), all at once: the same
  // words and final state as emitting its sub-runs one by one.  Lane p that
  // starts a sub-run other than the last writes that sub-run's word; the
  // last sub-run stays pending (the next ops may extend it).
  __device__ void emit_diag_run(uint32_t mm, int L, int lane) {
    const uint32_t lmask = L >= 32 ? 0xffffffffu : ((1u << L) - 1u);
    const uint32_t starts = ((mm ^ (mm << 1)) | 1u) & lmask;
    const int K = __builtin_popcount(starts);
    const int last = 31 - __builtin_clz(starts);
    const int op0 = (mm & 1u) ? ALN_OP_X : ALN_OP_EQ;
    const bool merge = cur == op0;
    if (!merge) flush(lane); // the pending word ends here (nothing if none)
    if (lane < L && lane != last && ((starts >> lane) & 1u)) {
      const int r = __builtin_popcount(starts & ((1u << lane) - 1u)); // sub-runs before
      const uint64_t after = (uint64_t)starts >> (lane + 1);          // non-zero: not last
      int len = __builtin_ctzll(after) + 1;
      if (r == 0 && merge) len += run;
      const int idx = w - 1 - r;
      const int op = ((mm >> lane) & 1u) ? ALN_OP_X : ALN_OP_EQ;
      if (idx >= 0) out[idx] = ((uint32_t)len << 4) | (uint32_t)op;
    }
    if (w - (K - 1) < 0) {
      overflow = true;
      w = 0;
    } else {
      w -= K - 1;
    }
    const int len_last = L - last + ((K == 1 && merge) ? run : 0);
    cur = ((mm >> last) & 1u) ? ALN_OP_X : ALN_OP_EQ;
    run = len_last;
  }
};

} // namespace

// ------------------------------------------------------------ strip layout
// Codes of strip s: step t (0..N+62), lane l, rows r = 0..R-1 packed two per
// byte at ((s*T + t)*64 + l)*(R/2) + r/2.  Cell (i, j) lives in strip
// (i-1)/(64R), lane ((i-1) mod 64R)/R, row (i-1) mod R, step t = j-1+lane;
// bit 2 of its code says E(i, j) opened from H(i, j-1), bit 3 that F(i, j)
// opened from H(i-1, j).  A block is TBK consecutive steps of one strip
// (TBK*32R <= 16 KB).  Blocks are numbered s*NTB + b; the walk never moves to
// a higher number.
//
// Like the diagonal-layout walk below, it advances by whole runs: lanes
// m < 32 read the codes of the m-th cell ahead (H: (i-m, j-m), E: (i, j-m),
// F: (i-m, j)) from the two resident blocks (the walk's block and the one
// before in the same strip), and a run also ends at the first cell outside
// them; the next iteration makes that cell's block resident.
//
// BAND: the static-band strips (columns jlo_s .. jhi_s of strip s, step t =
// j - jlo_s + lane) with lane-major code windows: lane l of strip s keeps Lw
// steps from u_l (a multiple of 16 bytes) at ((s*64 + l)*Lw + t - u_l)*(R/2).  A
// block is TBK steps of every lane (8 KB, 128 bytes a lane), read from each
// lane's window (zeros outside it); the window starts of the walk's strip sit
// in LDS for the reads.
template <bool BAND>
__global__ __launch_bounds__(64) void walk_strip_wave(WalkArgs a) {
  // band strips: 8 KB blocks, so that a launch of thousands of walks stays
  // resident at once
  constexpr int BLK = BAND ? kBlockBytes / 2 : kBlockBytes;
  constexpr int PRE = BLK / 16 / 64;
  __shared__ __align__(16) uint4 codes4[2][BLK / 16];
  __shared__ uint8_t qwin[256], rwin[256];
  __shared__ int ustart[64];
  const int lane = threadIdx.x;
  const int task = blockIdx.x;
  if (task >= a.ntasks) return;
  const PairTask tk = a.tasks[task];
  const int p = tk.pair;
  aln_result *res = a.res + p;
  const int status = uni(res->status);
  const int i_end = uni(res->q_end), j_end = uni(res->r_end);
  __syncthreads();
  if (lane == 0) {
    res->cigar_off = tk.cigar_off;
    res->cigar_len = 0;
  }
  if (status != ALN_R_OK) return;
  const int M = uni(a.b.q_len[p]), N = uni(a.b.r_len[p]);
  const uint8_t *Qs = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];
  const uint8_t *tb = a.tb + tk.tb_off;
  const int R = uni(tk.rows), HB = R / 2;
  const int invR = (65536 + R - 1) / R; // v / R = (v * invR) >> 16 for 0 <= v < 64
  // log2 of the block's steps (a lane's share of a block: BLK / 64 bytes;
  // band strips: 128 bytes, 128 steps at 2 rows per lane, 64 at 4)
  const int LTB = BAND ? (R <= 2 ? 7 : 6) : (R <= 4 ? 7 : (R <= 8 ? 6 : (R <= 16 ? 5 : 4)));
  const int TBK = 1 << LTB;
  const int HS = 64 * R;
  const int bw = a.band_w;
  // steps of a strip (BAND: an upper bound over the strips)
  const int T = BAND ? (int)band_strip_cols(M, N, bw, R) + 63 : N + 63;
  const int NTB = (T + TBK - 1) >> LTB;
  const int Lw = BAND ? band_code_steps(M, N, bw, R) : 0;
  const bool local = a.mode == ALN_LOCAL;
  const uint8_t *codes0 = reinterpret_cast<const uint8_t *>(codes4[0]);
  // first column of strip s
  auto strip_jlo = [&](int s) { return BAND ? max(1, band_centre((int64_t)s * HS + 1, M, N) - bw) : 1; };
  int cjlo = 1; // first column of the resident strip

  // block cache: slots hold (cs, cb) and (cs, cb - 1); `pre` holds (cs, cb - 2)
  uint4 pre[PRE];
  int pre_key = -1, cs = -1, cb = -1;
  auto fetch = [&](int s, int b) {
    if (BAND) {
      // lane segment l = u / (PRE) of the block, 16-byte part u % PRE of it
      const uint8_t *sb = tb + (size_t)s * 64 * (size_t)Lw * HB;
#pragma unroll
      for (int m = 0; m < PRE; ++m) {
        const int u = lane + 64 * m;
        const int l = u / PRE;
        const int tp = b * TBK - ustart[l] + (u % PRE) * (16 / HB);
        pre[m] = (tp >= 0 && tp < Lw)
                     ? *reinterpret_cast<const uint4 *>(sb + ((size_t)l * Lw + tp) * HB)
                     : make_uint4(0u, 0u, 0u, 0u);
      }
    } else {
      const int steps = min(TBK, T - b * TBK);
      const uint4 *src = reinterpret_cast<const uint4 *>(
          tb + ((size_t)s * T + (size_t)b * TBK) * 64 * HB);
      const int n4 = steps * 64 * HB / 16;
#pragma unroll
      for (int m = 0; m < PRE; ++m) {
        const int u = lane + 64 * m;
        pre[m] = u < n4 ? src[u] : make_uint4(0u, 0u, 0u, 0u);
      }
    }
    pre_key = s * NTB + b;
  };
  // BAND: window starts of strip s's lanes, and its first column
  auto enter_strip = [&](int s) {
    if (!BAND) return;
    const int jlo = strip_jlo(s);
    const int itop = s * HS + lane * R + 1;
    const int u = itop <= M ? (max(1, band_centre(itop, M, N) - bw) - jlo + lane) & ~(band_code_align(R) - 1)
                            : (1 << 30);
    __syncthreads();
    ustart[lane] = u;
    __syncthreads();
    cjlo = jlo;
  };
  auto install = [&](int key) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < PRE; ++m) codes4[key & 1][lane + 64 * m] = pre[m];
    __syncthreads();
  };
  auto make_resident = [&](int s, int b) {
    if (s == cs && b == cb) return;
    const int key = s * NTB + b;
    if (s == cs && b == cb - 1) { // the common step: one block older
      if (b >= 1) {
        if (pre_key != key - 1) fetch(s, b - 1);
        install(key - 1);
      }
    } else { // first use, or a new strip
      if (s != cs) enter_strip(s);
      fetch(s, b);
      install(key);
      if (b >= 1) {
        fetch(s, b - 1);
        install(key - 1);
      }
    }
    cs = s;
    cb = b;
    if (b >= 2) fetch(s, b - 2);
  };
  // position of row i (while i >= 1): strip rs, lane rl, row rr; rjlo the
  // first column of strip rs
  int i = i_end, j = j_end;
  int rs = 0, rl = 0, rr = 0;
  if (i >= 1) {
    const int within = (i - 1) % (64 * R);
    rs = (i - 1) / (64 * R);
    rl = within / R;
    rr = within - rl * R;
  }
  int rjlo = uni(strip_jlo(rs));
  // position of row i - m, 0 <= m <= 32 (one strip boundary at most)
  auto rowpos = [&](int m, int &s2, int &l2, int &r2) {
    const int x = rr - m;
    s2 = rs;
    l2 = rl;
    r2 = x;
    if (x < 0) {
      const int dl = ((R - 1 - x) * invR) >> 16; // ceil(-x / R)
      l2 = rl - dl;
      r2 = x + dl * R;
      if (l2 < 0) {
        l2 += 64;
        s2 -= 1;
      }
    }
  };
  auto up_by = [&](int n) {
    int s2, l2, r2;
    rowpos(n, s2, l2, r2);
    if (BAND && s2 != rs) rjlo = uni(strip_jlo(s2));
    rs = s2;
    rl = l2;
    rr = r2;
    i -= n;
  };
  // code of the cell at (strip s2, lane l2, row r2, column jj), or -1 when
  // its block is not resident
  auto code_at = [&](int s2, int l2, int r2, int jj) -> int {
    const int t = jj - cjlo + l2;
    const int b = t >> LTB;
    if (s2 != cs || t < 0 || b > cb || b < cb - 1) return -1;
    const int slot = (s2 * NTB + b) & 1;
    if (BAND) {
      // steps outside the lane's window read as zero codes: only cells of
      // the band lie on a path, and a run or gap read ahead stops at the
      // path's next cell, which is inside the band
      // eight steps are R words, word r2 row r2's nibbles, the earlier
      // step higher; nibble: not-diagonal, not-E (LOCAL: zero with the
      // first clear), E opened, F opened
      const int st = t - (b << LTB);
      const uint32_t wd = reinterpret_cast<const uint32_t *>(codes0)[
          (slot * BLK + l2 * (TBK * HB)) / 4 + (st >> 3) * R + r2];
      const int nib = (int)(wd >> (28 - 4 * (st & 7))) & 15;
      const int b0 = nib >> 3, b1 = (nib >> 2) & 1;
      const int hs = b0 ? (b1 ? 2 : 1) : ((local && b1) ? 3 : 0);
      return hs | ((nib & 2) << 1) | ((nib & 1) << 3);
    }
    const int byte = slot * BLK + ((t - (b << LTB)) * 64 + l2) * HB + (r2 >> 1);
    return (codes0[byte] >> ((r2 & 1) * 4)) & 15;
  };
  int qbase = 1 << 30, rbase = 1 << 30;
  auto cover = [&](const uint8_t *src, int len, uint8_t *win, int &base, int lo, int hi) {
    if (lo >= base && hi < base + 256) return;
    base = max(0, hi - 255);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int pidx = base + lane * 4 + t;
      win[lane * 4 + t] = pidx < len ? src[pidx] : 0;
    }
    __syncthreads();
  };

  WaveCigar cw{a.cigar + tk.cigar_off, tk.cigar_cap, -1, 0, false};
  auto emit_n = [&](int op, int n) {
    if (n <= 0) return;
    if (op == cw.cur) {
      cw.run += n;
      return;
    }
    cw.flush(lane);
    cw.cur = op;
    cw.run = n;
  };
  int state = 0;
  bool bad = false;
  const unsigned long long look_mask = (1ull << kLook) - 1;
  for (int guard = 2 * (i_end + j_end) + 2; guard > 0 && !bad; --guard) {
    if ((state == 1 && j < 1) || (state == 2 && i < 1) || i < 0 || j < 0) {
      bad = true;
      break;
    }
    if (state == 0) {
      if (i == 0 && j == 0) break;
      if (local && (i == 0 || j == 0)) break;
      if (i == 0) { emit_n(ALN_OP_D, j); j = 0; continue; }
      if (j == 0) { emit_n(ALN_OP_I, i); i = 0; continue; }
      make_resident(rs, (j - rjlo + rl) >> LTB);
      cover(Qs, M, qwin, qbase, max(0, i - 1 - kLook), i - 1);
      cover(Rs, N, rwin, rbase, max(0, j - 1 - kLook), j - 1);
      // lanes m < kLook: the cell m steps up the diagonal
      const int m = lane;
      const int ii = i - m, jj = j - m;
      int c = -1;
      bool neq = false; // the cell's letters differ (read with its code: one LDS wait)
      if (m < kLook && ii >= 1 && jj >= 1) {
        int s2, l2, r2;
        rowpos(m, s2, l2, r2);
        c = code_at(s2, l2, r2, jj);
        neq = qwin[ii - 1 - qbase] != rwin[jj - 1 - rbase];
      }
      const bool diag = c >= 0 && (c & 3) == 0;
      const int L = min(ctz64(~__ballot(diag) & look_mask), kLook); // diagonal run length
      if (L == 0) {
        const int hs0 = uni(c) & 3; // lane 0: the walk's own cell, always resident
        if (local && hs0 == 3) break;
        state = hs0; // 1: E, 2: F
        continue;
      }
      // '=' / 'X' of the run, first step of the walk first
      cw.emit_diag_run((uint32_t)(__ballot(neq) & ((1ull << L) - 1)), L, lane);
      up_by(L);
      j -= L;
      // the cell that ended the run is read already: take its move now
      // instead of in a step of its own
      // (and a gap of one, whose opening bit is in that same code)
      const int cL = __builtin_amdgcn_readlane(c, L); // -1: not read (L = kLook, edge, block)
      if (cL >= 0) {
        const int hs = cL & 3;
        if (local && hs == 3) break;
        if (hs == 1 && (cL & 4)) { // E(i, j) opened from H(i, j-1)
          emit_n(ALN_OP_D, 1);
          j -= 1;
        } else if (hs == 2 && (cL & 8)) { // F(i, j) opened from H(i-1, j)
          emit_n(ALN_OP_I, 1);
          up_by(1);
        } else {
          state = hs; // 1: E, 2: F
        }
      }
    } else if (state == 1) {
      // D moves: E(i, j-m) opened from H(i, j-m-1) per the code of (i, j-m)
      make_resident(rs, (j - rjlo + rl) >> LTB);
      const int jj = j - lane;
      const bool in = lane < kLook && jj >= 1;
      const int c = in ? code_at(rs, rl, rr, jj) : -1;
      const unsigned long long om = __ballot(c >= 0 && (c & 4)) & look_mask;
      const unsigned long long stop = __ballot(in && c < 0) & look_mask; // not resident
      const int first_open = ctz64(om), first_stop = ctz64(stop);
      if (first_open < first_stop && first_open < kLook) {
        emit_n(ALN_OP_D, first_open + 1);
        j -= first_open + 1;
        state = 0;
      } else {
        const int n = min(first_stop, min(kLook, j));
        if (n <= 0 || (first_stop >= kLook && j < kLook)) { bad = true; break; } // must open by column 1
        emit_n(ALN_OP_D, n);
        j -= n;
      }
    } else {
      // I moves: F(i-m, j) opened from H(i-m-1, j) per the code of (i-m, j)
      make_resident(rs, (j - rjlo + rl) >> LTB);
      const int ii = i - lane;
      const bool in = lane < kLook && ii >= 1;
      int c = -1;
      if (in) {
        int s2, l2, r2;
        rowpos(lane, s2, l2, r2);
        c = code_at(s2, l2, r2, j);
      }
      const unsigned long long om = __ballot(c >= 0 && (c & 8)) & look_mask;
      const unsigned long long stop = __ballot(in && c < 0) & look_mask;
      const int first_open = ctz64(om), first_stop = ctz64(stop);
      if (first_open < first_stop && first_open < kLook) {
        emit_n(ALN_OP_I, first_open + 1);
        up_by(first_open + 1);
        state = 0;
      } else {
        const int n = min(first_stop, min(kLook, i));
        if (n <= 0 || (first_stop >= kLook && i < kLook)) { bad = true; break; } // must open by row 1
        emit_n(ALN_OP_I, n);
        up_by(n);
      }
    }
  }
  cw.flush(lane);
  if (lane == 0) {
    res->q_begin = i;
    res->r_begin = j;
    if (bad || cw.overflow) {
      res->status = ALN_R_CIGAR_CAP;
    } else {
      res->cigar_len = tk.cigar_cap - cw.w;
      res->cigar_off = tk.cigar_off + cw.w;
    }
  }
}

// ---------------------------------------------------------- diagonal layout
// Per antidiagonal k the window base dbase(k) (ints, rounded up to 64), then
// per antidiagonal pair k/2 and lane S bytes (S = diag_stride: 8 for bands,
// 2 for X-drop / Z-drop regions): the RD/2 cells of the even antidiagonal in
// the low nibbles, then those of the odd one.  Cell (i, j): element e = (j -
// i) - dbase(k), lane e / RD, slot e mod RD.  A block is 64 antidiagonals:
// 2048*S bytes of codes plus 64 window bases.
//
// S = 1 is the layout of the sixteen-sides X-drop kernel (xdl_tb_table /
// xdl_tb_stream): per antidiagonal the code dwords of the 8-cell groups g0 ..
// g1 of its 64-cell window that hold candidates, packed; a byte per
// antidiagonal (g0, g1, the window base's step) and per 64 antidiagonals the
// block's stream offset and the window base before it.  Cell (i, j) of antidiagonal
// k sits at pos = ((j - i) - dbase(k) - (k & 1)) / 2, in group g = pos >> 3
// (stored if g0 <= g <= g1) at nibble 7 - (pos & 7), the high nibble of a
// byte for even pos.  A block's offsets and bases come from prefix sums of
// the bytes when it is fetched.  Its low two bits say "not the diagonal" and
// "not E" (the walk maps them to its diagonal / E / F choice); bits 2 and 3
// are the opening bits as in the other layouts.  A pair that overflowed that
// kernel's window is marked in its task (aux) and walked in the S = 2 layout
// by the pass that recomputed it.
//
// The walk advances by whole runs.  The two most recent blocks (the one
// holding the walk's antidiagonal and the one before) stay in two LDS slots,
// and the next older block is in flight in registers.  Every lane m < 32
// reads, in parallel, the code of the m-th cell ahead along the current move:
//   state H  cells (i-m, j-m): the diagonal run ends at the first cell whose
//            code does not choose the diagonal (one ballot); the run's '='
//            and 'X' come from a second ballot of sequence comparisons;
//   state E  cells (i, j-1-m): the gap ends at the first one whose code says
//            E(i, j-m) opened there;
//   state F  cells (i-1-m, j): likewise for the vertical gap.
// All those cells lie within 63 antidiagonals of the current one, so within
// the two resident blocks.

template <int S>
__global__ __launch_bounds__(64) void walk_diag_wave(WalkArgs a) {
  // two block slots of 2048*S bytes each (dynamic LDS, sized by the stride,
  // so that narrow layouts let more walks share a CU)
  extern __shared__ __align__(16) uint4 codes_dyn[];
  // per antidiagonal of a resident block: its window base; S = 1: ((in-block
  // dword of group 0 + 8) << 6 | g1 << 3 | g0) << 8 | the base minus the
  // block's (hb), which stays in a register (LDS per walk bounds the walks
  // per CU)
  __shared__ int dbl[2][64];
  __shared__ uint8_t qwin[256], rwin[256];
  const int lane = threadIdx.x;
  const int task = blockIdx.x;
  const int ntasks = a.dyn_ntasks ? min(*a.dyn_ntasks, a.ntasks) : a.ntasks;
  if (task >= ntasks) return;
  const PairTask tk = a.tasks[task];
  if (S == 1 && tk.aux != 0) return; // recomputed and walked in the S = 2 layout
  const int p = tk.pair;
  aln_result *res = a.res + p;
  const int status = uni(res->status);
  const int i_end = uni(res->q_end), j_end = uni(res->r_end);
  __syncthreads();
  if (lane == 0) {
    res->cigar_off = tk.cigar_off;
    res->cigar_len = 0;
  }
  if (status != ALN_R_OK) return;
  // X-drop / Z-drop: codes stop before the antidiagonal at which the region
  // outgrew the traceback window (aux, 0: never)
  if (S == 2 && tk.aux > 0 && i_end + j_end >= tk.aux) {
    if (lane == 0) res->status = ALN_R_CIGAR_CAP;
    return;
  }
  const int M = uni(a.b.q_len[p]), N = uni(a.b.r_len[p]);
  const uint8_t *Qs = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];
  const int RD = uni(tk.rows);
  // S: code bytes per lane and antidiagonal pair (S = 1: 32 bytes per
  // antidiagonal)
  constexpr int blk_bytes = 2048 * S;    // one block: 64 antidiagonals
  constexpr int n4 = 2 * S;              // uint4 per lane per block
  static_assert(n4 <= kPre, "block larger than the prefetch registers");
  const int inv = (65536 + RD - 1) / RD; // e / RD = (e * inv) >> 16 for 0 <= e < 64*RD
  const int nk = M + N + 1;
  const int nks = (M + N) / 2 + 1; // antidiagonal pairs stored
  const uint8_t *tbp = a.tb + tk.tb_off;
  const int *dbh = reinterpret_cast<const int *>(tbp);
  const int nblk = (nk + 63) / 64;
  const uint4 *cod = reinterpret_cast<const uint4 *>(tbp + (S == 1 ? (size_t)xdl_tb_stream(nblk)
                                                                   : (size_t)nblk * 64 * 4));
  const int2 *xtab = reinterpret_cast<const int2 *>(tbp + xdl_tb_table(nblk));
  const bool local = a.mode == ALN_LOCAL;

  // block cache: slots hold blocks cur and cur - 1; `pre` holds cur - 2
  uint4 pre[kPre];
  int pre_aux = 0, pre_blk = -1, cur = -1;
  uint32_t pre_meta = 0;                // S = 1: the fetched block's byte of antidiagonal 64b + lane
  int2 head_next = make_int2(0, 0);     // S = 1: table entry of block head_blk, loaded ahead
  int head_blk = -1;
  int hb0 = 0, hb1 = 0;                 // S = 1: window base before the block in slot 0 / 1
  auto fetch = [&](int b) {
    // uint4 of the block that hold stored antidiagonals (S = 1: at most 8
    // dwords per antidiagonal, from the block's 16-byte aligned offset,
    // whose table entry was loaded with the block before when the walk
    // goes one block back; nothing fetched is waited for here)
    const int have = S == 1 ? min(64, nk - b * 64) * 2 : min(32, nks - b * 32) * 4 * S;
    int2 head = make_int2(0, 0);
    if (S == 1) head = head_blk == b ? head_next : xtab[b];
    const uint4 *src = S == 1 ? cod + (head.x >> 2) : cod + (size_t)b * 128 * S; // 2048 S bytes per block
#pragma unroll
    for (int m = 0; m < kPre; ++m) {
      const int u = lane + 64 * m;
      if (m < n4) pre[m] = u < have ? src[u] : make_uint4(0u, 0u, 0u, 0u);
    }
    if (S == 1) {
      pre_meta = tbp[b * 64 + lane];
      pre_aux = head.y;
      if (b >= 1) {
        head_next = xtab[b - 1];
        head_blk = b - 1;
      }
    } else {
      pre_aux = dbh[b * 64 + lane];
    }
    pre_blk = b;
  };
  auto install = [&](int b) { // put block b (already fetched) into its slot
    int base_l = pre_aux;
    if (S == 1) {
      // lane = antidiagonal 64b + lane: its groups' first dword in the block
      // and its window base, from prefix sums of group counts and base steps
      // (the block's entry holds the base of antidiagonal 64b - 1)
      const int g0 = pre_meta & 7, g1 = (pre_meta >> 3) & 7;
      const int cnt = g1 + 1 - g0;
      const int st = (int)(pre_meta << 24) >> 30; // the base's step / 2: 0, 1 or -1
      // both sums in one (counts stay below 2^16), an inclusive DPP scan:
      // within rows of 16 lanes, then across rows
      int v = cnt + st * 65536;
      v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false); // row_shr:1
      v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false); // row_shr:2
      v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false); // row_shr:4
      v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false); // row_shr:8
      v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false); // row_bcast:15
      v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false); // row_bcast:31
      const int csum = v & 0xffff;
      base_l = ((((csum - cnt - g0 + 8) << 6) | (g1 << 3) | g0) << 8) | (((v - csum) >> 15) & 0xff);
      if (b & 1) hb1 = pre_aux;
      else hb0 = pre_aux;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kPre; ++m)
      if (m < n4) codes_dyn[(b & 1) * 128 * S + lane + 64 * m] = pre[m];
    dbl[b & 1][lane] = base_l;
    __syncthreads();
  };
  auto make_resident = [&](int b) { // blocks b and b - 1 resident, b - 2 in flight
    if (b == cur) return;
    if (b == cur - 1 && b >= 1) { // the common step: one block older
      if (pre_blk != b - 1) fetch(b - 1);
      install(b - 1);
    } else { // first use, or a jump
      fetch(b);
      install(b);
      if (b >= 1) {
        fetch(b - 1);
        install(b - 1);
      }
    }
    cur = b;
    if (b >= 2) fetch(b - 2);
  };
  const uint8_t *codes0 = reinterpret_cast<const uint8_t *>(codes_dyn);
  // code of (ii, jj), any lane; the cell must lie in a resident block
  auto code_at = [&](int ii, int jj, bool &bad_lane) -> int {
    const int kk = ii + jj;
    const int slot = (kk >> 6) & 1;
    if (S == 1) {
      const int x = dbl[slot][kk & 63], go = x >> 8;
      const int pos = ((jj - ii) - (slot ? hb1 : hb0) - (int)(int8_t)(x & 0xff) - (kk & 1)) >> 1;
      const int g = pos >> 3;
      // outside the window, or a group without candidates: the (in-slot)
      // byte read is not used
      const bool out = (unsigned)pos >= 64u || g < (go & 7) || g > ((go >> 3) & 7);
      bad_lane |= out;
      const int dw = ((go >> 6) - 8 + g) & 511;
      const int byte = slot * blk_bytes + dw * 4 + ((7 - (pos & 7)) >> 1);
      const int c = out ? 0 : (codes0[byte] >> (((7 - (pos & 7)) & 1) * 4)) & 15;
      // not-diagonal, not-E -> 0 diagonal, 1 E, 2 F
      return (c & 12) | ((c & 1) + (c & (c >> 1) & 1));
    }
    const int e = (jj - ii) - dbl[slot][kk & 63];
    if ((unsigned)e >= (unsigned)(64 * RD)) {
      bad_lane = true;
      return 0;
    }
    const int ln = (e * inv) >> 16;
    const int x = e - ln * RD;
    const int pos = (kk & 1) * (RD >> 1) + (x >> 1);
    const int byte = slot * blk_bytes + ((kk >> 1) & 31) * 64 * S + ln * S + (pos >> 1);
    return (codes0[byte] >> ((pos & 1) * 4)) & 15;
  };
  // sequence windows covering the next kLook + 1 positions below i and j
  int qbase = 1 << 30, rbase = 1 << 30;
  auto cover = [&](const uint8_t *src, int len, uint8_t *win, int &base, int lo, int hi) {
    if (lo >= base && hi < base + 256) return;
    base = max(0, hi - 255);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int pidx = base + lane * 4 + t;
      win[lane * 4 + t] = pidx < len ? src[pidx] : 0;
    }
    __syncthreads();
  };

  int i = i_end, j = j_end;
  WaveCigar cw{a.cigar + tk.cigar_off, tk.cigar_cap, -1, 0, false};
  auto emit_n = [&](int op, int n) {
    if (n <= 0) return;
    if (op == cw.cur) {
      cw.run += n;
      return;
    }
    cw.flush(lane);
    cw.cur = op;
    cw.run = n;
  };
  int state = 0;
  bool bad = false;
  const unsigned long long look_mask = (1ull << kLook) - 1;
  for (int guard = 2 * (i_end + j_end) + 2; guard > 0 && !bad; --guard) {
    if ((state == 1 && j < 1) || (state == 2 && i < 1) || i < 0 || j < 0) {
      bad = true;
      break;
    }
    if (state == 0) {
      if (i == 0 && j == 0) break;
      if (local && (i == 0 || j == 0)) break;
      if (i == 0) { emit_n(ALN_OP_D, j); j = 0; continue; }
      if (j == 0) { emit_n(ALN_OP_I, i); i = 0; continue; }
      make_resident((i + j) >> 6);
      cover(Qs, M, qwin, qbase, max(0, i - 1 - kLook), i - 1);
      cover(Rs, N, rwin, rbase, max(0, j - 1 - kLook), j - 1);
      // lanes m < kLook: the cell m steps up the diagonal
      const int ii = i - lane, jj = j - lane;
      const bool valid = lane < kLook && ii >= 1 && jj >= 1;
      bool bl = false;
      const int c = valid ? code_at(ii, jj, bl) : 0;
      // the cell's letters differ (read with its code: one LDS wait)
      const bool neq = valid && qwin[ii - 1 - qbase] != rwin[jj - 1 - rbase];
      const int hs = c & 3;
      const bool diag = valid && !bl && hs == 0;
      const unsigned long long badm = __ballot(valid && bl);
      if (badm & 1ull) { bad = true; break; }
      const int L = min(ctz64(~__ballot(diag) & look_mask), kLook); // diagonal run length
      if (L == 0) {
        const int hs0 = uni(hs);
        if (local && hs0 == 3) break;
        state = hs0; // 1: E, 2: F
        continue;
      }
      if (badm & ((1ull << L) - 1)) { bad = true; break; }
      // '=' / 'X' of the run, first step of the walk first
      cw.emit_diag_run((uint32_t)(__ballot(neq) & ((1ull << L) - 1)), L, lane);
      i -= L;
      j -= L;
      // the cell that ended the run is read already: take its move now
      // instead of in a step of its own
      const int hL = __builtin_amdgcn_readlane(valid && !bl ? hs : -1, L); // -1: not read
      if (hL >= 0) {
        if (local && hL == 3) break;
        // a gap of one cell: E(i, j) opened from H(i, j-1) is bit 2 of
        // code(i, j-1), F(i, j) from H(i-1, j) bit 3 of code(i-1, j).  That
        // cell's antidiagonal may lie two blocks back, which is not resident.
        bool bl1 = ((i + j - 1) >> 6) < cur - 1;
        const int c1 = bl1 ? 0 : (hL == 1 ? code_at(i, j - 1, bl1) : code_at(i - 1, j, bl1));
        if (!bl1 && (c1 & (hL == 1 ? 4 : 8))) {
          if (hL == 1) {
            emit_n(ALN_OP_D, 1);
            j -= 1;
          } else {
            emit_n(ALN_OP_I, 1);
            i -= 1;
          }
        } else {
          state = hL; // 1: E, 2: F
        }
      }
    } else if (state == 1) {
      // D moves from (i, j): E(i, j-m) opened from H(i, j-1-m) per code(i, j-1-m)
      make_resident((i + j) >> 6);
      const int jj = j - 1 - lane;
      const bool valid = lane < kLook && jj >= 0;
      bool bl = false;
      const int c = valid ? code_at(i, jj, bl) : 0;
      const bool open = valid && !bl && (c & 4);
      if (__ballot(valid && bl)) {
        // a bad code ahead: only a concern if the gap reaches it
        const int first_bad = ctz64(__ballot(valid && bl));
        const int first_open = ctz64(__ballot(open));
        if (first_bad <= first_open) { bad = true; break; }
      }
      const unsigned long long om = __ballot(open) & look_mask;
      if (om) {
        const int n = ctz64(om) + 1;
        emit_n(ALN_OP_D, n);
        j -= n;
        state = 0;
      } else {
        const int n = min(kLook, j);
        if (n < kLook) { bad = true; break; } // the gap must open by column 0
        emit_n(ALN_OP_D, n);
        j -= n;
      }
    } else {
      make_resident((i + j) >> 6);
      const int ii = i - 1 - lane;
      const bool valid = lane < kLook && ii >= 0;
      bool bl = false;
      const int c = valid ? code_at(ii, j, bl) : 0;
      const bool open = valid && !bl && (c & 8);
      if (__ballot(valid && bl)) {
        const int first_bad = ctz64(__ballot(valid && bl));
        const int first_open = ctz64(__ballot(open));
        if (first_bad <= first_open) { bad = true; break; }
      }
      const unsigned long long om = __ballot(open) & look_mask;
      if (om) {
        const int n = ctz64(om) + 1;
        emit_n(ALN_OP_I, n);
        i -= n;
        state = 0;
      } else {
        const int n = min(kLook, i);
        if (n < kLook) { bad = true; break; }
        emit_n(ALN_OP_I, n);
        i -= n;
      }
    }
  }
  cw.flush(lane);
  if (lane == 0) {
    res->q_begin = i;
    res->r_begin = j;
    if (bad || cw.overflow) {
      res->status = ALN_R_CIGAR_CAP;
    } else {
      res->cigar_len = tk.cigar_cap - cw.w;
      res->cigar_off = tk.cigar_off + cw.w;
    }
  }
}

hipError_t launch_walk(int layout, const WalkArgs &a, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (layout == 2) hipLaunchKernelGGL(walk_strip_wave<true>, dim3(a.ntasks), dim3(64), 0, s, a);
  else hipLaunchKernelGGL(walk_strip_wave<false>, dim3(a.ntasks), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_walk_diag(const WalkArgs &a, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (a.diag_stride == 8)
    hipLaunchKernelGGL(walk_diag_wave<8>, dim3(a.ntasks), dim3(64), (size_t)2 * 2048 * 8, s, a);
  else if (a.diag_stride == 2)
    hipLaunchKernelGGL(walk_diag_wave<2>, dim3(a.ntasks), dim3(64), (size_t)2 * 2048 * 2, s, a);
  else if (a.diag_stride == 1)
    hipLaunchKernelGGL(walk_diag_wave<1>, dim3(a.ntasks), dim3(64), (size_t)2 * 2048 * 1, s, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

} // namespace alnk
