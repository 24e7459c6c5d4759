// kernels_diag.hip -- banded and X-drop Gotoh H/E/F on gfx950 (int32),
// evaluated antidiagonal by antidiagonal in sheared coordinates.
//
// Coordinates (Sec. 6.2): antidiagonal k = i + j and diagonal d = j - i; the
// cells of antidiagonal k are those with d = k (mod 2).  Every dependency of
// cell (k, d) lies on earlier antidiagonals:
//   E(i,j) comes from (k-1, d-1),  F(i,j) from (k-1, d+1),  H(i-1,j-1) from
//   (k-2, d).
// So one register per diagonal holds that diagonal's latest H, the E value
// it passes right (EN = max(E + e, H + o + e)) and the F value it passes down
// (FN = max(F + e, H + o + e)); a step updates the diagonals of one parity
// in place.  One wavefront per pair; lane l owns RD consecutive diagonals of a
// 64*RD-wide window [dbase, dbase + 64*RD) that slides two diagonals at a time
// to follow the active region.  The only cross-lane traffic is one DPP
// (wave_shr or wave_shl) per step for the diagonal at a lane boundary.
//
// Domain per antidiagonal (Sec. 7): a contiguous range of diagonals
//   BAND  the static prune axis, centred on the rectangle's diagonal: row i
//         keeps floor(i*N/M) - w <= j <= floor(i*N/M) + w; on antidiagonal k
//         this is one interval of j, tracked incrementally;
//   XDROP the candidates [lo - 1, hi + 1] around the previous antidiagonal's
//         first and last surviving cells; a candidate is pruned (H = E = F =
//         minus infinity) when it scores more than X below the best score of
//         the earlier antidiagonals;
//   ZDROP the same, with the limit widened by the candidate's distance from
//         the best cell's diagonal (Sec. 9.3): pruned when it scores more
//         than Z + |d - d_best| below that best score.
// Cells outside the domain read as minus infinity.
//
// Traceback (BAND): per cell a 4-bit code -- bits 0-1 the term that gave H
// (0 diagonal, 1 E, 2 F, 3 LOCAL zero), bit 2 set when E(i,j+1) opens from
// H(i,j), bit 3 when F(i+1,j) opens from H(i,j) -- stored per lane and
// antidiagonal pair, with the window base of every antidiagonal.
#include <type_traits>

#include "internal.h"

namespace alnk {

constexpr int kSeqBuf = 2048; // circular LDS staging of sequence codes (per wave)
// Each ring is followed by a copy of its first kSeqMirror bytes, so a window
// of a few dwords read at any 4-aligned ring position never wraps.
constexpr int kSeqMirror = 32;
constexpr int kSeqStride = kSeqBuf + kSeqMirror;

__device__ __forceinline__ int dpp_wshr1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_wshl1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, false);
}

// Maximum over the wave by DPP: prefix maxima within each 16-lane row
// (row_shr 1, 2, 4, 8), then across rows (row_bcast 15 and 31); lane 63 ends
// with the maximum of all lanes.  Lanes without a source read INT32_MIN.
__device__ __forceinline__ int wave_max_i32(int v) {
  constexpr int lo = INT32_MIN;
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x111, 0xf, 0xf, false)); // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x112, 0xf, 0xf, false)); // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x114, 0xf, 0xf, false)); // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x118, 0xf, 0xf, false)); // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x142, 0xa, 0xf, false)); // row_bcast:15
  v = max(v, __builtin_amdgcn_update_dpp(lo, v, 0x143, 0xc, 0xf, false)); // row_bcast:31
  return __builtin_amdgcn_readlane(v, 63);
}

// end order: higher score, then smaller i, then smaller j
__device__ __forceinline__ bool better_end(int s, int i, int j, int bs, int bi, int bj) {
  if (s != bs) return s > bs;
  if (i != bi) return i < bi;
  return j < bj;
}

// h + |a - b| for a, b in [0, 2^31): one v_sad_u32.  Z-drop compares
// H + |d - d_best| with best - Z; diagonals are biased by kDiagBias so that
// both operands are non-negative.
constexpr int kDiagBias = 1 << 24;
__device__ __forceinline__ int add_absdiff(uint32_t a, uint32_t b, int h) {
  return (int)((max(a, b) - min(a, b)) + (uint32_t)h);
}

// Incremental tracker of the band's j-interval on antidiagonal k: the cells
// (k - j, j) inside the matrix with c(i) - w <= j <= c(i) + w, c(i) =
// floor(i*N/M).  As j grows, i = k - j shrinks and c(i) cannot grow, so both
// conditions cut the antidiagonal at one point each; as k grows both ends move
// right.  c(i) is stepped with a remainder (N = qn*M + rn), no division.
struct BandTrack {
  int M, N, w, qn, rn;
  int jl, cl, rl; // lower end j and c(k - j), (k - j)*N mod M
  int ju, cu, ru; // upper end
  __device__ void init(int M_, int N_, int w_) {
    M = M_; N = N_; w = w_;
    qn = N / M; rn = N % M;
    jl = cl = rl = 0;
    ju = cu = ru = 0;
  }
  __device__ void inc(int &c, int &r) const { r += rn; c += qn; if (r >= M) { r -= M; c += 1; } }
  __device__ void dec(int &c, int &r) const { r -= rn; c -= qn; if (r < 0) { r += M; c -= 1; } }
  // advance to antidiagonal k (called for k = 1, 2, ... in order)
  __device__ void step(int k) {
    inc(cl, rl); // i = k - jl grew by one
    inc(cu, ru);
    const int jmax = min(N, k);
    // lower end: smallest j >= k - M with j >= c(k - j) - w
    while (jl <= jmax && (jl < k - M || jl < cl - w)) { ++jl; dec(cl, rl); }
    // upper end: largest j <= min(N, k) with j <= c(k - j) + w
    for (;;) {
      if (ju + 1 > jmax) break;
      int c2 = cu, r2 = ru;
      dec(c2, r2);
      if (ju + 1 > c2 + w) break;
      ++ju; cu = c2; ru = r2;
    }
  }
};

template <int RD, int MODE, int PRUNE, bool TB, bool MM>
__device__ void diag_task(const DiagArgs &a, int task, int wave, int lane, uint8_t *smem,
                          const int8_t *smat) {
  static_assert(RD % 2 == 0, "a lane must hold whole diagonal pairs");
  constexpr bool DYN = PRUNE == ALN_XDROP || PRUNE == ALN_ZDROP; // dynamic pruning
  constexpr bool ZD = PRUNE == ALN_ZDROP;
  // Dynamic pruning with traceback: a full pass (results, widening queue)
  // that also writes every antidiagonal's codes, 2 bytes per lane and
  // antidiagonal pair.  When the region outgrows the window at antidiagonal
  // k, the codes of antidiagonals < k are complete; k goes to the task's aux
  // field, and the walk gives the pair a CIGAR only if its end cell (found
  // by the wider re-run) lies before it.
  constexpr bool TBX = TB && DYN;
  static_assert(!TBX || RD == 4, "dynamic-pruning codes are laid out for RD = 4");
  constexpr int W = 64 * RD;
  constexpr int HALF = RD / 2;
  const PairTask tk = a.tasks[task];
  const int p = tk.pair;
  aln_result *res = a.res + p;
  const int M = a.b.q_len[p];
  const int N = a.b.r_len[p];
  const uint8_t *Q = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];
  const int go = a.sc->gap_open, ge = a.sc->gap_extend, goe = go + ge;
  const int A = a.sc->alphabet;
  const int s_match = a.sc->match, s_mismatch = a.sc->mismatch; // MM: all that scores

  const int kstop = M + N; // last antidiagonal evaluated
  if (M == 0 || N == 0) {
    if (lane == 0) {
      if (MODE == ALN_GLOBAL) {
        res->score = (M + N == 0) ? 0 : go + (M + N) * ge;
        res->q_end = M;
        res->r_end = N;
      } else {
        res->score = 0;
        res->q_end = 0;
        res->r_end = 0;
      }
      res->cells = 0;
    }
    return;
  }

  uint8_t *qbuf = smem + (size_t)wave * 2 * kSeqStride;
  uint8_t *rbuf = qbuf + kSeqStride;
  int qtop = 0, rtop = 0; // codes [0, top) staged (modulo kSeqBuf)
  // Codes past the end read as the padding letter A.  The four loads are
  // unconditional (clamped index, len >= 1) so that they issue together and
  // the wave waits once per pass.
  auto stage = [&](const uint8_t *src, int len, uint8_t *buf, int &top, int need) {
    while (top < len && top <= need) {
      const int base = top + lane * 4;
      int raw[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) raw[b] = src[min(base + b, len - 1)];
      uint32_t w4 = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t c = (base + b < len) ? (uint32_t)min(raw[b], A) : (uint32_t)A;
        w4 |= c << (8 * b);
      }
      const int at = base & (kSeqBuf - 1);
      *reinterpret_cast<uint32_t *>(buf + at) = w4;
      if (at < kSeqMirror) *reinterpret_cast<uint32_t *>(buf + kSeqBuf + at) = w4;
      top += 256;
    }
  };
  // This lane's codes for one antidiagonal: the query codes q[i0-HALF ..
  // i0-1] and reference codes r[j0-1 .. j0+HALF-2] of its HALF cells, as
  // packed bytes (window byte b of the query belongs to cell HALF-1-b, byte
  // b of the reference to cell b).  One aligned read of NQW dwords and a
  // byte-align per register, instead of two byte reads per cell.
  constexpr int NWB = (HALF + 3) / 4;   // registers per window
  constexpr int NQW = (HALF + 3 + 3) / 4; // aligned dwords covering it
  static_assert(4 * NQW <= kSeqMirror, "window read beyond the ring's mirror");
  auto window = [&](const uint8_t *buf, int first, uint32_t (&w)[NWB]) {
    const uint32_t *src = reinterpret_cast<const uint32_t *>(buf + (first & (kSeqBuf - 4)));
    uint32_t d[NQW];
#pragma unroll
    for (int k = 0; k < NQW; ++k) d[k] = src[k];
#pragma unroll
    for (int k = 0; k < NWB; ++k)
      w[k] = __builtin_amdgcn_alignbyte(k + 1 < NQW ? d[k + 1] : 0u, d[k], (uint32_t)first & 3u);
  };

  // window state: element e = lane*RD + x  <->  diagonal dbase + e
  int H[RD], EN[RD], FN[RD];
#pragma unroll
  for (int x = 0; x < RD; ++x) { H[x] = NEG32; EN[x] = NEG32; FN[x] = NEG32; }
  int dbase = -(W / 2);
  const int e0 = lane * RD;

  // write values into the element holding diagonal d (wave-uniform d)
  auto set_elem = [&](int d, int h, int en, int fn) {
    const int e = d - dbase;
    if (e < 0 || e >= W) return;
    const int ln = e / RD, x = e - ln * RD;
#pragma unroll
    for (int y = 0; y < RD; ++y)
      if (y == x && lane == ln) { H[y] = h; EN[y] = en; FN[y] = fn; }
  };
  auto get_h = [&](int d) -> int {
    const int e = d - dbase;
    if (e < 0 || e >= W) return NEG32;
    const int ln = e / RD, x = e - ln * RD;
    int v = NEG32;
#pragma unroll
    for (int y = 0; y < RD; ++y)
      if (y == x) v = H[y];
    return __builtin_amdgcn_readlane(v, ln);
  };
  auto shift_right2 = [&]() { // dbase += 2
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int h0 = dpp_wshl1(NEG32, H[0]), en0 = dpp_wshl1(NEG32, EN[0]), fn0 = dpp_wshl1(NEG32, FN[0]);
#pragma unroll
      for (int x = 0; x < RD - 1; ++x) { H[x] = H[x + 1]; EN[x] = EN[x + 1]; FN[x] = FN[x + 1]; }
      H[RD - 1] = h0; EN[RD - 1] = en0; FN[RD - 1] = fn0;
    }
    dbase += 2;
  };
  auto shift_left2 = [&]() { // dbase -= 2
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int hl = dpp_wshr1(NEG32, H[RD - 1]), enl = dpp_wshr1(NEG32, EN[RD - 1]),
                fnl = dpp_wshr1(NEG32, FN[RD - 1]);
#pragma unroll
      for (int x = RD - 1; x > 0; --x) { H[x] = H[x - 1]; EN[x] = EN[x - 1]; FN[x] = FN[x - 1]; }
      H[0] = hl; EN[0] = enl; FN[0] = fnl;
    }
    dbase -= 2;
  };

  // k = 0: the cell (0,0)
  set_elem(0, 0, goe, goe);
  int best = 0, best_i = 0, best_j = 0; // running best through the last antidiagonal
  int lo = 0, hi = 0;                   // domain (XDROP: survivors) of the last antidiagonal
  long long cells = 0;
  BandTrack bt;
  const bool band_full = (PRUNE == ALN_BAND) && M == 0;
  if (PRUNE == ALN_BAND) bt.init(M, N, a.band_w);
  bool overflow = false;
  int kovf = 0; // antidiagonal at which the region outgrew the window

  // traceback output
  uint32_t *tbw = nullptr;
  int *dbh = nullptr;
  uint32_t code_lo = 0, code_hi = 0;
  int dbase_acc = 0;
  // codes of an even antidiagonal, and window bases of a block, are written
  // with the next odd antidiagonal / at the block's end; an extension that
  // stops early writes what is pending after the loop
  bool code_pend = false, dbase_pend = false;
  int kcode = 0, kdb = 0;
  if (TB) {
    const int nk = M + N + 1;
    dbh = reinterpret_cast<int *>(a.tb + tk.tb_off);
    tbw = reinterpret_cast<uint32_t *>(a.tb + tk.tb_off + (size_t)((nk + 63) / 64) * 64 * 4);
  }
  int gh = NEG32; // GLOBAL: H(M, N)

  const int KMAX = kstop;
  // One antidiagonal.  The window base and RD are even, so element x holds a
  // cell of antidiagonal k exactly when x = k (mod 2): with the parity a
  // compile-time constant every register index below is static.
  auto step = [&](auto par_tag, const int k) -> bool {
    constexpr int par = decltype(par_tag)::value;
    // ---- domain of antidiagonal k (in d), clipped to the matrix
    int dlo, dhi;
    const int mlo = max(-k, k - 2 * M), mhi = min(k, 2 * N - k);
    if (PRUNE == ALN_BAND) {
      if (band_full) {
        dlo = mlo; dhi = mhi;
      } else {
        bt.step(k);
        dlo = 2 * bt.jl - k;
        dhi = 2 * bt.ju - k;
      }
    } else {
      dlo = max(lo - 1, mlo);
      dhi = min(hi + 1, mhi);
      if (dlo > dhi) return false;
    }
    // ---- keep the domain inside the window
    if (dlo <= dhi) {
      if (dhi - dlo > W - 6) { overflow = true; kovf = k; return false; }
      while (dhi > dbase + W - 3) shift_right2();
      while (dlo < dbase + 2) shift_left2();
    }
    // ---- stage sequence codes for this step's window.  Under X-drop /
    // Z-drop every 8 antidiagonals: a domain end moves by at most one
    // diagonal per antidiagonal, so the window's largest i and j grow by at
    // most 8 in between, well inside the 64-code slack.  (A band of an
    // elongated rectangle can move faster and is checked every step.)
    if (!DYN || (par == 1 && ((k >> 1) & 3) == 0)) {
      const int needq = ((k - dbase) >> 1) + 64; // largest i on the window, plus slack
      const int needr = ((k + dbase + W) >> 1) + 64;
      stage(Q, M, qbuf, qtop, min(needq, M + 64));
      stage(Rs, N, rbuf, rtop, min(needr, N + 64));
    }
    if (TB) {
      if (lane == (k & 63)) dbase_acc = dbase;
      dbase_pend = true;
      kdb = k;
      if ((k & 63) == 63 || k == KMAX) {
        const int blk = k >> 6;
        if (lane <= (k & 63)) dbh[blk * 64 + lane] = dbase_acc;
        dbase_pend = false;
      }
    }
    // ---- neighbour values across the lane boundary
    int left_x = NEG32, right_x = NEG32;
    if constexpr (par == 0) left_x = dpp_wshr1(NEG32, EN[RD - 1]);
    else right_x = dpp_wshl1(NEG32, FN[0]);
    // ---- SIMD update of this parity's diagonals
    const int elo = dlo - dbase, ehi = dhi - dbase; // domain in element index
    const int thr = DYN ? max(best - a.xdrop, NEG32 / 2 + 1) : NEG32;
    int kkey = -1;                                  // (H << 11) | e of the best survivor
    const int d0 = dbase + e0 + par;
    // Z-drop: cell m of this lane lies on diagonal d0 + 2m, so its distance
    // to d_best is |(d0 + bias) - (d_best + bias - 2m)|
    const uint32_t zd_lane = (uint32_t)(d0 + kDiagBias);
    const int zd_best = best_j - best_i + kDiagBias;
    const int i0 = (k - d0) >> 1, j0 = (k + d0) >> 1;
    uint32_t cw = 0;
    uint32_t qw[NWB], rw[NWB];
    window(qbuf, i0 - HALF, qw);
    window(rbuf, j0 - 1, rw);
#pragma unroll
    for (int m = 0; m < HALF; ++m) {
      const int x = 2 * m + par;
      const int e = e0 + x;
      const int left = (x == 0) ? left_x : EN[(x + RD - 1) % RD];
      const int right = (x == RD - 1) ? right_x : FN[(x + 1) % RD];
      const int qb = HALF - 1 - m;
      const int qc = (int)((qw[qb >> 2] >> (8 * (qb & 3))) & 0xffu);
      const int rc = (int)((rw[m >> 2] >> (8 * (m & 3))) & 0xffu);
      const int sv = MM ? (qc == rc ? s_match : s_mismatch) : smat[qc * kMaxAlphabet + rc];
      const int hd = H[x] + sv;
      int h = max(max(hd, left), right);
      if (MODE == ALN_LOCAL) h = max(h, 0);
      bool keep = (unsigned)(e - elo) <= (unsigned)(ehi - elo) && elo <= ehi;
      if (PRUNE == ALN_XDROP) keep = keep && h >= thr;
      if (ZD) keep = keep && add_absdiff(zd_lane, (uint32_t)(zd_best - 2 * m), h) >= thr;
      // Outside a band only H needs the mask, with the open term formed
      // from the masked H: an E carries a real value only to the right of
      // the band and an F only to its left, and the band's edges move by
      // at most one diagonal per antidiagonal, so neither flows back in;
      // every other E and F stays at or below NEG + o + e.  X-drop prunes
      // inside its range, so there all three are masked.
      const int hk = keep ? h : NEG32;
      const int t = (PRUNE == ALN_BAND ? hk : h) + goe;
      const int en = max(left + ge, t);
      const int fn = max(right + ge, t);
      if (TB) {
        uint32_t hs = (h == hd) ? 0u : ((h == left) ? 1u : 2u);
        if (MODE == ALN_LOCAL && h == 0) hs = 3u;
        const uint32_t nib = hs | ((en == t) ? 4u : 0u) | ((fn == t) ? 8u : 0u);
        cw |= nib << (4 * m);
      }
      H[x] = hk;
      EN[x] = (PRUNE == ALN_BAND || keep) ? en : NEG32;
      FN[x] = (PRUNE == ALN_BAND || keep) ? fn : NEG32;
      if (MODE != ALN_GLOBAL) {
        const int key = keep ? ((max(h, -1) << 11) | e) : -1;
        kkey = max(kkey, key);
      }
    }
    // ---- boundary cells (i = 0 at d = k, j = 0 at d = -k) by formula
    if (k <= dhi + 1 || -k >= dlo - 1) {
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        const int d = side ? -k : k;
        if (d < dlo || d > dhi) continue;
        const int hb = (MODE == ALN_LOCAL) ? 0 : go + k * ge;
        bool kb = !(PRUNE == ALN_XDROP && hb < thr);
        if (ZD) kb = add_absdiff((uint32_t)(d + kDiagBias), (uint32_t)zd_best, hb) >= thr;
        set_elem(d, kb ? hb : NEG32, kb ? hb + goe : NEG32, kb ? hb + goe : NEG32);
        if (TB) {
          const int e = d - dbase, ln = e / RD, x = e - ln * RD;
          if (lane == ln) cw = (cw & ~(0xfu << (4 * (x >> 1)))) | (0xcu << (4 * (x >> 1)));
        }
        if (MODE != ALN_GLOBAL && kb) {
          const int key = (max(hb, -1) << 11) | (d - dbase);
          if (lane == 0) kkey = max(kkey, key);
        }
      }
    }
    if (TB) {
      if (par == 0) {
        code_lo = cw;
        code_pend = true;
        kcode = k;
      } else {
        code_hi = cw;
      }
      if (par == 1 || k == KMAX) {
        const uint32_t lo32 = code_lo | (HALF < 8 ? (code_hi << (4 * HALF)) : 0u);
        const uint32_t hi32 = (HALF < 8) ? (code_hi >> (32 - 4 * HALF)) : code_hi;
        if (TBX)
          reinterpret_cast<uint16_t *>(tbw)[(size_t)(k >> 1) * 64 + lane] = (uint16_t)lo32;
        else
          *reinterpret_cast<uint2 *>(tbw + ((size_t)(k >> 1) * 64 + lane) * 2) = make_uint2(lo32, hi32);
        code_lo = code_hi = 0;
        code_pend = false;
      }
    }
    // ---- cells evaluated on this antidiagonal (i >= 1 and j >= 1)
    {
      const int c_lo = max(dlo, 2 - k), c_hi = min(dhi, k - 2);
      if (c_lo <= c_hi) cells += (c_hi - c_lo) / 2 + 1;
    }
    // ---- best cell of this antidiagonal, next domain
    if (MODE != ALN_GLOBAL) {
      const int kb = wave_max_i32(kkey);
      if (kb >= 0 && (kb >> 11) >= best) { // the end order starts with the score
        const int sc = kb >> 11;
        const int d = dbase + (kb & 2047);
        const int bi = (k - d) >> 1, bj = (k + d) >> 1;
        if (better_end(sc, bi, bj, best, best_i, best_j)) { best = sc; best_i = bi; best_j = bj; }
      }
    }
    if (DYN) {
      // first and last surviving diagonals: each lane's first and last
      // surviving slot, then the first and last lane holding one
      int xf = RD, xl = -1;
#pragma unroll
      for (int m = 0; m < HALF; ++m) {
        const int x = 2 * m + par;
        const bool sv = H[x] > NEG32 / 2;
        xf = (sv && xf == RD) ? x : xf;
        xl = sv ? x : xl;
      }
      const unsigned long long bal = __ballot(xl >= 0);
      if (!bal) return false; // every candidate pruned: the extension stops
      const int lf = __ffsll((long long)bal) - 1;
      const int ll = 63 - __clzll((long long)bal);
      lo = dbase + lf * RD + __builtin_amdgcn_readlane(xf, lf);
      hi = dbase + ll * RD + __builtin_amdgcn_readlane(xl, ll);
    } else {
      lo = dlo;
      hi = dhi;
    }
    if (MODE == ALN_GLOBAL && k == KMAX) gh = get_h(N - M);
    return true;
  };
  for (int k = 1; k <= KMAX; k += 2) {
    if (!step(std::integral_constant<int, 1>{}, k)) break;
    if (k + 1 > KMAX || !step(std::integral_constant<int, 0>{}, k + 1)) break;
  }
  if (TB && code_pend) { // the last even antidiagonal, without its odd partner
    if (TBX)
      reinterpret_cast<uint16_t *>(tbw)[(size_t)(kcode >> 1) * 64 + lane] = (uint16_t)code_lo;
    else
      *reinterpret_cast<uint2 *>(tbw + ((size_t)(kcode >> 1) * 64 + lane) * 2) =
          make_uint2(code_lo, 0u);
  }
  if (TB && dbase_pend && lane <= (kdb & 63)) dbh[(kdb >> 6) * 64 + lane] = dbase_acc;

  if (lane == 0) {
    if (overflow) {
      if (TBX) const_cast<PairTask *>(a.tasks)[task].aux = kovf;
      res->flags |= ALN_F_WIDENED;
      if (a.widen_rows > 0) {
        const int slot = atomicAdd(a.widen_count, 1);
        PairTask t = tk;
        t.rows = a.widen_rows;
        a.widen[slot] = t;
      } else {
        res->status = ALN_R_TOO_WIDE; // region wider than the widest window
      }
    } else if (MODE == ALN_GLOBAL) {
      if (gh <= NEG32 / 2) {
        res->score = INT32_MIN;
        res->status = ALN_R_UNREACHABLE;
      } else {
        res->score = gh;
      }
      res->q_end = M;
      res->r_end = N;
    } else {
      res->score = best;
      res->q_end = best_i;
      res->r_end = best_j;
    }
    if (!overflow) res->cells = cells;
  }
}

template <int RD, int MODE, int PRUNE, bool TB, bool MM>
__global__ __launch_bounds__(256) void diag_kernel(DiagArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  // wave-uniform by construction; saying so keeps every per-pair and
  // per-antidiagonal quantity (task, lengths, domain, window base) scalar
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int8_t *smat = reinterpret_cast<int8_t *>(smem + 4 * 2 * kSeqStride);
  const int A = a.sc->alphabet;
  for (int k = threadIdx.x; k < kMaxAlphabet * kMaxAlphabet; k += blockDim.x) {
    const int qa = k / kMaxAlphabet, rc = k % kMaxAlphabet;
    smat[k] = (qa < A && rc < A) ? (int8_t)a.sc->mat[k] : (int8_t)-128;
  }
  __syncthreads();
  const int ntasks = a.dyn_ntasks ? min(*a.dyn_ntasks, a.ntasks) : a.ntasks;
  for (int task = blockIdx.x * 4 + wave; task < ntasks; task += gridDim.x * 4)
    diag_task<RD, MODE, PRUNE, TB, MM>(a, task, wave, lane, smem, smat);
}

// ------------------------------------------------------------------
// X-drop extension, four sides per wavefront.  Each 16-lane DPP row holds
// one side's window of 16*RD diagonals (with RD = 8 the same 128 diagonals a
// whole wavefront holds at two per lane), so a wavefront advances four sides
// per antidiagonal and every lane evaluates RD/2 cells per step.  The step is
// diag_task's for mode EXTEND with X-drop pruning; what that kernel keeps in
// scalar registers per pair (window base, domain, best cell, survivors) is
// here per row, in vector registers equal across the row's lanes.  Cross-lane
// moves use row_shr / row_shl; row reductions a DPP butterfly.
constexpr int kGroupSeq = 512; // LDS ring per sequence per side (bytes)

__device__ __forceinline__ int dpp_rshr1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x111, 0xf, 0xf, false); // row_shr:1
}
__device__ __forceinline__ int dpp_rshl1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x101, 0xf, 0xf, false); // row_shl:1
}
// maximum over the 16 lanes of each row, in every lane of the row
__device__ __forceinline__ int row_max_all(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xf, 0xf, false));  // quad_perm 1,0,3,2
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xf, 0xf, false));  // quad_perm 2,3,0,1
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x124, 0xf, 0xf, false)); // row_ror:4
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x128, 0xf, 0xf, false)); // row_ror:8
  return v;
}

template <int RD, bool MM, bool ZD>
__device__ void xdrop_group(const DiagArgs &a, int task4, int ntasks, int lane, uint8_t *smem,
                            const int8_t *smat) {
  static_assert(RD % 2 == 0, "a lane must hold whole diagonal pairs");
  constexpr int G = 16;
  constexpr int W = G * RD;
  constexpr int HALF = RD / 2;
  const int g = lane >> 4, gl = lane & 15;
  const int task = task4 + g;
  const bool has = task < ntasks;
  const int p = has ? a.tasks[task].pair : -1;
  const int M = has ? a.b.q_len[p] : 0;
  const int N = has ? a.b.r_len[p] : 0;
  const uint8_t *Q = has ? a.b.q + a.b.q_off[p] : nullptr;
  const uint8_t *Rs = has ? a.b.r + a.b.r_off[p] : nullptr;
  const int go = a.sc->gap_open, ge = a.sc->gap_extend, goe = go + ge;
  const int A = a.sc->alphabet;
  const int s_match = a.sc->match, s_mismatch = a.sc->mismatch;
  aln_result *res = has ? a.res + p : nullptr;

  bool alive = has && M > 0 && N > 0;
  if (has && !alive && gl == 0) {
    res->score = 0;
    res->q_end = 0;
    res->r_end = 0;
    res->cells = 0;
  }

  uint8_t *qbuf = smem + (size_t)g * 2 * kGroupSeq;
  uint8_t *rbuf = qbuf + kGroupSeq;
  int qtop = 0, rtop = 0;
  // each row's 16 lanes stage 64 codes per pass
  auto stage = [&](const uint8_t *src, int len, uint8_t *buf, int &top, int need) {
    while (alive && top < len && top <= need) {
      const int base = top + gl * 4;
      int raw[4]; // unconditional loads (clamped index), one wait per pass
#pragma unroll
      for (int b = 0; b < 4; ++b) raw[b] = src[min(base + b, len - 1)];
      uint32_t w4 = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t c = (base + b < len) ? (uint32_t)min(raw[b], A) : (uint32_t)A;
        w4 |= c << (8 * b);
      }
      *reinterpret_cast<uint32_t *>(buf + (base & (kGroupSeq - 1))) = w4;
      top += 64;
    }
  };

  int H[RD], EN[RD], FN[RD];
#pragma unroll
  for (int x = 0; x < RD; ++x) { H[x] = NEG32; EN[x] = NEG32; FN[x] = NEG32; }
  int dbase = -(W / 2);
  const int e0 = gl * RD;
  // write into the element of this row's window holding diagonal d
  auto set_elem = [&](bool on, int d, int h, int en, int fn) {
    const int e = d - dbase;
    const bool in = on && e >= 0 && e < W && gl == e / RD;
    const int x = e - gl * RD;
#pragma unroll
    for (int y = 0; y < RD; ++y)
      if (in && y == x) { H[y] = h; EN[y] = en; FN[y] = fn; }
  };
  // window moves by two diagonals in the rows where `on`
  auto shift_right2 = [&](bool on) { // dbase += 2
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int h0 = dpp_rshl1(NEG32, H[0]), en0 = dpp_rshl1(NEG32, EN[0]), fn0 = dpp_rshl1(NEG32, FN[0]);
      if (on) {
#pragma unroll
        for (int x = 0; x < RD - 1; ++x) { H[x] = H[x + 1]; EN[x] = EN[x + 1]; FN[x] = FN[x + 1]; }
        H[RD - 1] = h0; EN[RD - 1] = en0; FN[RD - 1] = fn0;
      }
    }
    if (on) dbase += 2;
  };
  auto shift_left2 = [&](bool on) { // dbase -= 2
#pragma unroll
    for (int pass = 0; pass < 2; ++pass) {
      const int hl = dpp_rshr1(NEG32, H[RD - 1]), enl = dpp_rshr1(NEG32, EN[RD - 1]),
                fnl = dpp_rshr1(NEG32, FN[RD - 1]);
      if (on) {
#pragma unroll
        for (int x = RD - 1; x > 0; --x) { H[x] = H[x - 1]; EN[x] = EN[x - 1]; FN[x] = FN[x - 1]; }
        H[0] = hl; EN[0] = enl; FN[0] = fnl;
      }
    }
    if (on) dbase -= 2;
  };

  set_elem(alive, 0, 0, goe, goe);
  int best = 0, best_i = 0, best_j = 0;
  int lo = 0, hi = 0;
  long long cells = 0;
  bool overflow = false;
  const int KMAX = M + N;
  int kmax_w = KMAX; // longest side of the wavefront
#pragma unroll
  for (int q = 0; q < 4; ++q) kmax_w = max(kmax_w, __builtin_amdgcn_readlane(KMAX, q * 16));

  auto step = [&](auto par_tag, const int k) {
    constexpr int par = decltype(par_tag)::value;
    if (k > KMAX) alive = false;
    // ---- domain: one step around the last antidiagonal's survivors
    const int mlo = max(-k, k - 2 * M), mhi = min(k, 2 * N - k);
    const int dlo = max(lo - 1, mlo), dhi = min(hi + 1, mhi);
    if (dlo > dhi) alive = false;
    if (alive && dhi - dlo > W - 6) {
      overflow = true;
      alive = false;
    }
    // ---- keep the domain inside the window (rows needing it shift together)
    while (__ballot(alive && dhi > dbase + W - 3)) shift_right2(alive && dhi > dbase + W - 3);
    while (__ballot(alive && dlo < dbase + 2)) shift_left2(alive && dlo < dbase + 2);
    // ---- stage codes
    {
      const int needq = ((k - dbase) >> 1) + 64;
      const int needr = ((k + dbase + W) >> 1) + 64;
      stage(Q, M, qbuf, qtop, min(needq, M + 64));
      stage(Rs, N, rbuf, rtop, min(needr, N + 64));
    }
    int left_x = NEG32, right_x = NEG32;
    if constexpr (par == 0) left_x = dpp_rshr1(NEG32, EN[RD - 1]);
    else right_x = dpp_rshl1(NEG32, FN[0]);
    const int elo = dlo - dbase, ehi = dhi - dbase;
    const int thr = max(best - a.xdrop, NEG32 / 2 + 1);
    int kkey = -1;
    const int d0 = dbase + e0 + par;
    const int i0 = (k - d0) >> 1, j0 = (k + d0) >> 1;
    const uint32_t zd_lane = (uint32_t)(d0 + kDiagBias); // Z-drop: as in diag_task
    const int zd_best = best_j - best_i + kDiagBias;
#pragma unroll
    for (int m = 0; m < HALF; ++m) {
      const int x = 2 * m + par;
      const int e = e0 + x;
      const int left = (x == 0) ? left_x : EN[(x + RD - 1) % RD];
      const int right = (x == RD - 1) ? right_x : FN[(x + 1) % RD];
      const int i = i0 - m, j = j0 + m;
      const int qc = qbuf[(i - 1) & (kGroupSeq - 1)];
      const int rc = rbuf[(j - 1) & (kGroupSeq - 1)];
      const int sv = MM ? (qc == rc ? s_match : s_mismatch) : smat[qc * kMaxAlphabet + rc];
      const int hd = H[x] + sv;
      const int h = max(max(hd, left), right);
      const int t = h + goe;
      const int en = max(left + ge, t);
      const int fn = max(right + ge, t);
      const int hz = ZD ? add_absdiff(zd_lane, (uint32_t)(zd_best - 2 * m), h) : h;
      const bool keep = alive && (unsigned)(e - elo) <= (unsigned)(ehi - elo) && hz >= thr;
      H[x] = keep ? h : NEG32;
      EN[x] = keep ? en : NEG32;
      FN[x] = keep ? fn : NEG32;
      const int key = keep ? ((max(h, -1) << 11) | e) : -1;
      kkey = max(kkey, key);
    }
    // ---- boundary cells (i = 0 at d = k, j = 0 at d = -k); past the first
    // antidiagonals no row's domain reaches them and the wave skips this
    const bool any_b = alive && ((k >= dlo && k <= dhi) || (-k >= dlo && -k <= dhi));
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (!__ballot(any_b)) break;
      const int d = side ? -k : k;
      const bool inb = alive && d >= dlo && d <= dhi;
      const int hb = go + k * ge;
      const bool kb =
          (ZD ? add_absdiff((uint32_t)(d + kDiagBias), (uint32_t)zd_best, hb) : hb) >= thr;
      set_elem(inb, d, kb ? hb : NEG32, kb ? hb + goe : NEG32, kb ? hb + goe : NEG32);
      if (inb && kb && gl == 0) kkey = max(kkey, (max(hb, -1) << 11) | (d - dbase));
    }
    // ---- cells evaluated on this antidiagonal (i >= 1 and j >= 1)
    if (alive) {
      const int c_lo = max(dlo, 2 - k), c_hi = min(dhi, k - 2);
      if (c_lo <= c_hi) cells += (c_hi - c_lo) / 2 + 1;
    }
    // ---- best cell of the antidiagonal (per row)
    const int kb = row_max_all(kkey);
    if (alive && kb >= 0) {
      const int sc = kb >> 11;
      const int d = dbase + (kb & 2047);
      const int bi = (k - d) >> 1, bj = (k + d) >> 1;
      if (better_end(sc, bi, bj, best, best_i, best_j)) { best = sc; best_i = bi; best_j = bj; }
    }
    // ---- first and last surviving diagonals of each row's window
    int slo = 1 << 30, shi = -(1 << 30);
#pragma unroll
    for (int m = 0; m < HALF; ++m) {
      const int x = 2 * m + par;
      const unsigned long long bal = __ballot(H[x] > NEG32 / 2);
      const uint32_t gb = (uint32_t)(bal >> (16 * g)) & 0xffffu;
      if (gb) {
        const int lf = __ffs((int)gb) - 1;
        const int ll = 31 - __clz((int)gb);
        slo = min(slo, dbase + lf * RD + x);
        shi = max(shi, dbase + ll * RD + x);
      }
    }
    if (slo > shi) alive = false; // every candidate pruned: the extension stops
    if (alive) {
      lo = slo;
      hi = shi;
    }
  };
  for (int k = 1; k <= kmax_w; k += 2) {
    if (!__ballot(alive)) break;
    step(std::integral_constant<int, 1>{}, k);
    if (k + 1 > kmax_w || !__ballot(alive)) break;
    step(std::integral_constant<int, 0>{}, k + 1);
  }

  if (has && gl == 0 && (M > 0 && N > 0)) {
    if (overflow) {
      res->flags |= ALN_F_WIDENED;
      if (a.widen_rows > 0) {
        const int slot = atomicAdd(a.widen_count, 1);
        PairTask t = a.tasks[task];
        t.rows = a.widen_rows;
        a.widen[slot] = t;
      } else {
        res->status = ALN_R_TOO_WIDE;
      }
    } else {
      res->score = best;
      res->q_end = best_i;
      res->r_end = best_j;
      res->cells = cells;
    }
  }
}

template <int RD, bool MM, bool ZD>
__global__ __launch_bounds__(256) void xdrop_group_kernel(DiagArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  int8_t *smat = reinterpret_cast<int8_t *>(smem + 4 * 4 * 2 * kGroupSeq);
  const int A = a.sc->alphabet;
  for (int k = threadIdx.x; k < kMaxAlphabet * kMaxAlphabet; k += blockDim.x) {
    const int qa = k / kMaxAlphabet, rc = k % kMaxAlphabet;
    smat[k] = (qa < A && rc < A) ? (int8_t)a.sc->mat[k] : (int8_t)-128;
  }
  __syncthreads();
  const int ntasks = a.ntasks;
  for (int t4 = (blockIdx.x * 4 + wave) * 4; t4 < ntasks; t4 += gridDim.x * 16)
    xdrop_group<RD, MM, ZD>(a, t4, ntasks, lane, smem + (size_t)wave * 4 * 2 * kGroupSeq, smat);
}

template <bool ZD>
static void launch_xdrop_group_t(const DiagArgs &a, hipStream_t s) {
  const size_t lds = (size_t)4 * 4 * 2 * kGroupSeq + kMaxAlphabet * kMaxAlphabet;
  const int blocks = (a.ntasks + 15) / 16;
  if (a.match_mismatch)
    hipLaunchKernelGGL((xdrop_group_kernel<8, true, ZD>), dim3(blocks), dim3(256), lds, s, a);
  else
    hipLaunchKernelGGL((xdrop_group_kernel<8, false, ZD>), dim3(blocks), dim3(256), lds, s, a);
}

hipError_t launch_xdrop_group(int prune, const DiagArgs &a, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (prune == ALN_ZDROP) launch_xdrop_group_t<true>(a, s);
  else if (prune == ALN_XDROP) launch_xdrop_group_t<false>(a, s);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int RD, int MODE, int PRUNE, bool TB>
static hipError_t launch_diag_t(const DiagArgs &a, hipStream_t s) {
  const bool mm = a.match_mismatch != 0;
  const size_t lds = (size_t)4 * 2 * kSeqStride + kMaxAlphabet * kMaxAlphabet;
  int blocks = (a.ntasks + 3) / 4;
  // a device-counted queue: the wide windows take few pairs (a capped grid,
  // grid-stride); the 256-diagonal window can take many, a wavefront each
  if (a.dyn_ntasks && RD >= 16) blocks = min(blocks, 2048);
  if (mm) hipLaunchKernelGGL((diag_kernel<RD, MODE, PRUNE, TB, true>), dim3(blocks), dim3(256), lds, s, a);
  else hipLaunchKernelGGL((diag_kernel<RD, MODE, PRUNE, TB, false>), dim3(blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int RD>
static hipError_t launch_diag_r(int mode, int prune, bool tb, const DiagArgs &a, hipStream_t s) {
  if (prune == ALN_XDROP || prune == ALN_ZDROP) {
    if constexpr (RD == 4) {
      if (tb) return prune == ALN_XDROP ? launch_diag_t<RD, ALN_EXTEND, ALN_XDROP, true>(a, s)
                                        : launch_diag_t<RD, ALN_EXTEND, ALN_ZDROP, true>(a, s);
    }
    if (tb) return hipErrorInvalidValue;
    return prune == ALN_XDROP ? launch_diag_t<RD, ALN_EXTEND, ALN_XDROP, false>(a, s)
                              : launch_diag_t<RD, ALN_EXTEND, ALN_ZDROP, false>(a, s);
  }
  switch (mode) {
  case ALN_GLOBAL:
    return tb ? launch_diag_t<RD, ALN_GLOBAL, ALN_BAND, true>(a, s)
              : launch_diag_t<RD, ALN_GLOBAL, ALN_BAND, false>(a, s);
  case ALN_LOCAL:
    return tb ? launch_diag_t<RD, ALN_LOCAL, ALN_BAND, true>(a, s)
              : launch_diag_t<RD, ALN_LOCAL, ALN_BAND, false>(a, s);
  default:
    return tb ? launch_diag_t<RD, ALN_EXTEND, ALN_BAND, true>(a, s)
              : launch_diag_t<RD, ALN_EXTEND, ALN_BAND, false>(a, s);
  }
}

hipError_t launch_diag(int rows, int mode, int prune, bool tb, const DiagArgs &a, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  switch (rows) {
  case 2: return launch_diag_r<2>(mode, prune, tb, a, s);
  case 4: return launch_diag_r<4>(mode, prune, tb, a, s);
  case 8: return launch_diag_r<8>(mode, prune, tb, a, s);
  case 10: return launch_diag_r<10>(mode, prune, tb, a, s);
  case 16: return launch_diag_r<16>(mode, prune, tb, a, s);
  case 32: return launch_diag_r<32>(mode, prune, tb, a, s);
  default: return hipErrorInvalidValue;
  }
}

} // namespace alnk
