// kernels_strip.hip -- full-matrix Gotoh H/E/F on gfx950 (int32 scores).
//
// Schedule.  One wavefront per pair.  Lane l owns R consecutive query rows
// (a 64*R-row "strip") and sweeps the reference columns; lane l runs one
// column behind lane l-1, so at step t lane l evaluates column j = t - l + 1:
// the wave advances an antidiagonal wavefront of R-row tiles (the paper's
// antidiagonal schedule, Sec. 6.2, with cells of one antidiagonal of tiles in
// flight together).  Within a tile the R cells of a column are evaluated top
// to bottom.  The bottom row's (H+o+e, F) and the reference code move to the
// next lane with one DPP wave_shr:1 each; lane 0 is fed the strip's top
// boundary (row 0 by formula, else the previous strip's bottom row kept in
// LDS).  Queries longer than 64*R run as successive strips.
//
// Recurrence (Sec. 3, Gotoh form; o = gap open, e = gap extend):
//   F(i,j) = max(F(i-1,j) + e, H(i-1,j) + o + e)
//   H(i,j) = max(H(i-1,j-1) + s(q_i, r_j), E(i,j), F(i,j))      [LOCAL: ,0]
//   E(i,j+1) = max(E(i,j) + e, H(i,j) + o + e)      (computed one column early)
//
// Optional traceback: a 4-bit code per cell (bits 0-1: which term gave H --
// 0 diagonal, 1 E, 2 F, 3 LOCAL zero; bit 2: E(i,j) opened from H(i,j-1);
// bit 3: F(i,j) opened from H(i-1,j)), R codes per lane per step stored
// contiguously so that a step of the wave writes one coalesced block.
#include <type_traits>

#include "internal.h"

namespace alnk {

__device__ __forceinline__ int dpp_wave_shr1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Strip pipeline (G > 1 wavefronts per pair).  Wave w of the workgroup runs
// strips w, w + G, w + 2G, ...; strip s reads strip s-1's bottom row (H, F per
// column) from LDS buffer (s-1) mod G as soon as it is written, so G strips
// advance together, each about 128 columns behind the one above.  Two LDS
// counters per buffer carry stamps s*(N+1) + column: `prog` (columns of
// strip s written, published every 64 steps) and `cons` (columns of strip s
// loaded by strip s+1).  A strip waits only for the strip above it (prog)
// and, before reusing a buffer, for the previous generation to have been
// read in full (cons); both point to earlier strips, so every wait ends.
// The spin bound only turns a broken invariant into ALN_R_INTERNAL instead
// of a hung workgroup.
constexpr int kSpinLimit = 1 << 22;

__device__ __forceinline__ bool lds_wait_geq(int *ctr, int need) {
  for (int k = 0; k < kSpinLimit; ++k) {
    const int v = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP));
    if (v >= need) return true;
    __builtin_amdgcn_s_sleep(1);
  }
  return false;
}
__device__ __forceinline__ void lds_publish(int *ctr, int v) {
  __hip_atomic_store(ctr, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// A chunk's feeds are loaded once and read over 64 steps.  Read directly,
// the loaded register makes every step wait for all memory operations in
// flight (the traceback stores included); one ALU copy at the chunk start
// (xor with a run-time zero the compiler cannot fold) takes that wait once.
__device__ __forceinline__ int settle(int v, int zero) { return v ^ zero; }

// end order: higher score, then smaller i, then smaller j
__device__ __forceinline__ bool strip_better(int s, int i, int j, int bs, int bi, int bj) {
  if (s != bs) return s > bs;
  if (i != bi) return i < bi;
  return j < bj;
}

template <int R, int MODE, bool TB, bool SMALLA, int G>
__device__ void strip_task(const StripArgs &a, int task, int wave, int lane, uint8_t *smem);

// G == 1: one wavefront per task, four tasks per workgroup; waves stride over
// the task list so that a grid smaller than the list (device-side counts)
// still covers it.  G > 1: one workgroup of G wavefronts per task.
template <int R, int MODE, bool TB, bool SMALLA, int G>
__global__ __launch_bounds__(G == 8 ? 512 : 256) void strip_kernel(StripArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int ntasks = a.dyn_ntasks ? min(*a.dyn_ntasks, a.ntasks) : a.ntasks;
  if (G == 1) {
    for (int task = blockIdx.x * 4 + wave; task < ntasks; task += gridDim.x * 4)
      strip_task<R, MODE, TB, SMALLA, 1>(a, task, wave, lane, smem);
  } else {
    for (int task = blockIdx.x; task < ntasks; task += gridDim.x) {
      strip_task<R, MODE, TB, SMALLA, G>(a, task, wave, lane, smem);
      __syncthreads(); // the next task re-initialises the counters
    }
  }
}

template <int R, int MODE, bool TB, bool SMALLA, int G>
__device__ void strip_task(const StripArgs &a, int task, int wave, int lane, uint8_t *smem) {
  const PairTask tk = a.tasks[task];
  const int p = tk.pair;
  const int M = a.b.q_len[p];
  const int N = a.b.r_len[p];
  const uint8_t *Q = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];
  const DevScoring *sc = a.sc;
  const int A = sc->alphabet;
  const int go = sc->gap_open, ge = sc->gap_extend, goe = go + ge;
  aln_result *res = a.res + p;

  if (M == 0 || N == 0) {
    if (lane == 0 && wave == (G == 1 ? wave : 0)) {
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

  // LDS.  G == 1: per wave [boundary row | profile].  G > 1: [G boundary
  // buffers | G profiles | prog[G], cons[G], per-wave results[5G] |
  // reference codes].  With the reference in LDS the step loop issues no
  // global load, so no step waits on the traceback stores in flight.
  uint8_t *wbase = (G == 1) ? smem + (size_t)wave * (a.lds_bnd + a.lds_prof) : smem;
  int8_t *prof = reinterpret_cast<int8_t *>(
      (G == 1) ? wbase + a.lds_bnd : smem + (size_t)G * a.lds_bnd + (size_t)wave * a.lds_prof);
  int *ctr = reinterpret_cast<int *>(smem + (size_t)G * (a.lds_bnd + a.lds_prof));
  int *prog = ctr, *cons = ctr + G, *red = ctr + 2 * G;
  uint8_t *rseq = reinterpret_cast<uint8_t *>(ctr + kStripCtrWords * G);
  auto ring = [&](int s) { return reinterpret_cast<int2 *>(wbase + (size_t)(G == 1 ? 0 : s % G) * a.lds_bnd); };
  auto stamp = [&](int s, int col) { return s * (N + 1) + col; };
  if (G > 1) {
    if (threadIdx.x < 2 * G) ctr[threadIdx.x] = -1;
    for (int k = threadIdx.x; k < N + 128; k += 64 * G) rseq[k] = k < N ? Rs[k] : 0;
    __syncthreads();
  }
  bool ok = true;
  const int zero = a.waves - G; // 0: the launcher matches G to a.waves

  constexpr int HS = 64 * R;      // strip height
  constexpr int NW = (R + 7) / 8; // code dwords per lane per step
  const int nstrips = (M + HS - 1) / HS;
  const int T = N + 63;           // steps per strip
  const bool multi = nstrips > 1;

  int best = 0, best_i = 0, best_j = 0; // LOCAL / EXTEND (wave-uniform)
  int gh = 0;                           // GLOBAL: H(M,N)

  for (int s = (G == 1 ? 0 : wave); s < nstrips; s += G) {
    const int itop = s * HS + lane * R + 1;

    // substitution scores of this lane's rows (padding rows: -128)
    uint32_t rowtab[SMALLA ? R : 1];
    if (SMALLA) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = itop + r;
        int c = (i <= M) ? (int)Q[i - 1] : -1;
        rowtab[r] = (c >= 0 && c < A) ? sc->rowtab[c] : 0x80808080u;
      }
    } else {
      for (int cc = 0; cc < A; ++cc) {
        uint32_t w[(R + 3) / 4];
#pragma unroll
        for (int k = 0; k < (R + 3) / 4; ++k) w[k] = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = itop + r;
          int c = (i <= M) ? (int)Q[i - 1] : -1;
          int v = (c >= 0 && c < A) ? sc->mat[c * kMaxAlphabet + cc] : -128;
          w[r >> 2] |= ((uint32_t)(v & 0xff)) << ((r & 3) * 8);
        }
        if constexpr (R == 2) {
          *reinterpret_cast<uint16_t *>(prof + ((size_t)cc * 64 + lane) * R) = (uint16_t)w[0];
        } else {
          uint32_t *dst = reinterpret_cast<uint32_t *>(prof + ((size_t)cc * 64 + lane) * R);
#pragma unroll
          for (int k = 0; k < (R + 3) / 4; ++k) dst[k] = w[k];
        }
      }
    }

    // left boundary (column 0) and trackers
    int Hl[R], EN[R], eo[R], rb[R], rj[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = itop + r;
      const int h0 = (MODE == ALN_LOCAL) ? 0 : go + i * ge;
      Hl[r] = h0;
      EN[r] = h0 + goe;
      eo[r] = 4;
      rb[r] = (i <= M) ? 0 : 0x7fffffff;
      rj[r] = 0;
    }
    int hd_top = (itop - 1 == 0) ? 0 : ((MODE == ALN_LOCAL) ? 0 : go + (itop - 1) * ge);
    int out_t = 0, out_f = NEG32, out_c = 0;

    // lane-0 feeds, 64 columns at a time, read when the chunk starts: the
    // reference codes and, for s > 0, the strip above's bottom row (LDS).  A
    // global load carried across steps would make every step wait for the
    // traceback stores in flight; loaded at the chunk start, the wait comes
    // once per 64 steps.
    const int2 *bnd_in = ring(s + G - 1);
    int2 *bnd_out = ring(s);
    const bool has_reader = multi && (s + 1 < nstrips);
    const bool write_bnd = has_reader && lane == 63;
    if (G > 1 && has_reader && s >= G) // buffer free: the previous generation was read in full
      ok = ok && lds_wait_geq(&cons[s % G], stamp(s - G, N));
    int chr_cur = 0;
    int bh_cur = 0, bf_cur = 0;
    uint8_t *tbp = TB ? (a.tb + tk.tb_off + (size_t)s * T * 64 * (R / 2)) : nullptr;

    for (int t = 0; t < T; ++t) {
      // feeds are read CH columns at a time; the pipeline uses shorter
      // chunks so that a strip can start sooner behind the one above
      constexpr int CH = G > 1 ? 16 : 64;
      const int tl = t & (CH - 1);
      if (tl == 0) {
        if (G > 1) chr_cur = settle(rseq[t + lane], zero); // t + lane < N + 127
        else chr_cur = settle((t + lane < N) ? Rs[t + lane] : 0, zero);
        if (s > 0) {
          const int upto = min(t + CH, N); // columns t+1 .. t+CH
          if (G > 1) ok = ok && lds_wait_geq(&prog[(s - 1) % G], stamp(s - 1, upto));
          const int2 v = bnd_in[min(t + lane + 1, N)];
          bh_cur = settle(v.x, zero);
          bf_cur = settle(v.y, zero);
          if (G > 1) lds_publish(&cons[(s - 1) % G], stamp(s - 1, upto));
        }
      }
      const int feed_c = __builtin_amdgcn_readlane(chr_cur, tl);
      int feed_h, feed_f;
      if (s == 0) {
        feed_h = (MODE == ALN_LOCAL) ? 0 : go + (t + 1) * ge;
        feed_f = NEG32;
      } else {
        feed_h = __builtin_amdgcn_readlane(bh_cur, tl);
        feed_f = __builtin_amdgcn_readlane(bf_cur, tl);
      }
      const int in_t = dpp_wave_shr1(feed_h + goe, out_t);
      const int in_f = dpp_wave_shr1(feed_f, out_f);
      const int in_c = dpp_wave_shr1(feed_c, out_c);
      const int j = t - lane + 1;
      if (j >= 1 && j <= N) {
        int tu = in_t, fu = in_f, hd = hd_top;
        uint32_t pw[SMALLA ? 1 : (R + 3) / 4];
        if (!SMALLA) {
          const int cc = min(in_c, A - 1);
          if constexpr (R == 2) {
            pw[0] = *reinterpret_cast<const uint16_t *>(prof + ((size_t)cc * 64 + lane) * R);
          } else {
            const uint32_t *src = reinterpret_cast<const uint32_t *>(prof + ((size_t)cc * 64 + lane) * R);
#pragma unroll
            for (int k = 0; k < (R + 3) / 4; ++k) pw[k] = src[k];
          }
        }
        const int c8 = in_c << 3;
        uint32_t cw[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) cw[k] = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          int sv;
          if (SMALLA) sv = __builtin_amdgcn_sbfe((int)rowtab[r], c8, 8);
          else sv = __builtin_amdgcn_sbfe((int)pw[r >> 2], (r & 3) * 8, 8);
          const int f = max(fu + ge, tu);
          const int hdiag = hd + sv;
          int h = max(max(hdiag, EN[r]), f);
          if (MODE == ALN_LOCAL) h = max(h, 0);
          const int tt = h + goe;
          const int en = max(EN[r] + ge, tt);
          if (TB) {
            uint32_t hs = (h == hdiag) ? 0u : ((h == EN[r]) ? 1u : 2u);
            if (MODE == ALN_LOCAL && h == 0) hs = 3u;
            const uint32_t nib = hs | (uint32_t)eo[r] | ((f == tu) ? 8u : 0u);
            cw[r >> 3] |= nib << ((r & 7) * 4);
            eo[r] = (en == tt) ? 4 : 0;
          }
          if (MODE != ALN_GLOBAL) {
            if (h > rb[r]) {
              rb[r] = h;
              rj[r] = j;
            }
          }
          hd = Hl[r];
          Hl[r] = h;
          EN[r] = en;
          tu = tt;
          fu = f;
        }
        hd_top = in_t - goe;
        out_t = tu;
        out_f = fu;
        out_c = in_c;
        if (write_bnd) bnd_out[j] = make_int2(Hl[R - 1], fu);
        if (TB) {
          if constexpr (R == 2) {
            tbp[(size_t)t * 64 + lane] = (uint8_t)cw[0];
          } else if constexpr (R / 2 < 4) {
            *reinterpret_cast<uint16_t *>(tbp + ((size_t)t * 64 + lane) * (R / 2)) = (uint16_t)cw[0];
          } else {
            uint32_t *dst = reinterpret_cast<uint32_t *>(tbp + ((size_t)t * 64 + lane) * (R / 2));
#pragma unroll
            for (int k = 0; k < NW; ++k) dst[k] = cw[k];
          }
        }
      }
      // columns <= t - 63 of this strip's bottom row are written
      if (G > 1 && has_reader && tl == CH - 1)
        lds_publish(&prog[s % G], stamp(s, min(max(t - 63, 0), N)));
    }
    if (G > 1 && has_reader) lds_publish(&prog[s % G], stamp(s, N));

    if (MODE == ALN_GLOBAL) {
      if (s == nstrips - 1) {
        const int within = (M - 1) - s * HS;
        const int lM = within / R, rM = within - lM * R;
        int hv = 0;
#pragma unroll
        for (int r = 0; r < R; ++r)
          if (r == rM) hv = Hl[r];
        gh = __builtin_amdgcn_readlane(hv, lM);
      }
    } else {
      int lb = 0, li = 0, lj = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = itop + r;
        if (i <= M && rb[r] > lb) {
          lb = rb[r];
          li = i;
          lj = rj[r];
        }
      }
      const int m = wave_max(lb);
      const unsigned long long ball = __ballot(lb == m);
      const int first = __ffsll((unsigned long long)ball) - 1;
      const int ci = __builtin_amdgcn_readlane(li, first);
      const int cj = __builtin_amdgcn_readlane(lj, first);
      if (m > best) {
        best = m;
        best_i = ci;
        best_j = cj;
      }
    }
  }

  if (G > 1) {
    // combine the waves' results: within a wave strips run in i order; across
    // waves the end order (score, then i, then j) decides
    if (lane == 0) {
      red[5 * wave + 0] = best;
      red[5 * wave + 1] = best_i;
      red[5 * wave + 2] = best_j;
      red[5 * wave + 3] = gh;
      red[5 * wave + 4] = ok ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    bool all_ok = true;
    best = red[0];
    best_i = red[1];
    best_j = red[2];
    for (int w = 0; w < G; ++w) {
      all_ok = all_ok && red[5 * w + 4] != 0;
      if (w > 0 && strip_better(red[5 * w], red[5 * w + 1], red[5 * w + 2], best, best_i, best_j)) {
        best = red[5 * w];
        best_i = red[5 * w + 1];
        best_j = red[5 * w + 2];
      }
    }
    gh = red[5 * ((nstrips - 1) % G) + 3];
    if (!all_ok) res->status = ALN_R_INTERNAL;
  } else if (lane != 0) {
    return;
  }
  if (MODE == ALN_GLOBAL) {
    res->score = gh;
    res->q_end = M;
    res->r_end = N;
  } else {
    res->score = best;
    res->q_end = best_i;
    res->r_end = best_j;
  }
  res->cells = (int64_t)M * N;
}

// v = 2v + bit: the bit comes from the lane's compare mask as the carry in
__device__ __forceinline__ void shift_in(uint32_t &v, bool bit) {
  const unsigned long long km = __builtin_amdgcn_ballot_w64(bit);
  unsigned long long cc;
  asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(v), "=s"(cc) : "v"(v), "s"(km));
  (void)cc;
}

// ---------------------------------------------------------------- band
// Static band (Sec. 7.1) on the strip schedule.  Strip s sweeps only the
// columns jlo_s .. jhi_s that hold in-band cells of its rows (the union of
// the rows' bands, clipped to 1..N); lane l is on column jlo_s + t - l at
// step t, as in the full-matrix form.  Cells of that range outside a row's
// band are evaluated and their H is set to minus infinity; E and F need no
// mask: to the left of a band only F can be finite and it flows down into
// cells that are also left of the band (the band's left edge never moves
// left as i grows), to the right only E can be finite and it flows right
// into cells right of the band.  The boundary cells inside the band (row 0
// for j <= w, column 0 for rows with c(i) <= w) take their formulas; every
// other boundary cell is minus infinity.
//
// Every lane runs every step.  Before its first column and after its last
// a lane evaluates columns outside 1..N, all masked to minus infinity,
// except column 0 where it takes the boundary formula: so a lane enters
// column jlo_s with exactly the state it needs, and leaves nothing behind
// that an in-band cell reads.  With no lane idle the step has no branch.
//
// The strip's bottom row (H, F per column) goes to an LDS ring of ring_cols
// columns (column j at j mod ring_cols), which holds a whole strip range:
// a reader takes the columns of the strip above inside that strip's range
// and minus infinity outside it.  G > 1 wavefronts run consecutive strips
// as in the full-matrix pipeline (each strip its own ring, stamps per
// column).  The strip's reference codes are copied into LDS when it starts,
// so the step loop issues no global load.  Lane 0's inputs (the reference
// code and the row above) are read for CH steps at once into lanes 0..CH-1
// and move down one lane per step.
//
// Codes (4 bits per cell): per strip and lane a window of band_code_steps()
// steps starting at u_l, the lane's first in-band step rounded down to
// band_code_align(R) (one store piece), lane-major: step t of lane l is R/2 bytes
// at ((s*64 + l) * Lw + (t - u_l)) * R/2.  Eight steps (t - u_l from a
// multiple of 8) are R 32-bit words, word r holding row r's eight nibbles,
// the earlier step higher; a row's nibble, from its
// top bit: H is not the diagonal term (LOCAL: and not zero), H is not E
// (LOCAL: or is zero; with the bit above clear this marks a zero), E(i, j)
// opened from H(i, j-1), F(i, j) opened from H(i-1, j).
__device__ __forceinline__ int dpp_wave_shl1(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);
}

template <int R, int MODE, bool TB, bool SMALLA, int G>
__device__ void band_task(const StripArgs &a, int task, int wave, int lane, uint8_t *smem) {
  static_assert(R == 2 || R == 4, "the band kernel is laid out for 2 or 4 rows per lane");
  constexpr int HB = R / 2;       // code bytes per lane and step
  constexpr int NWC = 8 * HB / 4; // code dwords per lane and 8 steps
  constexpr int PW = band_code_piece(R) / 4; // code dwords per store (a piece)
  constexpr int NG = PW / NWC;                // 8-step groups per piece
  const PairTask tk = a.tasks[task];
  const int p = tk.pair;
  const int M = a.b.q_len[p];
  const int N = a.b.r_len[p];
  const uint8_t *Q = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];
  const DevScoring *sc = a.sc;
  const int A = sc->alphabet;
  const int go = sc->gap_open, ge = sc->gap_extend, goe = go + ge;
  aln_result *res = a.res + p;

  if (M == 0 || N == 0) {
    if (lane == 0 && wave == (G == 1 ? wave : 0)) {
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

  const int w = a.band_w;
  // boundary ring of RB columns (a multiple of 16, at least 64): strip s
  // keeps its bottom row's column j at (j - jlo_s - 1) mod RB, so the writes
  // of steps 64.. (columns jlo_s + 1..) fill 8 consecutive slots per 8 steps
  const int RB = a.ring_cols;
  auto rmod = [&](int x) { x %= RB; return x < 0 ? x + RB : x; };
  const size_t slot = band_slot_bytes(RB, a.lds_prof);
  uint8_t *mine = smem + (size_t)wave * slot;
  int8_t *prof = reinterpret_cast<int8_t *>(mine + (size_t)RB * 8);
  uint8_t *rref = mine + (size_t)RB * 8 + a.lds_prof;
  int *ctr = reinterpret_cast<int *>(smem + (size_t)G * slot);
  int *prog = ctr, *cons = ctr + G, *red = ctr + 2 * G;
  auto ring = [&](int s) { return reinterpret_cast<int2 *>(smem + (size_t)(G == 1 ? wave : s % G) * slot); };
  auto stamp = [&](int s, int col) { return s * (N + 1) + col; };
  if (G > 1) {
    if (threadIdx.x < 2 * G) ctr[threadIdx.x] = -1;
    __syncthreads();
  }
  bool ok = true;
  const int zero = a.waves - G; // 0: the launcher matches G to a.waves

  constexpr int HS = 64 * R;
  const int nstrips = (M + HS - 1) / HS;
  const int Lw = band_code_steps(M, N, w, R);
  auto col0 = [&](int i) { // H(i, 0) where (i, 0) lies in the band, else minus infinity
    if (band_centre(i, M, N) > w) return NEG32;
    return (MODE == ALN_LOCAL || i == 0) ? 0 : go + i * ge;
  };

  int best = 0, best_i = 0, best_j = 0; // LOCAL / EXTEND (wave-uniform)
  int gh = NEG32;                       // GLOBAL: H(M,N)
  int64_t ncells = 0;                   // this lane's in-band cells

  for (int s = (G == 1 ? 0 : wave); s < nstrips; s += G) {
    const int i0 = s * HS + 1, i1 = min(M, s * HS + HS);
    const int jlo = max(1, band_centre(i0, M, N) - w);
    const int jhi = min(N, band_centre(i1, M, N) + w);
    const int range = max(jhi - jlo + 1, 0);
    int jlo_p = 1, jhi_p = 0; // the strip above's columns
    if (s > 0) {
      jlo_p = max(1, band_centre(i0 - HS, M, N) - w);
      jhi_p = min(N, band_centre(i0 - 1, M, N) + w);
    }
    const int itop = s * HS + lane * R + 1;

    // rows: substitution scores; the band clipped to 1..N as steps, cell in
    // band iff t - bb[r] (unsigned) <= wd[r]; column 0 (B, jlo = 1 only)
    uint32_t rowtab[SMALLA ? R : 1];
    int bb[R], wd[R], B[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = itop + r;
      B[r] = NEG32;
      bb[r] = 1 << 30; // no in-band cell: t - bb wraps above every width
      wd[r] = 0;
      if (i <= M) {
        const int c = band_centre(i, M, N);
        const int lo = max(1, c - w), hi = min(N, c + w);
        if (hi >= lo) {
          bb[r] = lo - jlo + lane;
          wd[r] = hi - lo;
          ncells += hi - lo + 1;
        }
        if (jlo == 1) B[r] = col0(i);
      }
      if (SMALLA) {
        const int cq = (i <= M) ? (int)Q[i - 1] : -1;
        rowtab[r] = (cq >= 0 && cq < A) ? sc->rowtab[cq] : 0x80808080u;
      }
    }
    if (!SMALLA) {
      for (int cc = 0; cc < A; ++cc) {
        uint32_t wdw = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const int i = itop + r;
          const int cq = (i <= M) ? (int)Q[i - 1] : -1;
          const int v = (cq >= 0 && cq < A) ? sc->mat[cq * kMaxAlphabet + cc] : -128;
          wdw |= ((uint32_t)(v & 0xff)) << (r * 8);
        }
        if constexpr (R == 2)
          *reinterpret_cast<uint16_t *>(prof + ((size_t)cc * 64 + lane) * R) = (uint16_t)wdw;
        else
          *reinterpret_cast<uint32_t *>(prof + ((size_t)cc * 64 + lane) * R) = wdw;
      }
    }
    // reference codes of columns jlo .. jhi (zero past the end)
    for (int k = lane; k < range + 140; k += 64) rref[k] = k < range ? Rs[jlo - 1 + k] : 0;

    // state at column jlo - 1: column 0 by formula, else out of band; lanes
    // other than 0 rebuild it on their way to column jlo
    int Hl[R], EN[R], rb[R], rj[R];
    bool eo[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      Hl[r] = B[r];
      EN[r] = B[r] == NEG32 ? NEG32 : B[r] + goe;
      eo[r] = true;
      rb[r] = 0;
      rj[r] = 0;
    }
    // H(itop - 1, jlo - 1) for lane 0: the strip above (read with the first
    // feeds), row 0 or column 0
    int hd_top = (jlo == 1) ? col0(itop - 1) : NEG32;
    if (s == 0 && jlo > 1)
      hd_top = (jlo - 1 <= w) ? ((MODE == ALN_LOCAL) ? 0 : go + (jlo - 1) * ge) : NEG32;
    // out_t: what the lane below takes at step 0, this lane's last row at
    // column jlo - 1 (lane 1 of a strip with jlo = 1 is then on column 0 and
    // needs H(itop + R - 1, 0) as the diagonal of its first row at column 1)
    int out_t = B[R - 1] + goe, out_f = NEG32, out_c = 0;
    int wbase = 0, rfeed = 0; // ring slots: this group's first write; the feed chunk's first column

    const int2 *bnd_in = ring(s + G - 1);
    int2 *bnd_out = ring(s);
    const bool has_reader = s + 1 < nstrips;
    const bool w63 = has_reader && lane == 63; // lane 63 writes the strip's bottom row
    if (G > 1 && has_reader && s >= G) // ring free: the previous generation was read in full
      ok = ok && lds_wait_geq(&cons[s % G], stamp(s - G, N));

    // code window of this lane
    int u_l = 1 << 30;
    uint8_t *tbl = nullptr;
    if (TB) {
      if (itop <= M) u_l = (max(1, band_centre(itop, M, N) - w) - jlo + lane) & ~(band_code_align(R) - 1);
      tbl = a.tb + tk.tb_off + ((size_t)s * 64 + lane) * (size_t)Lw * HB;
    }
    uint32_t acc[NWC], pend[PW];
#pragma unroll
    for (int k = 0; k < NWC; ++k) acc[k] = 0;
#pragma unroll
    for (int k = 0; k < PW; ++k) pend[k] = 0;

    // The codes of the last piece (NG groups of 8 steps: band_code_piece()
    // bytes) wait in `pend` and go out as one aligned store.  tp: the group's
    // first step in the window (a multiple of 8); `blank` appends a group of
    // zeros.
    auto push_group = [&](int tp, bool blank) {
#pragma unroll
      for (int v = 0; v < PW - NWC; ++v) pend[v] = pend[v + NWC];
#pragma unroll
      for (int v = 0; v < NWC; ++v) pend[PW - NWC + v] = blank ? 0u : acc[v];
      const int tp0 = tp - 8 * (NG - 1); // first step of the piece
      if (((tp >> 3) & (NG - 1)) == NG - 1 && (unsigned)tp0 < (unsigned)Lw) {
        uint4 *dst = reinterpret_cast<uint4 *>(tbl + (size_t)tp0 * HB);
#pragma unroll
        for (int v = 0; v < PW / 4; ++v)
          dst[v] = make_uint4(pend[4 * v], pend[4 * v + 1], pend[4 * v + 2], pend[4 * v + 3]);
      }
    };

    // GLOBAL: H(M, N) is the last strip's row M at the step its lane is on column N
    const bool last = s == nstrips - 1;
    const int lM = (M - 1 - s * HS) / R, rM = (M - 1 - s * HS) - lM * R;
    const int t_end = N - jlo + lM;

    constexpr int CH = G > 1 ? 16 : 64; // feed chunk (steps)
    int fh = 0, ff = 0, fc = 0;         // lane k: the feed of step t + k of the chunk
    auto load_feeds = [&](int t) {
      fc = settle((int)rref[t + lane] << 3, zero);
      const int jf = jlo + t + lane;
      if (s == 0) {
        fh = (jf <= w ? ((MODE == ALN_LOCAL) ? 0 : go + jf * ge) : NEG32) + goe;
        ff = NEG32;
      } else {
        const int upto = max(min(jhi_p, jlo + t + CH - 1), 0);
        if (G > 1) ok = ok && lds_wait_geq(&prog[(s - 1) % G], stamp(s - 1, upto));
        int rx = rfeed + lane; // jf mod RB: one wrap at most (lane < 64 <= RB)
        rx = rx >= RB ? rx - RB : rx;
        const int2 v = bnd_in[rx];
        const bool inr = jf >= jlo_p && jf <= jhi_p;
        fh = settle(inr ? v.x + goe : NEG32 + goe, zero);
        ff = settle(inr ? v.y : NEG32, zero);
        if (t == 0 && jlo > 1) {
          const int jd = jlo - 1;
          const int hv = bnd_in[rmod(jd - jlo_p - 1)].x;
          if (lane == 0) hd_top = (jd >= jlo_p && jd <= jhi_p) ? hv : NEG32;
        }
        if (G > 1) lds_publish(&cons[(s - 1) % G], stamp(s - 1, upto));
      }
    };

    // one step; ZC: the first 64 steps (a lane may be on column 0, or before
    // the strip's bottom row starts at step 63);
    // GH: the eight steps holding t_end (GLOBAL, last strip)
    auto step = [&](auto zc_tag, auto gh_tag, auto nm_tag, const int t, const int k) {
      constexpr bool ZC = decltype(zc_tag)::value;
      constexpr bool GH = decltype(gh_tag)::value;
      constexpr bool NM = decltype(nm_tag)::value; // every lane on an in-band column
      if (k == 0 && (t & (CH - 1)) == 0) {
        load_feeds(t);
        rfeed = rfeed + CH >= RB ? rfeed + CH - RB : rfeed + CH;
      }
      // lane 0 takes the chunk's next feed, every other lane the lane above
      const int nh = dpp_wave_shl1(fh), nf = dpp_wave_shl1(ff), nc = dpp_wave_shl1(fc);
      const int in_t = dpp_wave_shr1(fh, out_t);
      const int in_f = dpp_wave_shr1(ff, out_f);
      const int in_c = dpp_wave_shr1(fc, out_c);
      fh = nh;
      ff = nf;
      fc = nc;
      const bool at0 = ZC && t + 1 == lane; // on column jlo - 1 (column 0 when jlo = 1)
      int tu = in_t, fu = in_f, hd = hd_top;
      uint32_t pw = 0;
      if (!SMALLA) {
        const int cc = min(in_c >> 3, A - 1);
        if constexpr (R == 2)
          pw = *reinterpret_cast<const uint16_t *>(prof + ((size_t)cc * 64 + lane) * R);
        else
          pw = *reinterpret_cast<const uint32_t *>(prof + ((size_t)cc * 64 + lane) * R);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        int sv;
        if (SMALLA) sv = __builtin_amdgcn_sbfe((int)rowtab[r], in_c, 8);
        else sv = __builtin_amdgcn_sbfe((int)pw, r * 8, 8);
        const int f = max(fu + ge, tu);
        const int hdiag = hd + sv;
        int h = max(max(hdiag, EN[r]), f);
        if (MODE == ALN_LOCAL) h = max(h, 0);
        if (!NM) h = ((unsigned)(t - bb[r]) <= (unsigned)wd[r]) ? h : NEG32;
        if (ZC) h = at0 ? B[r] : h;
        const int tt = h + goe;
        const int en = max(EN[r] + ge, tt);
        if (TB) {
          const bool nd = h != hdiag, ne = h != EN[r];
          if (MODE == ALN_LOCAL) {
            const bool z = h == 0;
            shift_in(acc[r], nd && !z);
            shift_in(acc[r], (nd && ne) || z);
          } else {
            shift_in(acc[r], nd);
            shift_in(acc[r], ne);
          }
          shift_in(acc[r], eo[r]); // a word per row: R independent shift chains
          shift_in(acc[r], f == tu);
          eo[r] = en == tt;
        }
        if (MODE != ALN_GLOBAL) {
          if (h > rb[r]) {
            rb[r] = h;
            rj[r] = jlo + t - lane;
          }
        }
        hd = Hl[r];
        Hl[r] = h;
        EN[r] = en;
        tu = tt;
        fu = f;
      }
      hd_top = in_t - goe;
      out_t = tu;
      out_f = fu;
      out_c = in_c;
      // lane 63 on a column of the strip: the strip's bottom row
      // (up to 7 columns past jhi at the end: the ring's 8 spare columns
      // keep them off the columns the reader takes)
      if (ZC) {
        if (k == 7 && t == 63 && w63) bnd_out[RB - 1] = make_int2(Hl[R - 1], fu); // column jlo
      } else if (w63) {
        bnd_out[wbase + k] = make_int2(Hl[R - 1], fu); // column jlo + t - 63
      }
      if (TB && k == 7) push_group(t - 7 - u_l, false);
      if (MODE == ALN_GLOBAL && (ZC || GH) && last && t == t_end) {
        // row rM of lane lM, read row by row (a selected register would go
        // through memory)
        int g[R];
#pragma unroll
        for (int r = 0; r < R; ++r) g[r] = __builtin_amdgcn_readlane(Hl[r], lM);
        gh = g[0];
#pragma unroll
        for (int r = 1; r < R; ++r) gh = rM == r ? g[r] : gh;
      }
      // columns <= jlo + t - 63 of this strip's bottom row are written
      if (G > 1 && has_reader && k == 7 && (t & (CH - 1)) == CH - 1)
        lds_publish(&prog[s % G], stamp(s, max(min(jhi, jlo + t - 63), 0)));
    };

    const int T = range > 0 ? range + 63 : 0;
    // the first 64 steps take the column-0 form (with jlo > 1 its override
    // sets H of a column left of every row's band to minus infinity, as the
    // mask does)
    const int tz = min(T, 64);
    wbase = 0;                              // steps 64..71: columns jlo + 1..jlo + 8
    rfeed = s > 0 ? rmod(jlo - jlo_p - 1) : 0; // column jlo in the strip above's ring
    int t8 = 0;
    using Yes = std::integral_constant<bool, true>;
    using No = std::integral_constant<bool, false>;
    for (; t8 < tz; t8 += 8) {
#pragma unroll
      for (int k = 0; k < 8; ++k) step(Yes{}, No{}, No{}, t8 + k, k);
    }
    // a band past the matrix (w >= N: every row's band is 1..N): the groups
    // whose lanes all lie on columns 1..N (steps 64 .. N - 1) need no mask;
    // rows past M then hold values no kept result reads
    const int tnm = w >= N ? N - 8 : -1;
    for (; t8 < T; t8 += 8) {
      if (MODE == ALN_GLOBAL && last && (unsigned)(t_end - t8) < 8u) {
#pragma unroll
        for (int k = 0; k < 8; ++k) step(No{}, Yes{}, No{}, t8 + k, k);
      } else if (t8 <= tnm) {
#pragma unroll
        for (int k = 0; k < 8; ++k) step(No{}, No{}, Yes{}, t8 + k, k);
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) step(No{}, No{}, No{}, t8 + k, k);
      }
      wbase = wbase + 8 == RB ? 0 : wbase + 8;
    }
    if (TB) { // the piece the last steps began (blank groups after them)
#pragma unroll
      for (int f = 1; f < NG; ++f) push_group(t8 - 8 - u_l + 8 * f, true);
    }
    if (G > 1) {
      if (has_reader) lds_publish(&prog[s % G], stamp(s, N));
      if (s > 0) lds_publish(&cons[(s - 1) % G], stamp(s - 1, N));
    }

    if (MODE != ALN_GLOBAL) {
      int lb = 0, li = 0, lj = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = itop + r;
        if (i <= M && rb[r] > lb) {
          lb = rb[r];
          li = i;
          lj = rj[r];
        }
      }
      const int m = wave_max(lb);
      const unsigned long long ball = __ballot(lb == m);
      const int first = __ffsll((unsigned long long)ball) - 1;
      const int ci = __builtin_amdgcn_readlane(li, first);
      const int cj = __builtin_amdgcn_readlane(lj, first);
      if (m > best) {
        best = m;
        best_i = ci;
        best_j = cj;
      }
    }
  }

  // in-band cells: every wavefront adds its strips' count (the result was
  // zeroed by the validation launch)
  for (int o = 32; o >= 1; o >>= 1) ncells += __shfl_xor(ncells, o, 64);
  if (lane == 0 && ncells != 0)
    atomicAdd(reinterpret_cast<unsigned long long *>(&res->cells), (unsigned long long)ncells);

  if (G > 1) {
    if (lane == 0) {
      red[5 * wave + 0] = best;
      red[5 * wave + 1] = best_i;
      red[5 * wave + 2] = best_j;
      red[5 * wave + 3] = gh;
      red[5 * wave + 4] = ok ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    bool all_ok = true;
    best = red[0];
    best_i = red[1];
    best_j = red[2];
    for (int v = 0; v < G; ++v) {
      all_ok = all_ok && red[5 * v + 4] != 0;
      if (v > 0 && strip_better(red[5 * v], red[5 * v + 1], red[5 * v + 2], best, best_i, best_j)) {
        best = red[5 * v];
        best_i = red[5 * v + 1];
        best_j = red[5 * v + 2];
      }
    }
    gh = red[5 * ((nstrips - 1) % G) + 3];
    if (!all_ok) res->status = ALN_R_INTERNAL;
  } else if (lane != 0) {
    return;
  }
  if (MODE == ALN_GLOBAL) {
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
}

template <int R, int MODE, bool TB, bool SMALLA, int G>
__global__ __launch_bounds__(G == 8 ? 512 : 256) void band_kernel(StripArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (G == 1) {
    for (int task = blockIdx.x * 4 + wave; task < a.ntasks; task += gridDim.x * 4)
      band_task<R, MODE, TB, SMALLA, 1>(a, task, wave, lane, smem);
  } else {
    for (int task = blockIdx.x; task < a.ntasks; task += gridDim.x) {
      band_task<R, MODE, TB, SMALLA, G>(a, task, wave, lane, smem);
      __syncthreads(); // the next task re-initialises the counters
    }
  }
}

// ---------------------------------------------------------------- validate
// Initialises every result and flags pairs holding a code >= alphabet.  One
// wavefront per pair (grid-stride); the codes are read as 16-byte vectors
// between the first and last 16-byte boundaries, bytewise before and after.

// Some byte of w exceeds n (n <= 127), with lim = (127 - n) * 0x01010101: a
// byte below 128 carries into its top bit exactly when it exceeds n, a byte
// of 128 or more has it set already (its carry into the next byte can only
// raise a flag the word already has).
__device__ __forceinline__ uint32_t byte_above(uint32_t w, uint32_t lim) {
  return ((w + lim) | w) & 0x80808080u;
}

__device__ __forceinline__ uint32_t seq_bad(const uint8_t *s, int64_t len, int lane, int A,
                                            uint32_t lim) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(s), e = a0 + (uintptr_t)len;
  const uintptr_t b0 = (a0 + 15) & ~(uintptr_t)15, b1 = e & ~(uintptr_t)15;
  uint32_t bad = 0;
  if (len <= 0) return 0;
  if (b0 >= b1) { // no whole 16-byte block
    for (int64_t k = lane; k < len; k += 64) bad |= s[k] >= A;
    return bad;
  }
  const int h = (int)(b0 - a0), t = (int)(e - b1); // 0..15 each
  if (lane < h) bad |= s[lane] >= A;
  if (lane < t) bad |= reinterpret_cast<const uint8_t *>(b1)[lane] >= A;
  const uint4 *v = reinterpret_cast<const uint4 *>(b0);
  const int64_t nv = (int64_t)((b1 - b0) >> 4);
  for (int64_t k = lane; k < nv; k += 64) {
    const uint4 x = v[k];
    bad |= byte_above(x.x, lim) | byte_above(x.y, lim) | byte_above(x.z, lim) |
           byte_above(x.w, lim);
  }
  return bad;
}

__global__ __launch_bounds__(256) void validate_kernel(ValidateArgs a) {
  const int lane = threadIdx.x & 63;
  if (blockIdx.x == 0 && a.reset_counter && (int)threadIdx.x < a.n_reset)
    a.reset_counter[threadIdx.x] = 0;
  const int waves = gridDim.x * (blockDim.x >> 6);
  const uint32_t lim = (uint32_t)(127 - (a.alphabet - 1)) * 0x01010101u;
  for (int p = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); p < a.n; p += waves) {
    const uint32_t bad = seq_bad(a.b.q + a.b.q_off[p], a.b.q_len[p], lane, a.alphabet, lim) |
                         seq_bad(a.b.r + a.b.r_off[p], a.b.r_len[p], lane, a.alphabet, lim);
    const bool any = __ballot(bad != 0) != 0;
    if (lane == 0) {
      aln_result *r = a.res + p;
      r->score = 0;
      r->q_end = 0;
      r->r_end = 0;
      r->q_begin = 0;
      r->r_begin = 0;
      r->status = any ? ALN_R_BAD_SYMBOL : ALN_R_OK;
      r->flags = 0;
      r->cigar_len = 0;
      r->cells = 0;
      r->cigar_off = 0;
    }
  }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_validate(const ValidateArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  const int blocks = a.n < 4 * 4096 ? (a.n + 3) / 4 : 4096; // four wavefronts each, grid-stride
  hipLaunchKernelGGL(validate_kernel, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}


template <int R, int MODE, bool TB, bool SMALLA, int G>
static hipError_t launch_strip_t(const StripArgs &a, hipStream_t s) {
  const size_t per = (size_t)(a.lds_bnd + a.lds_prof);
  const size_t lds = (G == 1 ? 4 * per : G * per) + strip_extra_bytes(G, a.max_n);
  auto kern = strip_kernel<R, MODE, TB, SMALLA, G>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int blocks = G == 1 ? (a.ntasks + 3) / 4 : a.ntasks;
  if (a.dyn_ntasks) blocks = min(blocks, 1024);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * (G == 1 ? 4 : G)), lds, s, a);
  return hipGetLastError();
}

template <int R, int MODE, int G>
static hipError_t launch_strip_m(bool tb, bool small, const StripArgs &a, hipStream_t s) {
  if (tb) return small ? launch_strip_t<R, MODE, true, true, G>(a, s) : launch_strip_t<R, MODE, true, false, G>(a, s);
  return small ? launch_strip_t<R, MODE, false, true, G>(a, s) : launch_strip_t<R, MODE, false, false, G>(a, s);
}

template <int R, int G>
static hipError_t launch_strip_r(int mode, bool tb, bool small, const StripArgs &a, hipStream_t s) {
  switch (mode) {
  case ALN_GLOBAL: return launch_strip_m<R, ALN_GLOBAL, G>(tb, small, a, s);
  case ALN_LOCAL: return launch_strip_m<R, ALN_LOCAL, G>(tb, small, a, s);
  default: return launch_strip_m<R, ALN_EXTEND, G>(tb, small, a, s);
  }
}


hipError_t launch_strip(int rows, int mode, bool tb, bool small_alphabet, const StripArgs &a,
                        hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (a.waves == kStripPipeWaves) {
    if (rows == 4) return launch_strip_r<4, kStripPipeWaves>(mode, tb, small_alphabet, a, s);
    return hipErrorInvalidValue;
  }
  if (a.waves == kStripPipeWaves2) {
    if (rows == 2) return launch_strip_r<2, kStripPipeWaves2>(mode, tb, small_alphabet, a, s);
    return hipErrorInvalidValue;
  }
  if (a.waves != 1) return hipErrorInvalidValue;
  switch (rows) {
  case 8: return launch_strip_r<8, 1>(mode, tb, small_alphabet, a, s);
  case 16: return launch_strip_r<16, 1>(mode, tb, small_alphabet, a, s);
  case 24: return launch_strip_r<24, 1>(mode, tb, small_alphabet, a, s);
  case 32: return launch_strip_r<32, 1>(mode, tb, small_alphabet, a, s);
  default: return hipErrorInvalidValue;
  }
}

template <int R, int MODE, bool TB, bool SMALLA, int G>
static hipError_t launch_band_t(const StripArgs &a, hipStream_t s) {
  const size_t lds = band_lds_bytes(G, a.ring_cols, a.lds_prof);
  auto kern = band_kernel<R, MODE, TB, SMALLA, G>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int blocks = G == 1 ? (a.ntasks + 3) / 4 : a.ntasks;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(64 * (G == 1 ? 4 : G)), lds, s, a);
  return hipGetLastError();
}

template <int R, int G>
static hipError_t launch_band_g(int mode, bool tb, bool small, const StripArgs &a, hipStream_t s) {
  switch (mode) {
  case ALN_GLOBAL:
    if (tb) return small ? launch_band_t<R, ALN_GLOBAL, true, true, G>(a, s) : launch_band_t<R, ALN_GLOBAL, true, false, G>(a, s);
    return small ? launch_band_t<R, ALN_GLOBAL, false, true, G>(a, s) : launch_band_t<R, ALN_GLOBAL, false, false, G>(a, s);
  case ALN_LOCAL:
    if (tb) return small ? launch_band_t<R, ALN_LOCAL, true, true, G>(a, s) : launch_band_t<R, ALN_LOCAL, true, false, G>(a, s);
    return small ? launch_band_t<R, ALN_LOCAL, false, true, G>(a, s) : launch_band_t<R, ALN_LOCAL, false, false, G>(a, s);
  case ALN_EXTEND:
    if (tb) return small ? launch_band_t<R, ALN_EXTEND, true, true, G>(a, s) : launch_band_t<R, ALN_EXTEND, true, false, G>(a, s);
    return small ? launch_band_t<R, ALN_EXTEND, false, true, G>(a, s) : launch_band_t<R, ALN_EXTEND, false, false, G>(a, s);
  default: return hipErrorInvalidValue;
  }
}

hipError_t launch_band_strip(int rows, int mode, bool tb, bool small_alphabet, const StripArgs &a,
                             hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (a.ring_cols < 64 || a.ring_cols > 2048 || a.ring_cols % 16 != 0) return hipErrorInvalidValue;
  if (rows != 2 && rows != 4) return hipErrorInvalidValue;
  if (a.waves == kStripPipeWaves)
    return rows == 2 ? launch_band_g<2, kStripPipeWaves>(mode, tb, small_alphabet, a, s)
                     : launch_band_g<4, kStripPipeWaves>(mode, tb, small_alphabet, a, s);
  if (a.waves == kStripPipeWaves2 && rows == 2)
    return launch_band_g<2, kStripPipeWaves2>(mode, tb, small_alphabet, a, s);
  if (a.waves == 1)
    return rows == 2 ? launch_band_g<2, 1>(mode, tb, small_alphabet, a, s)
                     : launch_band_g<4, 1>(mode, tb, small_alphabet, a, s);
  return hipErrorInvalidValue;
}

} // namespace alnk
