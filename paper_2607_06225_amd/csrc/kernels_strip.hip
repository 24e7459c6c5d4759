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
#include "internal.h"

namespace alnk {

__device__ __forceinline__ int dpp_wave_shr1(int old, int v) {
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}

__device__ __forceinline__ int wave_max(int v) {
  for (int o = 32; o >= 1; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

template <int R, int MODE, bool TB, bool SMALLA>
__device__ void strip_task(const StripArgs &a, int task, int wave, int lane, uint8_t *smem);

// One wavefront per task; waves stride over the task list so that a grid
// smaller than the list (device-side counts) still covers it.
template <int R, int MODE, bool TB, bool SMALLA>
__global__ __launch_bounds__(256) void strip_kernel(StripArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int ntasks = a.dyn_ntasks ? min(*a.dyn_ntasks, a.ntasks) : a.ntasks;
  for (int task = blockIdx.x * 4 + wave; task < ntasks; task += gridDim.x * 4)
    strip_task<R, MODE, TB, SMALLA>(a, task, wave, lane, smem);
}

template <int R, int MODE, bool TB, bool SMALLA>
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

  uint8_t *wbase = smem + (size_t)wave * (a.lds_bnd + a.lds_prof);
  int2 *bnd = reinterpret_cast<int2 *>(wbase);
  int8_t *prof = reinterpret_cast<int8_t *>(wbase + a.lds_bnd);

  constexpr int HS = 64 * R;      // strip height
  constexpr int NW = (R + 7) / 8; // code dwords per lane per step
  const int nstrips = (M + HS - 1) / HS;
  const int T = N + 63;           // steps per strip
  const bool multi = nstrips > 1;

  int best = 0, best_i = 0, best_j = 0; // LOCAL / EXTEND (wave-uniform)
  int gh = 0;                           // GLOBAL: H(M,N)

  for (int s = 0; s < nstrips; ++s) {
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
        uint32_t *dst = reinterpret_cast<uint32_t *>(prof + ((size_t)cc * 64 + lane) * R);
#pragma unroll
        for (int k = 0; k < (R + 3) / 4; ++k) dst[k] = w[k];
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

    // 64-column chunks of lane-0 feeds: reference codes and (strip > 0) the
    // previous strip's bottom row; double-buffered
    int chr_cur = 0, chr_nxt = 0, bh_cur = 0, bh_nxt = 0, bf_cur = 0, bf_nxt = 0;
    {
      const int j0 = lane, j1 = 64 + lane;
      chr_cur = (j0 < N) ? Rs[j0] : 0;
      chr_nxt = (j1 < N) ? Rs[j1] : 0;
      if (s > 0) {
        int2 v0 = bnd[min(j0 + 1, N)];
        int2 v1 = bnd[min(j1 + 1, N)];
        bh_cur = v0.x; bf_cur = v0.y;
        bh_nxt = v1.x; bf_nxt = v1.y;
      }
    }
    const bool write_bnd = multi && (s + 1 < nstrips) && lane == 63;
    uint8_t *tbp = TB ? (a.tb + tk.tb_off + (size_t)s * T * 64 * (R / 2)) : nullptr;

    for (int t = 0; t < T; ++t) {
      const int tl = t & 63;
      if (tl == 0 && t > 0) {
        chr_cur = chr_nxt;
        bh_cur = bh_nxt;
        bf_cur = bf_nxt;
        const int jn = t + 64 + lane;
        chr_nxt = (jn < N) ? Rs[jn] : 0;
        if (s > 0) {
          int2 v = bnd[min(jn + 1, N)];
          bh_nxt = v.x;
          bf_nxt = v.y;
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
          const uint32_t *src = reinterpret_cast<const uint32_t *>(prof + ((size_t)cc * 64 + lane) * R);
#pragma unroll
          for (int k = 0; k < (R + 3) / 4; ++k) pw[k] = src[k];
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
        if (write_bnd) bnd[j] = make_int2(Hl[R - 1], fu);
        if (TB) {
          uint32_t *dst = reinterpret_cast<uint32_t *>(tbp + ((size_t)t * 64 + lane) * (R / 2));
#pragma unroll
          for (int k = 0; k < NW; ++k) dst[k] = cw[k];
        }
      }
    }

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

  if (lane == 0) {
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
}

// ---------------------------------------------------------------- validate
// Initialises every result and flags pairs holding a code >= alphabet.
__global__ __launch_bounds__(256) void validate_kernel(ValidateArgs a) {
  const int p = blockIdx.x;
  if (p >= a.n) return;
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  const int M = a.b.q_len[p], N = a.b.r_len[p];
  const uint8_t *Q = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];
  int mine = 0;
  for (int k = threadIdx.x; k < M; k += blockDim.x) mine |= (Q[k] >= a.alphabet);
  for (int k = threadIdx.x; k < N; k += blockDim.x) mine |= (Rs[k] >= a.alphabet);
  if (mine) atomicOr(&bad, 1);
  __syncthreads();
  if (p == 0 && a.reset_counter && (int)threadIdx.x < a.n_reset) a.reset_counter[threadIdx.x] = 0;
  if (threadIdx.x == 0) {
    aln_result *r = a.res + p;
    r->score = 0;
    r->q_end = 0;
    r->r_end = 0;
    r->q_begin = 0;
    r->r_begin = 0;
    r->status = bad ? ALN_R_BAD_SYMBOL : ALN_R_OK;
    r->flags = 0;
    r->cigar_len = 0;
    r->cells = 0;
    r->cigar_off = 0;
  }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_validate(const ValidateArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(validate_kernel, dim3(a.n), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <int R, int MODE, bool TB, bool SMALLA>
static hipError_t launch_strip_t(const StripArgs &a, hipStream_t s) {
  const size_t lds = (size_t)4 * (a.lds_bnd + a.lds_prof);
  auto kern = strip_kernel<R, MODE, TB, SMALLA>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  int blocks = (a.ntasks + 3) / 4;
  if (a.dyn_ntasks) blocks = min(blocks, 1024);
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

template <int R, int MODE>
static hipError_t launch_strip_m(bool tb, bool small, const StripArgs &a, hipStream_t s) {
  if (tb) return small ? launch_strip_t<R, MODE, true, true>(a, s) : launch_strip_t<R, MODE, true, false>(a, s);
  return small ? launch_strip_t<R, MODE, false, true>(a, s) : launch_strip_t<R, MODE, false, false>(a, s);
}

template <int R>
static hipError_t launch_strip_r(int mode, bool tb, bool small, const StripArgs &a, hipStream_t s) {
  switch (mode) {
  case ALN_GLOBAL: return launch_strip_m<R, ALN_GLOBAL>(tb, small, a, s);
  case ALN_LOCAL: return launch_strip_m<R, ALN_LOCAL>(tb, small, a, s);
  default: return launch_strip_m<R, ALN_EXTEND>(tb, small, a, s);
  }
}

hipError_t launch_strip(int rows, int mode, bool tb, bool small_alphabet, const StripArgs &a,
                        hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  switch (rows) {
  case 8: return launch_strip_r<8>(mode, tb, small_alphabet, a, s);
  case 16: return launch_strip_r<16>(mode, tb, small_alphabet, a, s);
  case 24: return launch_strip_r<24>(mode, tb, small_alphabet, a, s);
  case 32: return launch_strip_r<32>(mode, tb, small_alphabet, a, s);
  default: return hipErrorInvalidValue;
  }
}


} // namespace alnk
