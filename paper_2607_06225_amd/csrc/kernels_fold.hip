// kernels_fold.hip -- Nussinov RNA folding on gfx950, unpruned or with X-drop
// pruning transferred from alignment.
//
// Recurrence (the RNA-folding row of the example-recurrence table, Sec. 3),
// for 0 <= i < j < n:
//   F(i,j) = max( F(i+1,j), F(i,j-1), F(i+1,j-1) + in1(i,j),
//                 max over i <= k < j of F(i,k) + F(k+1,j) ),
// F(i,i) = 0, the empty interval F(i+1,i) = 0.  The bifurcation terms at
// k = i and k = j-1 are F(i+1,j) and F(i,j-1) (F(i,i) = F(j,j) = 0), so the
// reduction over k covers the first two terms as well.
//
// Every term reads a shorter interval, so the cells of one span t = j - i are
// independent: one workgroup per sequence walks the spans t = 1 .. n-1 (the
// triangle's wavefronts; with rows flipped they are its antidiagonals, which
// the pruning rule of Sec. 9.5 counts) with a barrier between them.
//
// Storage: the whole triangle lives in LDS, folded into ceil(n/2) rows of a
// compile-time stride SC >= n + 1: row v holds span v (positions 0 .. n-1-v)
// followed by span n-1-v (positions 0 .. v), so F(p, p+t) sits at
//   t <  ceil(n/2):  t*SC + p
//   t >= ceil(n/2):  (n-1-t)*SC + t + 1 + p.
// For cell (i, i+t) the term of split k = i+u reads F(i, i+u) (span u,
// position i) and F(i+u+1, i+t) (span t-1-u, position i+u+1).  As u steps by
// one, each of the two addresses moves by SC (its span in the upper half of
// the rows, resp. the lower) or by 1 - SC: between the two break points u =
// ceil(n/2) and u = t - ceil(n/2) both steps are compile-time constants, so
// a block of eight splits reads with immediate offsets from two address
// registers and costs an add and a max per term.  Lanes take consecutive
// cells i, so the reads of a wave are consecutive bytes.  Elements are int16
// (minus infinity = -32768) or, when every score fits, uint8 (at most 253;
// 255 is minus infinity), which halves LDS so that 500-nt sequences fit a CU.
//
// Work split per wavefront: each wave takes 64 consecutive cells; when there
// are fewer such chunks than waves, the u-range of each chunk is split among
// waves and their partial maxima meet in LDS (one more barrier).
//
// X-drop (Sec. 7.2 rule, Sec. 9.5 transfer): candidates of span t are the
// positions from one before the first survivor of span t-1 to its last
// survivor, inside the triangle; past the warm-up (t > warmup) a cell more
// than X below the best score of the earlier spans is removed (reads as minus
// infinity).  A cell with no live term reads minus infinity too.  The result
// is the best surviving cell: highest F, then the largest span, then the
// smallest i.
#include "internal.h"

namespace alnk {

namespace {


// element traits: minus infinity and the per-term / final encodings
template <typename T, bool XD> struct FoldElt;
template <bool XD> struct FoldElt<int16_t, XD> {
  static constexpr int kDead = -32768;
  // term of two stored values; minus infinity stays negative
  __device__ static int term(int l, int r) { return l + r; }
  // a live result v >= 0
  __device__ static bool live(int v) { return v >= 0; }
  __device__ static int value(int v) { return v; }
  __device__ static int inner(int in, int s) { return in + s; } // in: stored F(i+1,j-1)
  static constexpr int kAccInit = -65536;
};
template <> struct FoldElt<uint8_t, false> { // every cell live: plain sums
  static constexpr int kDead = 255;
  __device__ static int term(int l, int r) { return l + r; }
  __device__ static bool live(int v) { return v >= 0; }
  __device__ static int value(int v) { return v; }
  __device__ static int inner(int in, int s) { return in + s; }
  static constexpr int kAccInit = -1;
};
template <> struct FoldElt<uint8_t, true> {
  // live values 0..253, 255 = minus infinity.  A term l + r + 1 is at most
  // 254 when both are live (it is a lower bound of F(i,j) + 1) and at least
  // 256 when one is 255; read as a signed 9-bit field it is F + 1 > 0 or
  // negative.
  static constexpr int kDead = 255;
  __device__ static int term(int l, int r) {
    return __builtin_amdgcn_sbfe(l + r + 1, 0, 9);
  }
  __device__ static bool live(int v) { return v >= 1; }
  __device__ static int value(int v) { return v - 1; }
  __device__ static int inner(int in, int s) { return __builtin_amdgcn_sbfe(in + s + 1, 0, 9); }
  static constexpr int kAccInit = -1;
};

// Maximum / minimum over the wave by DPP (prefix within each 16-lane row,
// then across rows); lane 63 ends with the result.  Lanes without a source
// read the identity.
__device__ __forceinline__ int fold_wave_max(int v) {
  constexpr int id = INT32_MIN;
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false)); // row_shr:1
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false)); // row_shr:2
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false)); // row_shr:4
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false)); // row_shr:8
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false)); // row_bcast:15
  v = max(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false)); // row_bcast:31
  return v;
}
__device__ __forceinline__ int fold_wave_min(int v) {
  constexpr int id = INT32_MAX;
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x111, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x112, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x114, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x118, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x142, 0xa, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(id, v, 0x143, 0xc, 0xf, false));
  return v;
}

} // namespace

// Element index of F(p, p+u) in the folded triangle (H = ceil(n/2)).
template <int SC>
__device__ __forceinline__ int fold_at(int u, int p, int n, int H) {
  return u < H ? u * SC + p : (n - 1 - u) * SC + u + 1 + p;
}

// cnt splits with compile-time address steps D1 / D2, eight per block from
// the block's lowest address (immediate offsets), into two accumulators.
template <typename T, bool XD, int D1, int D2>
__device__ __forceinline__ void fold_run(const T *G, int &a1, int &a2, int cnt, int &acc0,
                                         int &acc1) {
  using E = FoldElt<T, XD>;
  constexpr int U = 8;
  for (; cnt >= U; cnt -= U) {
    // the block's lowest addresses; the empty asm keeps the compiler from
    // folding them back into one add per read (DS offsets are unsigned)
    int b1 = D1 > 0 ? a1 : a1 + (U - 1) * D1;
    int b2 = D2 > 0 ? a2 : a2 + (U - 1) * D2;
    asm volatile("" : "+v"(b1), "+v"(b2));
    const T *p1 = G + b1;
    const T *p2 = G + b2;
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int o1 = D1 > 0 ? k * D1 : (U - 1 - k) * -D1;
      const int o2 = D2 > 0 ? k * D2 : (U - 1 - k) * -D2;
      const int tv = E::term((int)p1[o1], (int)p2[o2]);
      if (k & 1) acc1 = max(acc1, tv);
      else acc0 = max(acc0, tv);
    }
    a1 += U * D1;
    a2 += U * D2;
  }
  for (; cnt > 0; --cnt) {
    acc0 = max(acc0, E::term((int)G[a1], (int)G[a2]));
    a1 += D1;
    a2 += D2;
  }
}

// Maximum over splits u in [u0, u1) of the bifurcation terms of cell (i, i+t).
template <typename T, bool XD, int SC>
__device__ __forceinline__ int fold_partial(const T *G, int n, int H, int t, int i, int u0,
                                            int u1) {
  using E = FoldElt<T, XD>;
  int acc0 = E::kAccInit, acc1 = E::kAccInit;
  int u = u0;
  int a1 = fold_at<SC>(u, i, n, H), a2 = fold_at<SC>(t - 1 - u, i + u + 1, n, H);
  while (u < u1) {
    // the segment up to the next break point: span u leaves the upper rows
    // at u = H, span t-1-u enters them at u = t - H
    int e = u1;
    if (u < H) e = min(e, H);
    if (u < t - H) e = min(e, t - H);
    const int cnt = e - u;
    const bool top1 = u < H, top2 = t - 1 - u < H;
    if (top1 && top2) fold_run<T, XD, SC, 1 - SC>(G, a1, a2, cnt, acc0, acc1);
    else if (top1) fold_run<T, XD, SC, SC>(G, a1, a2, cnt, acc0, acc1);
    else if (top2) fold_run<T, XD, 1 - SC, 1 - SC>(G, a1, a2, cnt, acc0, acc1);
    else fold_run<T, XD, 1 - SC, SC>(G, a1, a2, cnt, acc0, acc1);
    u = e;
    // crossing a break point moves an address by other than its step
    if (u < u1) {
      a1 = fold_at<SC>(u, i, n, H);
      a2 = fold_at<SC>(t - 1 - u, i + u + 1, n, H);
    }
  }
  return max(acc0, acc1);
}

template <typename T, bool XD, int B, int SC>
__global__ __launch_bounds__(B) void fold_kernel(FoldArgs a) {
  using E = FoldElt<T, XD>;
  constexpr int W = B / 64;
  extern __shared__ __align__(16) uint8_t smem[];
  const FoldTask tk = a.tasks[blockIdx.x];
  const int n = tk.n;
  const int sq = tk.seq;
  aln_fold_result *res = a.res + sq;
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63;

  // LDS: G (folded triangle) | codes | partial maxima (one int per cell of
  // a span) | control
  const int H = (n + 1) >> 1;
  const int gbytes = (int)(((size_t)((a.max_n + 1) >> 1) * SC * sizeof(T) + 15) & ~(size_t)15);
  T *G = reinterpret_cast<T *>(smem);
  uint8_t *xs = smem + gbytes;
  int *red = reinterpret_cast<int *>(smem + gbytes + ((n + 15) & ~15));
  int *ctl = red + a.max_n; // [slot][0 lo, 1 hi, 2 best key]
  __shared__ int bad;
  __shared__ int pair[16];

  if (tid == 0) bad = 0;
  if (tid < 16) pair[tid] = a.pair[tid];
  for (int s = tid; s < kFoldCtlSlots * 4; s += B) ctl[s] = (s % 4 == 0) ? INT32_MAX : -1;
  for (int s = tid; s < n; s += B) red[s] = E::kAccInit;
  __syncthreads();
  const uint8_t *src = a.x + a.off[sq];
  int mine = 0;
  for (int p = tid; p < n; p += B) {
    const uint8_t c = src[p];
    mine |= c > 3;
    xs[p] = c;
  }
  if (mine) atomicOr(&bad, 1);
  // span 0: F(i,i) = 0; every longer span starts as minus infinity when
  // cells can be left unevaluated (X-drop)
  if (XD)
    for (int e = tid; e < H * SC; e += B) G[e] = (T)E::kDead;
  __syncthreads();
  for (int p = tid; p < n; p += B) G[p] = (T)0; // span 0 (row 0, upper part)
  __syncthreads();
  if (bad || n <= 1) {
    if (tid == 0) {
      res->score = 0;
      res->i = 0;
      res->j = 0;
      res->full = (!bad && n == 1) ? 1 : 0;
      res->cells = 0;
      res->terms = 0;
      res->status = bad ? ALN_R_BAD_SYMBOL : ALN_R_OK;
      res->reserved = 0;
    }
    return;
  }

  int best = 0, bi = 0, bj = 0; // best cell through the last span (span 0: F = 0 at (0,0))
  int lo = 0, hi = n - 1;       // survivors of the last span
  long long cells = 0, terms = 0;
  int full = 0;
  const int X = a.xdrop;
  for (int t = 1; t < n; ++t) {
    const int ca = XD ? max(lo - 1, 0) : 0;
    const int cb = XD ? min(hi, n - 1 - t) : n - 1 - t;
    if (ca > cb) break;
    const int c = cb - ca + 1;
    cells += c;
    terms += (long long)c * t;
    const int slot = t % kFoldCtlSlots;
    int *cs = ctl + 4 * slot;
    const bool prune = XD && t > a.warmup;
    // survivors / best of this span; the slot two spans back is free again
    if (tid == 0) {
      int *nx = ctl + 4 * ((t + 1) % kFoldCtlSlots);
      nx[0] = INT32_MAX;
      nx[1] = -1;
      nx[2] = -1;
    }
    // this thread's survivors and best cell of the span, combined per wave
    // (DPP) and then per workgroup (one LDS atomic per wave)
    int my_lo = INT32_MAX, my_hi = -1, my_key = -1;
    // finish cell i of span t from its bifurcation maximum
    auto finish = [&](int i, int acc) {
      const int j = i + t;
      const int in = (t == 1) ? 0 : (int)G[fold_at<SC>(t - 2, i + 1, n, H)];
      const int s = (j - i > a.min_loop) ? pair[xs[i] * 4 + xs[j]] : 0;
      int v = max(acc, E::inner(in, s));
      bool keep = E::live(v);
      const int f = keep ? E::value(v) : 0;
      if (keep && prune && best - f > X) keep = false;
      G[fold_at<SC>(t, i, n, H)] = keep ? (T)f : (T)E::kDead;
      if (keep) {
        my_lo = min(my_lo, i);
        my_hi = max(my_hi, i);
        my_key = max(my_key, (f << 16) | (0xffff - i)); // highest F, then smallest i
      }
    };
    // 64 cells per wave; when fewer chunks than waves, each chunk's
    // u-range is cut into S = 2^ls pieces of len splits (shifts only: the
    // scalar unit, shared by the CU's waves, has no divide)
    const int chunks = (c + 63) >> 6;
    const int cl = chunks > 1 ? 32 - __builtin_clz(chunks - 1) : 0; // ceil(log2(chunks))
    const int ls = chunks >= W ? 0 : (31 - __builtin_clz(W)) - cl;
    const int S = 1 << ls;
    const int len = (t + S - 1) >> ls;
    int *rb = red;
    for (int item = wave; item < chunks * S; item += W) {
      const int ch = item >> ls, seg = item & (S - 1);
      const int u0 = min(seg * len, t), u1 = min(u0 + len, t);
      const int q = ch * 64 + lane;
      // lanes past the last cell read inside the triangle and drop the result
      const int i = ca + min(q, c - 1);
      const int acc = fold_partial<T, XD, SC>(G, n, H, t, i, u0, u1);
      if (q < c) {
        if (S == 1) finish(ca + q, acc);
        else atomicMax(&rb[q], acc);
      }
    }
    if (S > 1) {
      __syncthreads();
      for (int q = tid; q < c; q += B) {
        finish(ca + q, rb[q]);
        rb[q] = E::kAccInit; // ready for the next span (its atomics follow the barrier below)
      }
    }
    {
      const int wk = fold_wave_max(my_key);
      const int wl = XD ? fold_wave_min(my_lo) : 0;
      const int wh = XD ? fold_wave_max(my_hi) : 0;
      if (lane == 63 && wk >= 0) {
        if (XD) {
          atomicMin(&cs[0], wl);
          atomicMax(&cs[1], wh);
        }
        atomicMax(&cs[2], wk);
      }
    }
    __syncthreads();
    // every thread reads the span's outcome (the slot is not written again
    // before two more barriers)
    const int key = cs[2];
    if (key >= 0) {
      const int f = key >> 16, wi = 0xffff - (key & 0xffff);
      if (f >= best) { // a longer span wins ties
        best = f;
        bi = wi;
        bj = wi + t;
      }
    }
    if (XD) {
      if (key < 0) break; // nothing survived: the fold stops
      lo = cs[0];
      hi = cs[1];
    }
    if (t == n - 1) full = key >= 0;
  }
  if (tid == 0) {
    res->score = best;
    res->i = bi;
    res->j = bj;
    res->full = full;
    res->cells = cells;
    res->terms = terms;
    res->status = ALN_R_OK;
    res->reserved = 0;
  }
}


template <typename T, bool XD, int B, int SC>
static hipError_t launch_fold_t(const FoldArgs &a, hipStream_t s) {
  const size_t lds = fold_lds_bytes(sizeof(T), SC, a.max_n);
  auto kern = fold_kernel<T, XD, B, SC>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(a.ntasks), dim3(B), lds, s, a);
  return hipGetLastError();
}

template <typename T, bool XD, int B>
static hipError_t launch_fold_s(int stride, const FoldArgs &a, hipStream_t s) {
  switch (stride) {
  case 128: return launch_fold_t<T, XD, B, 128>(a, s);
  case 256: return launch_fold_t<T, XD, B, 256>(a, s);
  case 384: return launch_fold_t<T, XD, B, 384>(a, s);
  case 512: return launch_fold_t<T, XD, B, 512>(a, s);
  default: return hipErrorInvalidValue;
  }
}

template <typename T, bool XD>
static hipError_t launch_fold_b(int block, int stride, const FoldArgs &a, hipStream_t s) {
  switch (block) {
  case 256: return launch_fold_s<T, XD, 256>(stride, a, s);
  case 512: return launch_fold_s<T, XD, 512>(stride, a, s);
  case 1024: return launch_fold_s<T, XD, 1024>(stride, a, s);
  default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fold(int elt_bytes, int block, int stride, const FoldArgs &a, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  if (a.max_n + 1 > stride) return hipErrorInvalidValue;
  const bool xd = a.xdrop >= 0;
  if (elt_bytes == 2)
    return xd ? launch_fold_b<int16_t, true>(block, stride, a, s)
              : launch_fold_b<int16_t, false>(block, stride, a, s);
  if (elt_bytes == 1)
    return xd ? launch_fold_b<uint8_t, true>(block, stride, a, s)
              : launch_fold_b<uint8_t, false>(block, stride, a, s);
  return hipErrorInvalidValue;
}

} // namespace alnk
