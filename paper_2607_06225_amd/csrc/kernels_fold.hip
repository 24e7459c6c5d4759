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
// Storage: the whole triangle lives in LDS in sheared, span-major order,
// G[t][p] = F(p, p+t) at element rowoff(t) + p, rowoff(t) = t*n - t(t-1)/2.
// For cell (i, i+t) the term of split k = i+u reads G[u][i] and
// G[t-1-u][i+u+1]: as lanes take consecutive cells i, both reads are
// consecutive elements across the wave (no bank conflicts), and with the
// loop over u the same for every lane the row offsets stay in scalar
// registers.  Elements are int16 (minus infinity = -32768) or, when every
// score fits, uint8 (254 at most; 255 is minus infinity), which halves LDS
// so that 500-nt sequences fit and more short sequences share a CU.
//
// Work split per wavefront: each wave takes 64*CPL consecutive cells (CPL =
// 1, 2 or 4 cells per lane, the cells of a lane adjacent so their reads share
// one address register); when there are fewer cell chunks than waves, the
// u-range of each chunk is split among waves and their partial maxima meet in
// LDS (one more barrier).  CPL and the split are chosen per span for the
// fewest instructions on the busiest wave.
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

constexpr int kFoldCtlSlots = 3; // per-span survivor / best slots, reused every third span

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

__device__ __forceinline__ int rowoff(int t, int n) { return t * n - ((t * (t - 1)) >> 1); }

} // namespace

// Partial maxima of CPL adjacent cells i0 .. i0+CPL-1 (span t) over splits u
// in [u0, u1): acc[m] = max over u of term(G[u][i0+m], G[t-1-u][i0+m+u+1]).
template <typename T, bool XD, int CPL>
__device__ __forceinline__ void fold_partial(const T *G, int n, int t, int i0, int u0, int u1,
                                             int (&acc)[CPL]) {
  using E = FoldElt<T, XD>;
  int accb[CPL];
#pragma unroll
  for (int m = 0; m < CPL; ++m) {
    acc[m] = E::kAccInit;
    accb[m] = E::kAccInit;
  }
  // scalar row offsets of the two operands, stepped with u
  int r1 = rowoff(u0, n);          // G[u]
  int r2 = rowoff(t - 1 - u0, n);  // G[t-1-u]
  int u = u0;
  // two splits per iteration into separate accumulators (shorter max chains)
  for (; u + 1 < u1; u += 2) {
    const T *a1 = G + r1 + i0;
    const T *b1 = G + r2 + i0 + u + 1;
    const int r1n = r1 + (n - u);
    const int w = t - 1 - u;
    const int r2n = r2 - (n - w + 1);
    const T *a2 = G + r1n + i0;
    const T *b2 = G + r2n + i0 + u + 2;
#pragma unroll
    for (int m = 0; m < CPL; ++m) {
      acc[m] = max(acc[m], E::term((int)a1[m], (int)b1[m]));
      accb[m] = max(accb[m], E::term((int)a2[m], (int)b2[m]));
    }
    r1 = r1n + (n - u - 1);
    r2 = r2n - (n - w + 2);
  }
  if (u < u1) {
    const T *a1 = G + r1 + i0;
    const T *b1 = G + r2 + i0 + u + 1;
#pragma unroll
    for (int m = 0; m < CPL; ++m) acc[m] = max(acc[m], E::term((int)a1[m], (int)b1[m]));
  }
#pragma unroll
  for (int m = 0; m < CPL; ++m) acc[m] = max(acc[m], accb[m]);
}

template <typename T, bool XD, int B>
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

  // LDS: G (triangle) | codes | partial maxima (one int per cell of a span) |
  // control
  const int gbytes = (int)(((size_t)n * (n + 1) / 2 * sizeof(T) + 15) & ~(size_t)15);
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
  for (int p = tid; p < n; p += B) G[p] = (T)0;
  if (XD)
    for (int e = n + tid; e < n * (n + 1) / 2; e += B) G[e] = (T)E::kDead;
  __syncthreads();
  if (bad || n <= 1) {
    if (tid == 0) {
      res->score = 0;
      res->i = 0;
      res->j = 0;
      res->full = (!bad && n == 1) ? 1 : 0;
      res->cells = 0;
      res->status = bad ? ALN_R_BAD_SYMBOL : ALN_R_OK;
      res->reserved = 0;
    }
    return;
  }

  int best = 0, bi = 0, bj = 0; // best cell through the last span (span 0: F = 0 at (0,0))
  int lo = 0, hi = n - 1;       // survivors of the last span
  long long cells = 0;
  int full = 0;
  const int X = a.xdrop;
  for (int t = 1; t < n; ++t) {
    const int ca = XD ? max(lo - 1, 0) : 0;
    const int cb = XD ? min(hi, n - 1 - t) : n - 1 - t;
    if (ca > cb) break;
    const int c = cb - ca + 1;
    cells += c;
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
    // finish cell i of span t from its bifurcation maximum
    auto finish = [&](int i, int acc) {
      const int j = i + t;
      const int in = (t == 1) ? 0 : (int)G[rowoff(t - 2, n) + i + 1];
      const int s = (j - i > a.min_loop) ? pair[xs[i] * 4 + xs[j]] : 0;
      int v = max(acc, E::inner(in, s));
      bool keep = E::live(v);
      const int f = keep ? E::value(v) : 0;
      if (keep && prune && best - f > X) keep = false;
      G[rowoff(t, n) + i] = keep ? (T)f : (T)E::kDead;
      if (keep) {
        if (XD) {
          atomicMin(&cs[0], i);
          atomicMax(&cs[1], i);
        }
        atomicMax(&cs[2], (f << 16) | (0xffff - i)); // highest F, then smallest i
      }
    };
    // cells per lane (CPL) and the split of each chunk's u-range among
    // waves (S): the choice with the fewest instructions on the busiest
    // wave, about (t / S) * (2 + 2 CPL) per item (two address adds per split
    // plus an add and a max per cell)
    int cpl = 1, chunks = 1, S = 1;
    {
      long long best_cost = -1;
      for (int cand = 1; cand <= 4; cand *= 2) {
        const int ch = (c + 64 * cand - 1) / (64 * cand);
        int sp = 1;
        long long cost;
        if (ch >= W) {
          cost = (long long)((ch + W - 1) / W) * t * (2 + 2 * cand);
        } else {
          sp = min(W / ch, t);
          cost = (long long)((t + sp - 1) / sp) * (2 + 2 * cand);
        }
        if (best_cost < 0 || cost < best_cost) {
          best_cost = cost;
          cpl = cand;
          chunks = ch;
          S = sp;
        }
      }
    }
    const int chunk_cells = 64 * cpl;
    int *rb = red;
    for (int item = wave; item < chunks * S; item += W) {
      const int ch = item / S, seg = item - ch * S;
      const int u0 = (int)((long long)seg * t / S), u1 = (int)((long long)(seg + 1) * t / S);
      const int q0 = ch * chunk_cells + lane * cpl; // first cell of this lane
      // lanes past the last cell read inside the triangle (clamped) and drop
      // their result
      const int qc = min(q0, c - cpl > 0 ? c - cpl : 0);
      const int i0 = ca + qc;
      int acc[4];
      if (cpl == 4) fold_partial<T, XD, 4>(G, n, t, i0, u0, u1, reinterpret_cast<int(&)[4]>(acc));
      else if (cpl == 2) fold_partial<T, XD, 2>(G, n, t, i0, u0, u1, reinterpret_cast<int(&)[2]>(acc));
      else fold_partial<T, XD, 1>(G, n, t, i0, u0, u1, reinterpret_cast<int(&)[1]>(acc));
      // acc[m] belongs to cell qc + m; a clamped lane owns cells q0 .. c-1
      for (int m = 0; m < cpl; ++m) {
        const int q = qc + m;
        if (q < q0 || q >= c) continue;
        if (S == 1) finish(ca + q, acc[m]);
        else atomicMax(&rb[q], acc[m]);
      }
    }
    if (S > 1) {
      __syncthreads();
      for (int q = tid; q < c; q += B) {
        finish(ca + q, rb[q]);
        rb[q] = E::kAccInit; // ready for the next span (its atomics follow the barrier below)
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
    res->status = ALN_R_OK;
    res->reserved = 0;
  }
}

size_t fold_lds_bytes(int elt_bytes, int max_n) {
  return (((size_t)max_n * (max_n + 1) / 2 * elt_bytes + 15) & ~(size_t)15) +
         (((size_t)max_n + 15) & ~(size_t)15) + ((size_t)max_n + 4 * kFoldCtlSlots) * sizeof(int);
}

template <typename T, bool XD, int B>
static hipError_t launch_fold_t(const FoldArgs &a, hipStream_t s) {
  const size_t lds = fold_lds_bytes(sizeof(T), a.max_n);
  auto kern = fold_kernel<T, XD, B>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(a.ntasks), dim3(B), lds, s, a);
  return hipGetLastError();
}

template <typename T, bool XD>
static hipError_t launch_fold_b(int block, const FoldArgs &a, hipStream_t s) {
  switch (block) {
  case 256: return launch_fold_t<T, XD, 256>(a, s);
  case 512: return launch_fold_t<T, XD, 512>(a, s);
  case 1024: return launch_fold_t<T, XD, 1024>(a, s);
  default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fold(int elt_bytes, int block, const FoldArgs &a, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  const bool xd = a.xdrop >= 0;
  if (elt_bytes == 2)
    return xd ? launch_fold_b<int16_t, true>(block, a, s) : launch_fold_b<int16_t, false>(block, a, s);
  if (elt_bytes == 1)
    return xd ? launch_fold_b<uint8_t, true>(block, a, s) : launch_fold_b<uint8_t, false>(block, a, s);
  return hipErrorInvalidValue;
}

} // namespace alnk
