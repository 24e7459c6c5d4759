// kernels_search.hip -- the score-major search schedule (Sec. 6.3) on
// gfx950: unit-cost edit distance, and gap-affine penalties (further below).
//
// The search transformation re-indexes the edit-distance recurrence by score:
// F(s, d) is the furthest row i reached on diagonal d = j - i with exactly s
// edits.  From F(s-1, .) three costly moves lead to diagonal d --
//   a mismatch   from (i, j) on d:     row F(s-1, d) + 1,
//   an insertion from (i, j) on d + 1: row F(s-1, d+1) + 1  (steps down),
//   a deletion   from (i, j) on d - 1: row F(s-1, d-1)      (steps right) --
// each kept only if it stays inside the matrix (row <= min(M, N - d)); the
// furthest survivor then advances for free along matching characters
// (extend).  The active diagonals widen by one on each side per score,
// clipped to the matrix: [max(-s, -M), min(s, N)].  The search stops at the
// first score s whose diagonal N - M reaches row M: s is the edit distance.
//
// One workgroup per pair, with both sequences and F (int16 per diagonal,
// -32768 for "not reached", so rows are at most 32767) in LDS.  Two forms:
// - search_group_kernel: four wavefronts and two F rows (previous score,
//   current score), used whenever both rows fit;
// - search_edit_kernel: one wavefront updating a single row in place, for
//   the longest pairs.  Lanes take 64 consecutive diagonals at a time; the
//   neighbours' old values come by DPP, the chunk's left neighbour from a
//   register saved before the previous chunk overwrote it, and its right
//   neighbour from LDS (not yet updated).
// Extension compares sixteen characters per step: five aligned dword reads
// per sequence and four byte aligns, then the first differing byte.
#include "internal.h"

namespace alnk {

// "Not reached": -32768 in the LDS row and, sign-extended, in registers.  A
// move from it stays negative (at most -32767) and every store maps a
// negative row back to -32768, so it never drifts towards a real row.
constexpr int16_t kNegF16 = -32768;
constexpr int kNegF = kNegF16;

__device__ __forceinline__ int fload(const int16_t *F, int idx) { return F[idx]; }

__device__ __forceinline__ int sdpp_shr1(int old, int v) { // lane l <- lane l-1
  return __builtin_amdgcn_update_dpp(old, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ int sdpp_shl1(int old, int v) { // lane l <- lane l+1
  return __builtin_amdgcn_update_dpp(old, v, 0x130, 0xf, 0xf, false);
}

// sixteen codes starting at byte `off` of an LDS sequence buffer (readable
// up to off + 19): five aligned dword reads and four byte aligns
__device__ __forceinline__ void load16(const uint8_t *buf, int off, uint64_t &lo, uint64_t &hi) {
  const uint32_t *w = reinterpret_cast<const uint32_t *>(buf + (off & ~3));
  const uint32_t sh = (uint32_t)(off & 3);
  const uint32_t w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3], w4 = w[4];
  lo = ((uint64_t)__builtin_amdgcn_alignbyte(w2, w1, sh) << 32) | __builtin_amdgcn_alignbyte(w1, w0, sh);
  hi = ((uint64_t)__builtin_amdgcn_alignbyte(w4, w3, sh) << 32) | __builtin_amdgcn_alignbyte(w3, w2, sh);
}

// advance row f of diagonal d while the next characters match, up to lim
// (sixteen characters per step: one LDS round trip and one loop test)
__device__ __forceinline__ int extend(const uint8_t *qs, const uint8_t *rs, int f, int d, int lim) {
  while (f < lim) {
    uint64_t qa, qb, ra, rb;
    load16(qs, f, qa, qb);
    load16(rs, f + d, ra, rb);
    const uint64_t x0 = qa ^ ra, x1 = qb ^ rb;
    const int n = x0 ? (__builtin_ctzll(x0) >> 3) : (x1 ? 8 + (__builtin_ctzll(x1) >> 3) : 16);
    f = min(f + n, lim);
    if (n < 16) break;
  }
  return f;
}

__global__ __launch_bounds__(64) void search_edit_kernel(SearchArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int lane = threadIdx.x;
  const int task = blockIdx.x;
  if (task >= a.ntasks) return;
  const int p = __builtin_amdgcn_readfirstlane(a.tasks[task].pair);
  aln_result *res = a.res + p;
  if (__builtin_amdgcn_readfirstlane(res->status) != ALN_R_OK) return; // bad symbol
  const int M = __builtin_amdgcn_readfirstlane(a.b.q_len[p]);
  const int N = __builtin_amdgcn_readfirstlane(a.b.r_len[p]);
  const uint8_t *Q = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];

  // LDS: query codes (M + 20 bytes, padding 0xFE), reference codes (N + 20,
  // padding 0xFF; the paddings never match each other or a code), F[d + M]
  uint8_t *qs = smem;
  uint8_t *rs = smem + a.lds_q;
  int16_t *F = reinterpret_cast<int16_t *>(smem + a.lds_q + a.lds_r);
  for (int k = lane; k < M + 20; k += 64) qs[k] = k < M ? Q[k] : 0xFE;
  for (int k = lane; k < N + 20; k += 64) rs[k] = k < N ? Rs[k] : 0xFF;
  for (int k = lane; k <= M + N; k += 64) F[k] = kNegF16;
  __syncthreads();

  const int dt = N - M; // the end cell's diagonal
  int s = 0, dmin = 0, dmax = 0;
  long long cells = 1;
  {
    const int f0 = extend(qs, rs, 0, 0, min(M, N));
    if (lane == 0) F[M] = (int16_t)f0;
  }
  __syncthreads();
  bool done = dt == 0 && __builtin_amdgcn_readfirstlane(fload(F, M)) >= M;
  while (!done && s < M + N) {
    ++s;
    dmin = max(dmin - 1, -M);
    dmax = min(dmax + 1, N);
    cells += dmax - dmin + 1;
    int carry = kNegF; // F(s-1, d0 - 1), saved before its chunk was overwritten
    for (int d0 = dmin; d0 <= dmax; d0 += 64) {
      const int d = d0 + lane;
      const bool act = d <= dmax;
      const int old = act ? fload(F, d + M) : kNegF;
      int right = sdpp_shl1(kNegF, old);
      int left = sdpp_shr1(kNegF, old);
      if (lane == 63) right = (d + 1 <= N) ? fload(F, d + 1 + M) : kNegF;
      if (lane == 0) left = carry;
      carry = __builtin_amdgcn_readlane(old, 63);
      const int lim = min(M, N - d);
      int f = kNegF;
      if (old + 1 <= lim) f = max(f, old + 1);     // mismatch
      if (right + 1 <= lim) f = max(f, right + 1); // insertion
      if (left <= lim) f = max(f, left);           // deletion
      if (act && f >= 0) f = extend(qs, rs, f, d, lim);
      if (act) F[d + M] = f >= 0 ? (int16_t)f : kNegF16;
    }
    done = dt >= dmin && dt <= dmax && __builtin_amdgcn_readfirstlane(fload(F, dt + M)) >= M;
  }
  if (lane == 0) {
    res->score = -s;
    res->q_end = M;
    res->r_end = N;
    res->cells = cells;
  }
}

// Several wavefronts per pair.  F(s-1, .) and F(s, .) live in two LDS rows
// that swap roles every score, so a step reads only the previous row and
// needs no carried neighbour: the active diagonals are cut into 64-diagonal
// chunks dealt round-robin to the wavefronts, and one barrier per score
// separates the writes of a score from the reads of the next.  A row entry
// outside the previous score's diagonals was never written (the active
// diagonals only widen, and each row is written on every other score), so it
// still reads "not reached".
template <int NWV>
__global__ __launch_bounds__(64 * NWV) void search_group_kernel(SearchArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int task = blockIdx.x;
  if (task >= a.ntasks) return;
  const int p = __builtin_amdgcn_readfirstlane(a.tasks[task].pair);
  aln_result *res = a.res + p;
  // the same status for every wavefront: the whole workgroup leaves
  if (__builtin_amdgcn_readfirstlane(res->status) != ALN_R_OK) return;
  const int M = __builtin_amdgcn_readfirstlane(a.b.q_len[p]);
  const int N = __builtin_amdgcn_readfirstlane(a.b.r_len[p]);
  const uint8_t *Q = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];

  uint8_t *qs = smem;
  uint8_t *rs = smem + a.lds_q;
  int16_t *Fp = reinterpret_cast<int16_t *>(smem + a.lds_q + a.lds_r);
  int16_t *Fn = reinterpret_cast<int16_t *>(smem + a.lds_q + a.lds_r + a.lds_f);
  for (int k = tid; k < M + 20; k += 64 * NWV) qs[k] = k < M ? Q[k] : 0xFE;
  for (int k = tid; k < N + 20; k += 64 * NWV) rs[k] = k < N ? Rs[k] : 0xFF;
  for (int k = tid; k <= M + N; k += 64 * NWV) {
    Fp[k] = kNegF16;
    Fn[k] = kNegF16;
  }
  __syncthreads();
  if (tid == 0) Fp[M] = (int16_t)extend(qs, rs, 0, 0, min(M, N));
  __syncthreads();

  const int dt = N - M;
  int s = 0, dmin = 0, dmax = 0;
  long long cells = 1;
  bool done = dt == 0 && __builtin_amdgcn_readfirstlane(fload(Fp, M)) >= M;
  while (!done && s < M + N) {
    ++s;
    dmin = max(dmin - 1, -M);
    dmax = min(dmax + 1, N);
    cells += dmax - dmin + 1;
    for (int d0 = dmin + 64 * wave; d0 <= dmax; d0 += 64 * NWV) {
      const int d = d0 + lane;
      const bool act = d <= dmax;
      int old = kNegF, left = kNegF, right = kNegF;
      if (act) {
        old = fload(Fp, d + M);
        if (d > -M) left = fload(Fp, d - 1 + M);
        if (d < N) right = fload(Fp, d + 1 + M);
      }
      const int lim = min(M, N - d);
      int f = kNegF;
      if (old + 1 <= lim) f = max(f, old + 1);     // mismatch
      if (right + 1 <= lim) f = max(f, right + 1); // insertion
      if (left <= lim) f = max(f, left);           // deletion
      if (act && f >= 0) f = extend(qs, rs, f, d, lim);
      if (act) Fn[d + M] = f >= 0 ? (int16_t)f : kNegF16;
    }
    __syncthreads();
    int16_t *t = Fp;
    Fp = Fn;
    Fn = t;
    done = dt >= dmin && dt <= dmax && __builtin_amdgcn_readfirstlane(fload(Fp, dt + M)) >= M;
  }
  if (tid == 0) {
    res->score = -s;
    res->q_end = M;
    res->r_end = N;
    res->cells = cells;
  }
}

// Gap-affine penalties: mismatch x > 0, a gap of length L costs o + L e
// (o >= 0, e > 0), a match 0.  The search keeps three wavefronts per score,
// furthest rows as before:
//   E(s, d) = max(H(s-o-e, d-1), E(s-e, d-1))       a step right, same row
//   F(s, d) = max(H(s-o-e, d+1), F(s-e, d+1)) + 1   a step down
//   H(s, d) = max(H(s-x, d) + 1, E(s, d), F(s, d)), then extended along
//             matches,
// each candidate kept only if its source was reached and it stays inside the
// matrix (row <= min(M, N - d)).  A path of penalty s spends at least e per
// diagonal it moves, so the active diagonals are |d| <= s / e, clipped to the
// matrix.  The search stops at the first s with H(s, N - M) = M: s is the
// smallest penalty, minus the Gotoh global score under (0, -x, -o, -e).
// Rows for past scores live in LDS rings (H: ring_h rows, E and F: ring_e
// rows each, slot s mod ring size); four wavefronts share a pair as in
// search_group_kernel, one barrier per score.  A slot's earlier scores had
// narrower diagonal ranges, all rewritten when it is reused, so an entry
// outside a row's range still reads "not reached".
// Rows first hold diagonals -dcap..dcap only, so that several pairs share a
// CU; a pair whose range would leave them is flagged and recomputed by a
// second launch with rows of every diagonal.  A source diagonal outside the
// stored ones was never active (the range at an earlier score was inside
// them), so it reads "not reached".
template <int NWV>
__global__ __launch_bounds__(64 * NWV) void search_affine_kernel(SearchArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int task = blockIdx.x;
  if (task >= a.ntasks) return;
  const int p = __builtin_amdgcn_readfirstlane(a.tasks[task].pair);
  aln_result *res = a.res + p;
  if (__builtin_amdgcn_readfirstlane(res->status) != ALN_R_OK) return;
  const int M = __builtin_amdgcn_readfirstlane(a.b.q_len[p]);
  const int N = __builtin_amdgcn_readfirstlane(a.b.r_len[p]);
  const uint8_t *Q = a.b.q + a.b.q_off[p];
  const uint8_t *Rs = a.b.r + a.b.r_off[p];
  if (a.pass == 1 && !(__builtin_amdgcn_readfirstlane(res->flags) & ALN_F_WIDENED)) return;
  const int X = a.pen_x, O = a.pen_o, E = a.pen_e, RH = a.ring_h, RE = a.ring_e;
  const bool capped = a.dcap > 0;
  const int off = capped ? a.dcap : M;             // row index of diagonal 0
  const int lo_st = capped ? max(-M, -a.dcap) : -M; // stored diagonals lo_st..hi_st
  const int hi_st = capped ? min(N, a.dcap) : N;

  uint8_t *qs = smem;
  uint8_t *rs = smem + a.lds_q;
  uint8_t *rows = smem + a.lds_q + a.lds_r;
  const int stride = a.lds_f; // bytes per row
  // ring slots by index (the slot of score s is s mod ring size, kept
  // incrementally below: no division in the score loop)
  auto hrow = [&](int k) { return reinterpret_cast<int16_t *>(rows + (size_t)k * stride); };
  auto erow = [&](int k) { return reinterpret_cast<int16_t *>(rows + (size_t)(RH + k) * stride); };
  auto frow = [&](int k) { return reinterpret_cast<int16_t *>(rows + (size_t)(RH + RE + k) * stride); };
  for (int k = tid; k < M + 20; k += 64 * NWV) qs[k] = k < M ? Q[k] : 0xFE;
  for (int k = tid; k < N + 20; k += 64 * NWV) rs[k] = k < N ? Rs[k] : 0xFF;
  {
    int16_t *all = reinterpret_cast<int16_t *>(rows);
    const int n16 = (RH + 2 * RE) * (stride / 2);
    for (int k = tid; k < n16; k += 64 * NWV) all[k] = kNegF16;
  }
  __syncthreads();
  if (tid == 0) hrow(0)[off] = (int16_t)extend(qs, rs, 0, 0, min(M, N));
  __syncthreads();

  const int dt = N - M;
  const int smax = 2 * O + E * (M + N); // a gap of the whole query, then one of the reference
  int s = 0;
  int sh = 0, se = 0;  // s mod RH, s mod RE
  int w = 0, wr = 0;   // s / E, s mod E
  long long cells = 1;
  bool done = dt == 0 && __builtin_amdgcn_readfirstlane(fload(hrow(0), off)) >= M;
  bool outgrown = false;
  while (!done && s < smax) {
    ++s;
    sh = sh + 1 == RH ? 0 : sh + 1;
    se = se + 1 == RE ? 0 : se + 1;
    if (++wr == E) {
      wr = 0;
      ++w;
    }
    const int dmin = max(-M, -w), dmax = min(N, w);
    if (dmin < lo_st || dmax > hi_st) { // only with capped rows (uniform)
      outgrown = true;
      break;
    }
    cells += dmax - dmin + 1;
    const bool hx = s >= X, ho = s >= O + E, ge = s >= E;
    // slots of s - X and s - O - E (both < RH back) and s - E (< RE back)
    const int shx = sh - X < 0 ? sh - X + RH : sh - X;
    const int sho = sh - O - E < 0 ? sh - O - E + RH : sh - O - E;
    const int see = se - E < 0 ? se - E + RE : se - E;
    const int16_t *Hx = hrow(shx);
    const int16_t *Ho = hrow(sho);
    const int16_t *Ee = erow(see);
    const int16_t *Fe = frow(see);
    int16_t *Hn = hrow(sh), *En = erow(se), *Fn = frow(se);
    for (int d0 = dmin + 64 * wave; d0 <= dmax; d0 += 64 * NWV) {
      const int d = d0 + lane;
      if (d <= dmax) {
        const int lim = min(M, N - d);
        int ev = kNegF, fv = kNegF, hv = kNegF;
        if (d > lo_st) { // a step right from diagonal d - 1
          int src = kNegF;
          if (ho) src = fload(Ho, d - 1 + off);
          if (ge) src = max(src, fload(Ee, d - 1 + off));
          if (src >= 0 && src <= lim) ev = src;
        }
        if (d < hi_st) { // a step down from diagonal d + 1
          int src = kNegF;
          if (ho) src = fload(Ho, d + 1 + off);
          if (ge) src = max(src, fload(Fe, d + 1 + off));
          if (src >= 0 && src + 1 <= lim) fv = src + 1;
        }
        if (hx) { // a mismatch on diagonal d
          const int v = fload(Hx, d + off);
          if (v >= 0 && v + 1 <= lim) hv = v + 1;
        }
        int h = max(hv, max(ev, fv));
        if (h >= 0) h = extend(qs, rs, h, d, lim);
        En[d + off] = ev >= 0 ? (int16_t)ev : kNegF16;
        Fn[d + off] = fv >= 0 ? (int16_t)fv : kNegF16;
        Hn[d + off] = h >= 0 ? (int16_t)h : kNegF16;
      }
    }
    __syncthreads();
    done = dt >= dmin && dt <= dmax && __builtin_amdgcn_readfirstlane(fload(hrow(sh), dt + off)) >= M;
  }
  if (tid == 0) {
    if (outgrown) {
      res->flags |= ALN_F_WIDENED;
    } else {
      res->score = -s;
      res->q_end = M;
      res->r_end = N;
      res->cells = cells;
    }
  }
}

template <typename K>
static hipError_t launch_search_k(K kern, int threads, size_t lds, const SearchArgs &a,
                                  hipStream_t s) {
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(kern, dim3(a.ntasks), dim3(threads), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_search(const SearchArgs &a, hipStream_t s) {
  if (a.ntasks <= 0) return hipSuccess;
  const size_t one = (size_t)a.lds_q + a.lds_r + a.lds_f;
  if (a.pen_x > 0) {
    if (a.waves != 4 || a.pen_e <= 0 || a.ring_h < 1 || a.ring_e < 1) return hipErrorInvalidValue;
    const size_t lds = (size_t)a.lds_q + a.lds_r + (size_t)(a.ring_h + 2 * a.ring_e) * a.lds_f;
    return launch_search_k(search_affine_kernel<4>, 256, lds, a, s);
  }
  switch (a.waves) {
  case 1: return launch_search_k(search_edit_kernel, 64, one, a, s);
  case 4: return launch_search_k(search_group_kernel<4>, 256, one + a.lds_f, a, s);
  default: return hipErrorInvalidValue;
  }
}

} // namespace alnk
