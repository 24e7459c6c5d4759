// kernels_sw16.hip -- Smith-Waterman (LOCAL, full matrix, score + end cell)
// in packed 16-bit integers on gfx950.
//
// Layout.  A group of G lanes (G = 16: one DPP row; G = 64: the whole
// wavefront) aligns two pairs at once: every 32-bit register holds pair A in
// its low half and pair B in its high half, so each packed instruction
// (v_pk_*_i16 / _u16) advances two cells.  Lane l of a group owns R
// consecutive query rows of a G*R-row strip and runs one column behind lane
// l-1 (an antidiagonal wavefront of R-row tiles); the bottom row's H and F
// and the reference codes move to the next lane with one DPP shift, and lane
// 0 is fed the strip's top row through a ring shifted the other way, and
// lane G-1's bottom row is staged in LDS and written out G columns at a
// time.  A
// wavefront runs either four 16-lane groups or one 64-lane group; the
// planner gives the wide form to pairs whose strips would otherwise make
// the launch wait on one wavefront.
//
// Local-alignment clamp.  With E+ = max(E, 0) and F+ = max(F, 0) the local
// recurrence is unchanged: H = max(H(i-1,j-1) + s, E+, F+), and
//   E+(i,j+1) = max(E+(i,j) + e, max(H(i,j) + o + e, 0)),
//   F+(i+1,j) = max(F+(i,j) + e, max(H(i,j) + o + e, 0)),
// where max(H + o + e, 0) is one unsigned saturating subtract (H >= 0).  So
// the zero of Smith-Waterman costs no instruction.
//
// Scores.  A per-strip int8 query profile in LDS: prof[c][lane][r] =
// s(q_row(r), c), one 8-byte read per pair and step; each byte is sign-
// extended and added to the diagonal H of its half by one SDWA add.
//
// End cell.  Per row, a 32-bit key (H << 16) | (0xffff - j) is maximised:
// the highest score, then the smallest column.  Rows are reduced in order,
// giving the first maximum in row-major order (highest score, then smallest
// i, then smallest j).
//
// Overflow.  A pair whose best score reaches 32767 - max(s) may have
// saturated; it is flagged and appended to a queue that the int32 kernel
// recomputes.  Below that bound no intermediate value can leave int16.
#include <type_traits>

#include "internal.h"

namespace alnk {

typedef unsigned short us2 __attribute__((ext_vector_type(2)));
typedef short ss2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t pk_max_i16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(ss2, a),
                                                                __builtin_bit_cast(ss2, b)));
}
__device__ __forceinline__ uint32_t pk_add_16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_bit_cast(us2, a) + __builtin_bit_cast(us2, b));
}
__device__ __forceinline__ uint32_t pk_subsat_u16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(us2, a),
                                                                    __builtin_bit_cast(us2, b)));
}

// hd + (sext(byte K of pa), sext(byte K of pb)) per 16-bit half, into a new
// register: the first SDWA add writes the low half and zero-fills the high
// one, the second writes the high half and preserves the low one.  hd is
// only read, so it needs no copy.
#define ALN_SDWA_ADD_BYTES(K)                                                                   \
  asm("v_add_u16_sdwa %0, %1, sext(%2) dst_sel:WORD_0 dst_unused:UNUSED_PAD "                  \
      "src0_sel:WORD_0 src1_sel:BYTE_" #K                                                      \
      : "=v"(out) : "v"(hd), "v"(pa));                                                         \
  asm("v_add_u16_sdwa %0, %1, sext(%2) dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE "             \
      "src0_sel:WORD_1 src1_sel:BYTE_" #K                                                      \
      : "+v"(out) : "v"(hd), "v"(pb))

template <int K>
__device__ __forceinline__ uint32_t add_score_bytes(uint32_t hd, uint32_t pa, uint32_t pb) {
  uint32_t out;
  if constexpr (K == 0) { ALN_SDWA_ADD_BYTES(0); }
  else if constexpr (K == 1) { ALN_SDWA_ADD_BYTES(1); }
  else if constexpr (K == 2) { ALN_SDWA_ADD_BYTES(2); }
  else { ALN_SDWA_ADD_BYTES(3); }
  return out;
}

__device__ __forceinline__ unsigned long long max_u64(unsigned long long a, unsigned long long b) {
  return a > b ? a : b;
}

// end-cell key: score, then smaller i, then smaller j (i, j < 2^20)
__device__ __forceinline__ unsigned long long end_key(int score, int i, int j) {
  return ((unsigned long long)(uint32_t)score << 40) |
         ((unsigned long long)(0xFFFFFu - (uint32_t)i) << 20) | (0xFFFFFu - (uint32_t)j);
}

// DPP lane shifts inside a group of G lanes: a 16-lane group is one DPP row
// (row_shr/row_shl), a 64-lane group the whole wavefront (wave_shr/wave_shl).
// Lane 0 of a right shift, and lane G-1 of a left shift, keep `old`.
template <int G>
__device__ __forceinline__ uint32_t grp_shr1(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, G == 16 ? 0x111 : 0x138, 0xf, 0xf,
                                               false);
}
template <int G>
__device__ __forceinline__ uint32_t grp_shl1(uint32_t old, uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, G == 16 ? 0x101 : 0x130, 0xf, 0xf,
                                               false);
}
// left shift with no `old`: lane G-1 reads zero, and the result needs no
// copy of another register first
template <int G>
__device__ __forceinline__ uint32_t grp_shl1z(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, G == 16 ? 0x101 : 0x130, 0xf, 0xf, true);
}

// One work item of the packed kernel: `count` tasks (two pairs each) on the
// four 16-lane groups of the wavefront (G = 16), or one task on all 64 lanes
// (G = 64).  A wide item runs 64*R-row strips, so a long pair takes a
// quarter of the strips, and of the serial time, of a 16-lane group.
template <int R, int G>
__device__ __forceinline__ void sw16_item(const Sw16Args &a, int8_t *prof, const int8_t *smat,
                                          uint2 *stage_all, int first, int count) {
  static_assert(G == 16 || G == 64, "group width");
  constexpr int NG = 64 / G;       // groups per wavefront
  constexpr int HS = G * R;        // strip height
  constexpr int NWD = R / 4;       // profile dwords per lane and letter
  const int lane = threadIdx.x;
  const int g = lane / G;
  const int gl = lane % G;
  const int A = a.sc->alphabet;
  const int PADC = A;              // profile letter for padding columns
  const int L = A + 1;             // profile letters
  const int go = a.sc->gap_open, ge = a.sc->gap_extend;
  const uint32_t goe_abs = (uint32_t)(-(go + ge)) & 0xffffu;
  const uint32_t goe2 = goe_abs | (goe_abs << 16);
  const uint32_t ge16 = (uint32_t)ge & 0xffffu;
  const uint32_t ge2 = ge16 | (ge16 << 16);

  // profile: [group][pair][letter][G lanes][R bytes]
  const size_t pair_stride = (size_t)L * G * R;
  int8_t *profA = prof + ((size_t)g * 2 + 0) * pair_stride;
  int8_t *profB = prof + ((size_t)g * 2 + 1) * pair_stride;
  uint2 *stage = stage_all + g * G; // lane G-1's bottom row over one G-step block

  Sw16Task tk;
  if (g < count) tk = a.tasks[first + g];
  else { tk.pa = -1; tk.pb = -1; tk.nstrips = 0; tk.nmax = 0; tk.bnd_off = 0; }
  int MA = 0, NA = 0, MB = 0, NB = 0;
  const uint8_t *QA = nullptr, *RA = nullptr, *QB = nullptr, *RB = nullptr;
  if (tk.pa >= 0) {
    MA = a.b.q_len[tk.pa]; NA = a.b.r_len[tk.pa];
    QA = a.b.q + a.b.q_off[tk.pa]; RA = a.b.r + a.b.r_off[tk.pa];
  }
  if (tk.pb >= 0) {
    MB = a.b.q_len[tk.pb]; NB = a.b.r_len[tk.pb];
    QB = a.b.q + a.b.q_off[tk.pb]; RB = a.b.r + a.b.r_off[tk.pb];
  }
  const int my_ns = tk.nstrips, my_nmax = tk.nmax;
  // wave-uniform trip counts: the largest over the groups
  int ns_w = 0, nmax_w = 0;
#pragma unroll
  for (int q = 0; q < NG; ++q) {
    ns_w = max(ns_w, __builtin_amdgcn_readlane(my_ns, q * G));
    nmax_w = max(nmax_w, __builtin_amdgcn_readlane(my_nmax, q * G));
  }
  const int T_w = nmax_w + G - 1;
  uint2 *bnd = reinterpret_cast<uint2 *>(a.ws + tk.bnd_off);
  unsigned long long bestA = 0, bestB = 0;

  for (int s = 0; s < ns_w; ++s) {
    const bool gact = s < my_ns;
    const int itop = s * HS + gl * R + 1;
    // ---- query profile of this lane's rows for both pairs
    if (gact) {
      int qa[R], qb[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = itop + r;
        qa[r] = (i <= MA) ? min((int)QA[i - 1], A) : A;
        qb[r] = (i <= MB) ? min((int)QB[i - 1], A) : A;
      }
      for (int c = 0; c < L; ++c) {
        uint32_t wa[NWD], wb[NWD];
#pragma unroll
        for (int k = 0; k < NWD; ++k) { wa[k] = 0; wb[k] = 0; }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          wa[r >> 2] |= ((uint32_t)(uint8_t)smat[qa[r] * kMaxAlphabet + c]) << ((r & 3) * 8);
          wb[r >> 2] |= ((uint32_t)(uint8_t)smat[qb[r] * kMaxAlphabet + c]) << ((r & 3) * 8);
        }
        uint32_t *da = reinterpret_cast<uint32_t *>(profA + ((size_t)c * G + gl) * R);
        uint32_t *db = reinterpret_cast<uint32_t *>(profB + ((size_t)c * G + gl) * R);
#pragma unroll
        for (int k = 0; k < NWD; ++k) { da[k] = wa[k]; db[k] = wb[k]; }
      }
    }
    if (s > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");

    // ---- state: H(i, j-1), E+(i, j), per-row keys
    uint32_t Hl[R], EN[R], kA[R], kB[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { Hl[r] = 0; EN[r] = 0; kA[r] = 0; kB[r] = 0; }
    uint32_t hd_top = 0;
    uint32_t out_h = 0, out_f = 0;
    // reference codes travel as profile offsets, c * G * R bytes (< 2^16),
    // pair A in the low half, pair B in the high half
    constexpr uint32_t CS = (uint32_t)G * R;
    const uint32_t padc2 = (uint32_t)PADC * CS | (((uint32_t)PADC * CS) << 16);
    auto load_c = [&](int col) -> uint32_t {
      const uint32_t ca = (col >= 1 && col <= NA) ? (uint32_t)min((int)RA[col - 1], PADC) : (uint32_t)PADC;
      const uint32_t cb = (col >= 1 && col <= NB) ? (uint32_t)min((int)RB[col - 1], PADC) : (uint32_t)PADC;
      return ca * CS | ((cb * CS) << 16);
    };
    const bool from_bnd = gact && s > 0;
    // Row rings (one per value, shifted left by one lane every step): at the
    // start of G-step block b, lane k holds the strip's top-row input for
    // column G*b + k + 1, which lane 0 consumes at step G*b + k.  At step
    // G*b + k lane G-1 stages its bottom-row output (column G*b + k + 2 - G)
    // in LDS entry k; after the block lane k writes entry k, one coalesced
    // store.  Inputs are prefetched two blocks ahead.
    auto load_blk = [&](int blk, uint32_t &c, uint32_t &h, uint32_t &f) {
      const int col = blk * G + gl + 1;
      c = padc2;
      h = 0;
      f = 0;
      if (gact) {
        c = load_c(col);
        if (from_bnd) {
          const uint2 v = bnd[min(col, my_nmax)];
          h = v.x;
          f = v.y;
        }
      }
    };
    uint32_t ring_c, ring_h, ring_f, n1_c, n1_h, n1_f, n2_c, n2_h, n2_f;
    load_blk(0, ring_c, ring_h, ring_f);
    load_blk(1, n1_c, n1_h, n1_f);
    load_blk(2, n2_c, n2_h, n2_f);
    const bool write_bnd = gact && (s + 1 < my_ns);
    auto flush = [&](int t_last, int k_done) {
      const int col = t_last - k_done + 1 + gl + 2 - G; // entry gl: step t_last - k_done + 1 + gl
      if (write_bnd && gl < k_done && col >= 1 && col <= my_nmax) bnd[col] = stage[gl];
    };

    // Reference codes travel one lane per step; lane l's code for step t+1
    // is lane l-1's code for step t, so each step reads the profile words
    // of the next step ahead of use.
    const int8_t *laneA = profA + (size_t)gl * R, *laneB = profB + (size_t)gl * R;
    auto prof_words = [&](uint32_t cc, uint32_t *wa, uint32_t *wb) {
      const uint32_t *pa = reinterpret_cast<const uint32_t *>(laneA + (cc & 0xffffu));
      const uint32_t *pb = reinterpret_cast<const uint32_t *>(laneB + (cc >> 16));
#pragma unroll
      for (int k = 0; k < NWD; ++k) { wa[k] = pa[k]; wb[k] = pb[k]; }
    };
    uint32_t cur_c = grp_shr1<G>(ring_c, padc2);
    uint32_t wa[NWD], wb[NWD], wa2[NWD], wb2[NWD];
    prof_words(cur_c, wa, wb);

    // One column step.  (wc, wbc) hold this step's profile words, (wn, wbn)
    // receive the next step's; the loop below alternates the two buffers.
    // End-cell keys of an even step are parked in (pA, pB) and folded in
    // with the odd step's keys by one three-input max.
    uint32_t pA[R], pB[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { pA[r] = 0; pB[r] = 0; }
    auto step = [&](int t, auto odd_tag, const uint32_t (&wc)[NWD], const uint32_t (&wbc)[NWD],
                    uint32_t (&wn)[NWD], uint32_t (&wbn)[NWD]) {
      constexpr bool odd = decltype(odd_tag)::value;
      const int kb = t & (G - 1);
      if (kb == 0 && t > 0) {
        flush(t - 1, G);
        ring_c = n1_c; ring_h = n1_h; ring_f = n1_f;
        n1_c = n2_c; n1_h = n2_h; n1_f = n2_f;
        load_blk(t / G + 2, n2_c, n2_h, n2_f);
      }
      // the rings move first, so that lane 0's input is taken from the old
      // ring register in place
      const uint32_t nh = grp_shl1z<G>(ring_h), nf = grp_shl1z<G>(ring_f);
      const uint32_t in_h = grp_shr1<G>(ring_h, out_h);
      const uint32_t in_f = grp_shr1<G>(ring_f, out_f);
      ring_h = nh;
      ring_f = nf;
      ring_c = grp_shl1<G>(ring_c, ring_c);
      const uint32_t lane0_next = (kb == G - 1) ? n1_c : ring_c;
      const uint32_t next_c = grp_shr1<G>(lane0_next, cur_c);
      prof_words(next_c, wn, wbn);
      // Every lane computes every step.  A lane before its first column sees
      // only the padding letter (score -128) and zero state, so all its
      // values stay 0; a lane past the last column feeds only lanes past it,
      // and its keys lose to the real cells' (its scores derive from theirs
      // by negative steps, ties go to the smaller column).  Keys of H = 0
      // are never candidates.
      const int j = t + 1 - gl;
      {
        // diagonal inputs of every row first, from H(i-1, j-1) before any
        // row overwrites its H(i, j-1)
        uint32_t hdg[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t hd = r == 0 ? hd_top : Hl[r - 1];
          switch (r & 3) {
          case 0: hdg[r] = add_score_bytes<0>(hd, wc[r >> 2], wbc[r >> 2]); break;
          case 1: hdg[r] = add_score_bytes<1>(hd, wc[r >> 2], wbc[r >> 2]); break;
          case 2: hdg[r] = add_score_bytes<2>(hd, wc[r >> 2], wbc[r >> 2]); break;
          default: hdg[r] = add_score_bytes<3>(hd, wc[r >> 2], wbc[r >> 2]); break;
          }
        }
        uint32_t tu = pk_subsat_u16(in_h, goe2);
        uint32_t fu = in_f;
        // 0xffff - j in the low half (the keys take only that half)
        const uint32_t jinv = 0xffffu - (uint32_t)j;
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const uint32_t f = pk_max_i16(pk_add_16(fu, ge2), tu);
          const uint32_t h = pk_max_i16(pk_max_i16(hdg[r], EN[r]), f);
          const uint32_t tt = pk_subsat_u16(h, goe2);
          const uint32_t en = pk_max_i16(pk_add_16(EN[r], ge2), tt);
          // bytes (high to low): pair A's H, then jinv; pair B's H, then jinv
          const uint32_t keyA = __builtin_amdgcn_perm(h, jinv, 0x05040100u);
          const uint32_t keyB = __builtin_amdgcn_perm(h, jinv, 0x07060100u);
          if constexpr (odd) {
            kA[r] = max(kA[r], max(pA[r], keyA));
            kB[r] = max(kB[r], max(pB[r], keyB));
          } else {
            pA[r] = keyA;
            pB[r] = keyB;
          }
          Hl[r] = h;
          EN[r] = en;
          tu = tt;
          fu = f;
        }
        hd_top = in_h;
        out_h = Hl[R - 1];
        out_f = fu;
      }
      if (gl == G - 1) stage[kb] = make_uint2(out_h, out_f);
      cur_c = next_c;
    };
    int t = 0;
    for (; t + 1 < T_w; t += 2) {
      step(t, std::false_type{}, wa, wb, wa2, wb2);
      step(t + 1, std::true_type{}, wa2, wb2, wa, wb);
    }
    if (t < T_w) step(t, std::false_type{}, wa, wb, wa2, wb2);
#pragma unroll
    for (int r = 0; r < R; ++r) { // keys still parked by a final even step
      kA[r] = max(kA[r], pA[r]);
      kB[r] = max(kB[r], pB[r]);
    }
    flush(T_w - 1, ((T_w - 1) & (G - 1)) + 1);
    // The strip's bottom row is written to HBM and read back by the next
    // strip of this same one-wave workgroup: workgroup-scope ordering
    // (all of its lanes share one L1) is all the hand-over needs.
    if (s + 1 < ns_w) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");

    // ---- fold this strip's row maxima into the pair's end-cell key
    unsigned long long la = 0, lb = 0;
    if (gact) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int i = itop + r;
        const int ha = (int)kA[r] >> 16, hb = (int)kB[r] >> 16;
        if (i <= MA && ha > 0) la = max_u64(la, end_key(ha, i, 0xffff - (int)(kA[r] & 0xffffu)));
        if (i <= MB && hb > 0) lb = max_u64(lb, end_key(hb, i, 0xffff - (int)(kB[r] & 0xffffu)));
      }
    }
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) {
      la = max_u64(la, __shfl_xor(la, o, G));
      lb = max_u64(lb, __shfl_xor(lb, o, G));
    }
    bestA = max_u64(bestA, la);
    bestB = max_u64(bestB, lb);
  }

  // ---- results
  for (int half = 0; half < 2; ++half) {
    const int pair = half ? tk.pb : tk.pa;
    if (gl != half || pair < 0) continue;
    const unsigned long long k = half ? bestB : bestA;
    const int M = half ? MB : MA, N = half ? NB : NA;
    aln_result *res = a.res + pair;
    const int score = (int)(k >> 40);
    res->score = score;
    res->q_end = score > 0 ? (int)(0xFFFFFu - ((k >> 20) & 0xFFFFFu)) : 0;
    res->r_end = score > 0 ? (int)(0xFFFFFu - (k & 0xFFFFFu)) : 0;
    res->cells = (int64_t)M * N;
    if (score >= a.rerun_threshold) {
      res->flags |= ALN_F_I16_RERUN;
      const int slot = atomicAdd(a.rerun_count, 1);
      PairTask t;
      t.pair = pair;
      t.rows = 16;
      t.tb_off = -1;
      t.cigar_off = 0;
      t.cigar_cap = 0;
      t.aux = 0;
      a.rerun[slot] = t;
    }
  }
}

// One workgroup (one wavefront) per work item.  Items come from the plan's
// table in the order the planner chose (longest first); without a table
// every task is its own wide item (one pair per launch).
template <int R>
__global__ __launch_bounds__(64) void sw16_kernel(Sw16Args a) {
  extern __shared__ __align__(16) uint8_t smem[];
  static_assert(R % 4 == 0, "R must be a multiple of 4");
  const int A = a.sc->alphabet;
  const int L = A + 1;
  // LDS: four groups' (or one wide group's) profiles of two pairs each, then
  // the substitution matrix as int8 [32][32] (row = query letter; letter A
  // is padding: -128)
  int8_t *prof = reinterpret_cast<int8_t *>(smem);
  int8_t *smat = prof + (size_t)8 * L * 16 * R;
  uint2 *stage = reinterpret_cast<uint2 *>(smat + kMaxAlphabet * kMaxAlphabet);
  for (int k = threadIdx.x; k < kMaxAlphabet * kMaxAlphabet; k += 64) {
    const int qa = k / kMaxAlphabet, rc = k % kMaxAlphabet;
    smat[k] = (qa < A && rc < A) ? (int8_t)a.sc->mat[k] : (int8_t)-128;
  }
  __syncthreads();
  const int item = blockIdx.x;
  Sw16Item it{item, -1};
  if (a.items != nullptr) {
    if (item >= a.nitems) return;
    it = a.items[item];
  } else if (item >= a.ntasks) {
    return;
  }
  if (it.count < 0) sw16_item<R, 64>(a, prof, smat, stage, it.first, 1);
  else sw16_item<R, 16>(a, prof, smat, stage, it.first, it.count);
}

hipError_t launch_sw16(int rows, const Sw16Args &a, hipStream_t s) {
  const int blocks = a.items ? a.nitems : a.ntasks;
  if (blocks <= 0) return hipSuccess;
  const size_t lds = sw16_lds_bytes(rows, a.sc_alphabet);
  auto go = [&](auto kern) -> hipError_t {
    if (lds > 64 * 1024) {
      hipError_t e = hipFuncSetAttribute((const void *)kern,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(64), lds, s, a);
    return hipGetLastError();
  };
  switch (rows) {
  case 4: return go(sw16_kernel<4>);
  case 8: return go(sw16_kernel<8>);
  case 12: return go(sw16_kernel<12>);
  case 16: return go(sw16_kernel<16>);
  default: return hipErrorInvalidValue;
  }
}

} // namespace alnk
