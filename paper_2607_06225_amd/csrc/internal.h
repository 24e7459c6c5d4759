// internal.h -- declarations shared by the host runtime (aln_api.cpp) and the
// gfx950 kernels.  Not part of the public ABI (include/aln.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "aln.h"

namespace alnk {

// Minus infinity in int32 kernels.  Far enough from INT32_MIN that sums of a
// few "minus infinity" terms with scores and gap penalties cannot wrap.
constexpr int32_t NEG32 = -(1 << 30);
constexpr int kMaxAlphabet = 32;

// Scoring scheme resident on the device (one per aln_set_scoring call).
struct DevScoring {
  int32_t alphabet;
  int32_t gap_open;
  int32_t gap_extend;
  int32_t max_s;        // largest substitution score
  int32_t min_s;        // smallest substitution score
  int32_t match_mismatch; // 1: diagonal all equal, off-diagonal all equal
  int32_t match, mismatch;
  int32_t mat[kMaxAlphabet * kMaxAlphabet]; // s(a,b) = mat[a*32+b]
  // rowtab[a]: bytes s(a,0..3) packed little-endian (alphabet <= 4)
  uint32_t rowtab[kMaxAlphabet];
};

// One pair's entry in a launch's work list (uploaded into the workspace).
struct PairTask {
  int32_t pair;      // index into the batch
  int32_t rows;      // rows per lane (strip kernel) / window elements per lane
  int64_t tb_off;    // byte offset of the pair's traceback codes (-1: none)
  int64_t cigar_off; // first word of the pair's CIGAR slot
  int32_t cigar_cap; // words in the slot
  int32_t aux;       // kernel-specific
};

struct BatchPtrs {
  const uint8_t *q;
  const int64_t *q_off;
  const int32_t *q_len;
  const uint8_t *r;
  const int64_t *r_off;
  const int32_t *r_len;
};

struct StripArgs {
  BatchPtrs b;
  const PairTask *tasks;
  int32_t ntasks;            // upper bound when dyn_ntasks is set
  const int32_t *dyn_ntasks; // device-side task count (re-run queues), or null
  int32_t mode;
  const DevScoring *sc;
  uint8_t *tb;        // traceback base (workspace)
  aln_result *res;
  int32_t lds_bnd;    // bytes of LDS per wave for the inter-strip row (0: none)
  int32_t lds_prof;   // bytes of LDS per wave for the query profile (0: none)
  int32_t waves;      // wavefronts per pair: 1, or kStripPipeWaves / kStripPipeWaves2
                      // (a pipeline of strips handed over through LDS; 4 / 2
                      // rows per lane)
  int32_t max_n;      // pipeline: largest N of the launch (reference codes in LDS)
  int32_t band_w;     // static band on strips: half-width w (band kernel only)
  int32_t ring_cols;  // band kernel: columns of one LDS boundary ring (power of two)
};

// Wavefronts per pair of the full-matrix strip pipeline: four (4 rows per
// lane), or eight (2 rows per lane: two wavefronts per SIMD of the CU).
constexpr int kStripPipeWaves = 4;
constexpr int kStripPipeWaves2 = 8;
constexpr int kStripCtrWords = 7; // per pipeline wave: prog, cons, 5 result words
// LDS of a G-wavefront pipeline workgroup beyond its buffers and profiles:
// prog[G], cons[G] and five result words per wave, then the reference codes
// (N + 128 bytes, the last 128 zero)
inline size_t strip_extra_bytes(int G, int n) {
  return G > 1 ? (size_t)kStripCtrWords * G * 4 + (((size_t)n + 128 + 15) & ~(size_t)15) : 0;
}
// LDS bytes of one strip-kernel workgroup.
inline size_t strip_lds_bytes(int waves, int lds_bnd, int lds_prof, int max_n) {
  const size_t per = (size_t)(lds_bnd + lds_prof);
  return waves == 1 ? 4 * per : (size_t)waves * per + strip_extra_bytes(waves, max_n);
}

// Static band on strips (Sec. 7.1 on the schedule of Sec. 6.2): row i keeps
// c(i) - w <= j <= c(i) + w, c(i) = floor(i*N/M).  Strip s (rows s*64R + 1 ..
// s*64R + 64R) sweeps columns jlo_s .. jhi_s, the union of its rows' bands
// clipped to 1..N; its steps run t = 0 .. jhi_s - jlo_s + 63 with lane l on
// column jlo_s + t - l.
__host__ __device__ inline int band_centre(int64_t i, int32_t M, int32_t N) {
  return (int)((i * (int64_t)N) / (int64_t)M);
}
// Codes per lane and strip: the lane's R rows have their in-band columns in
// [c(i) - w, c(i + R - 1) + w] and in 1..N, at most min(2w + 2 +
// floor((R-1)N/M), N) steps; the lane's window starts at the first of them
// rounded down to a multiple of band_code_align(R) steps (one piece of
// band_code_piece(R) bytes, the fill's store unit) and is a multiple of it
// long.
// (R = 4: 16 bytes, stored as each 8 steps end; R = 2: 64 bytes, 64 steps,
// since a lane's 128-byte line then takes 128 steps to fill and smaller
// stores leave partly written lines to the memory: 133 GB written for 31 GB
// of band_long codes with 8-byte stores, 51.6 GB with 32-byte ones (whole
// sectors, and a window of 576 steps instead of 640), 44 GB with 64-byte ones)
__host__ __device__ constexpr int band_code_piece(int R) { return R == 2 ? 64 : 16; }
__host__ __device__ inline int band_code_align(int R) { return band_code_piece(R) * 2 / R; }
__host__ __device__ inline int band_code_steps(int32_t M, int32_t N, int32_t w, int R) {
  const int64_t al = band_code_align(R);
  int64_t span = 2 * (int64_t)w + 2 + ((int64_t)(R - 1) * N) / M;
  if (span > N) span = N;
  const int64_t v = span + (al - 1);
  return (int)((v + al - 1) & ~(al - 1));
}
// Columns of one strip's range, at most: 2w + 1 + c(i + 64R - 1) - c(i).
__host__ __device__ inline int64_t band_strip_cols(int32_t M, int32_t N, int32_t w, int R) {
  const int64_t v = 2 * (int64_t)w + 2 + ((int64_t)(64 * R - 1) * N) / M;
  return v < N ? v : N;
}
// LDS of the band kernel per wave slot: boundary ring (int2 per column),
// query profile, reference codes of the strip's columns (+192 bytes of the
// chunk reads past the end); G > 1 adds the pipeline counters.
__host__ __device__ inline size_t band_slot_bytes(int ring_cols, int lds_prof) {
  return (size_t)ring_cols * 8 + (size_t)lds_prof + (size_t)ring_cols + 192;
}
inline size_t band_lds_bytes(int G, int ring_cols, int lds_prof) {
  const size_t slot = band_slot_bytes(ring_cols, lds_prof);
  return G == 1 ? 4 * slot : G * slot + (size_t)kStripCtrWords * G * sizeof(int);
}

// Traceback region of one side of the sixteen-sides X-drop kernel, nb =
// ceil((M + N + 1) / 64) blocks of 64 antidiagonals: from byte 0 one byte per
// antidiagonal (its first and last stored 8-cell group, and the window
// base's step from the antidiagonal before), from xdl_tb_table(nb) per block
// an int2 (the stream offset of its first code dword, 16-byte aligned, and
// the window base of the antidiagonal before it), from xdl_tb_stream(nb) the
// code dwords of every antidiagonal's stored groups, one after the other.
__host__ __device__ constexpr int64_t xdl_tb_table(int64_t nb) { return 64 * nb; }
__host__ __device__ constexpr int64_t xdl_tb_stream(int64_t nb) { return 128 * nb; }

struct WalkArgs {
  BatchPtrs b;
  const PairTask *tasks;
  int32_t ntasks;
  int32_t mode;
  int32_t layout;     // 0: strip layout, 1: diagonal layout, 2: band strips
  int32_t diag_stride; // diagonal layout: code bytes per lane and antidiagonal
                       // pair (8: bands; 2: X-drop / Z-drop, 4 diagonals per lane;
                       // 1: the sixteen-sides X-drop kernel's packed 8-cell groups)
  const int32_t *dyn_ntasks; // device-side task count (a re-run queue), or null
  int32_t band_w;            // layout 2: band half-width
  const DevScoring *sc;
  const uint8_t *tb;
  aln_result *res;
  uint32_t *cigar;
};

struct ValidateArgs {
  BatchPtrs b;
  int32_t n;
  int32_t alphabet;
  aln_result *res;
  int32_t *reset_counter; // counters zeroed by the first block (re-run queues)
  int32_t n_reset;
};

// Two pairs aligned by one 16-lane group of the packed int16 kernel.
struct Sw16Task {
  int32_t pa, pb;    // pair indices (pb = -1: none)
  int32_t nstrips;   // strips of the taller pair (16*R or, in a wide item, 64*R rows)
  int32_t nmax;      // max(N_a, N_b)
  int64_t bnd_off;   // byte offset of the group's strip-boundary row in ws
};

// One wavefront's work in the packed kernel: `count` (1..4) tasks on 16-lane
// groups, or (count < 0) the single task `first` on all 64 lanes.
struct Sw16Item {
  int32_t first;
  int32_t count;
};

// LDS of one packed-kernel workgroup: eight pairs' int8 profiles of
// (alphabet + 1) letters x 16 lanes x R rows (equally two pairs x 64 lanes),
// then the 32x32 int8 substitution matrix.
inline size_t sw16_lds_bytes(int rows, int alphabet) {
  // profiles, the int8 substitution matrix, 64 staged bottom-row entries
  return (size_t)8 * (alphabet + 1) * 16 * rows + kMaxAlphabet * kMaxAlphabet + 64 * 8;
}

struct Sw16Args {
  BatchPtrs b;
  const Sw16Task *tasks;
  int32_t ntasks;
  const Sw16Item *items;   // work items, one per workgroup; null: every task wide
  int32_t nitems;
  const DevScoring *sc;
  int32_t sc_alphabet;     // host copy of the alphabet (LDS sizing)
  uint8_t *ws;
  aln_result *res;
  int32_t *rerun_count;    // queue of pairs to recompute in int32
  PairTask *rerun;
  int32_t rerun_threshold; // best >= this: may have saturated
};

// Antidiagonal kernel (BAND, XDROP and ZDROP).
struct DiagArgs {
  BatchPtrs b;
  const PairTask *tasks;      // rows = window elements per lane (RD)
  int32_t ntasks;
  const int32_t *dyn_ntasks;  // device-side count (widening queues), or null
  int32_t band_w;
  int32_t xdrop;              // X (XDROP) or Z (ZDROP)
  const DevScoring *sc;
  uint8_t *tb;                // traceback codes + per-antidiagonal window base
  aln_result *res;
  int32_t *widen_count;       // XDROP pairs whose region outgrew the window
  PairTask *widen;
  int32_t widen_rows;         // RD of the next wider kernel (0: none)
  int32_t match_mismatch;     // 1: the scoring is one match and one mismatch score
};

// X-drop extension, sixteen sides per wavefront (match / mismatch scoring,
// alphabet <= 4, no traceback): a persistent grid takes tasks from a queue.
struct XdlArgs {
  BatchPtrs b;
  const PairTask *tasks;     // longest first
  int32_t ntasks;
  int32_t *queue;            // two counters, zero at launch; zero again at exit
  int32_t xdrop;
  int32_t gap_open, gap_extend, match, mismatch;
  aln_result *res;
  int32_t *widen_count;      // regions wider than 64 cells per antidiagonal
  PairTask *widen;
  int32_t widen_rows;        // RD of the wider kernel
  uint8_t *tb;               // traceback form: code regions (task tb_off)
  int32_t zdrop;             // 1: Z-drop (xdrop holds Z), scores only
};

// Score-major search for unit-cost edit distance: one workgroup per task,
// of `waves` wavefronts (1: one F row in LDS; 4: two rows, the previous
// score's and the current one's).
struct SearchArgs {
  BatchPtrs b;
  const PairTask *tasks;
  int32_t ntasks;
  aln_result *res;
  int32_t lds_q, lds_r, lds_f; // LDS bytes: query codes, reference codes, one F row
  int32_t waves;
  // gap-affine penalties (pen_x = 0: unit edit costs) and the number of
  // score rows each wavefront ring keeps: H rows for s - x and s - o - e,
  // E and F rows for s - e
  int32_t pen_x, pen_o, pen_e, ring_h, ring_e;
  // gap-affine: dcap > 0 stores diagonals -dcap..dcap only (rows of lds_f
  // bytes); a pair whose range outgrows them is flagged ALN_F_WIDENED and
  // left to a second launch with dcap = 0 (rows of every diagonal), which
  // skips unflagged pairs (pass = 1)
  int32_t dcap, pass;
};

// Nussinov folding: one workgroup per sequence (tasks in LPT order).
struct FoldTask {
  int32_t seq; // index into the batch
  int32_t n;   // its length
};
struct FoldArgs {
  const uint8_t *x;
  const int64_t *off;
  const int32_t *len;
  const FoldTask *tasks;
  int32_t ntasks;
  int32_t pair[16];  // in1 of (x_i, x_j) = pair[x_i*4 + x_j]
  int32_t min_loop;  // pairs score only when j - i > min_loop
  int32_t xdrop;     // < 0: unpruned
  int32_t warmup;    // spans t <= warmup are never pruned
  int32_t max_n;     // longest sequence of the launch (LDS size)
  aln_fold_result *res;
};
// Row strides (elements) of the folded triangle, and the LDS bytes of one
// folding workgroup for sequences up to max_n long (stride >= max_n + 1).
constexpr int kFoldStrides[4] = {128, 256, 384, 512};
constexpr int kFoldCtlSlots = 3; // per-span survivor / best slots, reused every third span
inline size_t fold_lds_bytes(int elt_bytes, int stride, int max_n) {
  return (((size_t)((max_n + 1) / 2) * stride * elt_bytes + 15) & ~(size_t)15) +
         (((size_t)max_n + 15) & ~(size_t)15) + ((size_t)max_n + 4 * kFoldCtlSlots) * sizeof(int);
}

// Launchers (defined in the kernel translation units).
hipError_t launch_validate(const ValidateArgs &a, hipStream_t s);
hipError_t launch_strip(int rows, int mode, bool tb, bool small_alphabet,
                        const StripArgs &a, hipStream_t s);
// static band on strips, 2 or 4 rows per lane; a.waves wavefronts per pair
// (1 or kStripPipeWaves)
hipError_t launch_band_strip(int rows, int mode, bool tb, bool small_alphabet, const StripArgs &a,
                             hipStream_t s);
hipError_t launch_walk(int layout, const WalkArgs &a, hipStream_t s);
hipError_t launch_sw16(int rows, const Sw16Args &a, hipStream_t s);
hipError_t launch_diag(int rows, int mode, int prune, bool tb, const DiagArgs &a, hipStream_t s);
// X-drop or Z-drop (EXTEND, prune ALN_XDROP or ALN_ZDROP), four sides per
// wavefront, 8 diagonals per lane
hipError_t launch_xdrop_group(int prune, const DiagArgs &a, hipStream_t s);
hipError_t launch_walk_diag(const WalkArgs &a, hipStream_t s);
// tb: the form that also writes traceback codes (4 x 8 bytes per side and
// antidiagonal, after the window bases)
hipError_t launch_xdrop_lanes(bool tb, const XdlArgs &a, int waves, hipStream_t s);
int xdrop_lanes_waves_per_cu(bool tb); // resident wavefronts per CU
size_t xdrop_lanes_lds_bytes();
hipError_t launch_search(const SearchArgs &a, hipStream_t s);
// elt_bytes 1 (uint8 triangle) or 2 (int16); block 256, 512 or 1024 threads;
// stride one of kFoldStrides
hipError_t launch_fold(int elt_bytes, int block, int stride, const FoldArgs &a, hipStream_t s);

} // namespace alnk
