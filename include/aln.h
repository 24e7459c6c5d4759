/*
 * aln.h -- C ABI of libaln_hip.so: affine-gap (Gotoh H/E/F) pairwise alignment
 * on AMD Instinct MI355X (gfx950).
 *
 * Problem statement (paper "Compiling Bioinformatics Recurrences"):
 *   - a query q on the vertical axis (rows i = 1..M) and a reference r on the
 *     horizontal axis (columns j = 1..N); cell (i,j) scores the prefixes
 *     q[1..i] and r[1..j] (Sec. 2);
 *   - a substitution score per pair of letters and two gap constants (the
 *     sequence-alignment recurrence of Sec. 3: one match array and two gap
 *     arrays coupled through max), evaluated in Gotoh's H/E/F form with a gap
 *     of length L scoring  gap_open + L * gap_extend;
 *   - an alignment mode: GLOBAL (Needleman-Wunsch), LOCAL (Smith-Waterman:
 *     scores clamped at 0, best cell anywhere) or EXTEND (seed extension:
 *     global boundaries, best cell anywhere, the empty extension scores 0);
 *   - a pruning rule (Sec. 7): FULL (no pruning), BAND (static prune axis
 *     -w <= diag(i,j) <= w, Sec. 7.1, centred on the rectangle's diagonal:
 *     row i keeps floor(i*N/M) - w <= j <= floor(i*N/M) + w) or XDROP (dynamic
 *     pruning, Sec. 2 / Sec. 5.2 / Sec. 7.2: evaluated antidiagonal by
 *     antidiagonal, a cell scoring more than X below the best score of the
 *     earlier antidiagonals is removed and the next antidiagonal is evaluated
 *     only between the first and last surviving cells, plus one step right);
 *   - the result: optimal score, end cell, cells evaluated and, optionally,
 *     the traceback path (Sec. 2) as a CIGAR.
 * The schedule (which cells run in parallel, in what order) never changes a
 * result (Sec. 6: iteration reordering preserves values and traceback).
 *
 * Conventions
 *   Memory    Every d_* pointer is device memory owned by the caller (for
 *             example a torch tensor's data_ptr()).  The library never frees
 *             or reallocates caller memory.  *_host pointers are host memory.
 *   Streams   `stream` is a hipStream_t passed as void*; NULL is the legacy
 *             default stream.  Calls enqueue work and return; outputs are
 *             valid once the stream has synchronised.
 *   Errors    Calls return an aln_status and never abort; aln_last_error()
 *             describes the last failure on a context.  Per-pair problems go
 *             to aln_result.status (ALN_R_*).
 *   Threads   A context may be used by one host thread at a time.
 *   Codes     Sequences are byte codes 0..alphabet-1 (DNA: A,C,G,T = 0..3).
 *             A code >= alphabet marks the pair ALN_R_BAD_SYMBOL.
 *   CIGAR     BAM-style words (run_length << 4) | op with SAM op codes:
 *             I = 1 (vertical move, consumes q_i), D = 2 (horizontal move,
 *             consumes r_j), = 7, X = 8.  Runs are listed start to end.
 *   Ties      End cell: highest score, then smallest i, then smallest j.
 *             Traceback from the end cell, in state H: (LOCAL and H == 0:
 *             stop), diagonal, E, F; in E or F: open before extend.
 */
#ifndef ALN_H
#define ALN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ALN_ABI_VERSION 1

typedef int32_t aln_status;
enum {
  ALN_OK = 0,
  ALN_E_INVAL = -1,       /* bad argument                                     */
  ALN_E_NOMEM = -2,       /* host or device allocation failed                 */
  ALN_E_DEVICE = -3,      /* a HIP call failed                                */
  ALN_E_CAPACITY = -4,    /* caller buffer (workspace / CIGAR) too small      */
  ALN_E_UNSUPPORTED = -5  /* parameters outside what the kernels implement    */
};

enum { ALN_GLOBAL = 0, ALN_LOCAL = 1, ALN_EXTEND = 2 };
/* ALN_ZDROP (EXTEND only) is XDROP with the Z-drop condition of Sec. 9.3: a
 * cell (i,j) is removed when the best score of the earlier antidiagonals
 * exceeds its H by more than Z + |(j - i) - (j* - i*)|, (i*,j*) the cell of
 * that best score; Z is passed in aln_params.xdrop. */
/* ALN_SEARCH evaluates the score-major search schedule of Sec. 6.3: GLOBAL
 * mode, no CIGAR, a scoring of penalties -- every diagonal entry 0, every
 * off-diagonal entry -x < 0, gap_open -o <= 0, gap_extend -e < 0 (a gap of
 * length L costs o + L e) -- so the score is minus the smallest penalty.
 * For s = 0, 1, ... it keeps, per diagonal d = j - i with |d| <= s / e
 * (clipped to the matrix), the furthest row reached with penalty s, extended
 * along matches, and stops when diagonal N - M reaches row M.  `cells` then
 * counts those (score, diagonal) entries, s = 0 included.
 * Unit edit costs (x = 1, o = 0, e = 1: the score is minus the edit
 * distance) keep one row per score: pairs need M <= 32767 and the batch's
 * longest M plus its longest N at most about 54 000.  Other penalties keep
 * three wavefronts (H, E, F) of past scores in LDS: max(x, o + e) + 1 + 2 (e
 * + 1) rows of 2 (maxM + maxN + 1) bytes plus both sequences must fit 160 KB
 * (about 2 500 + 2 500 bases at x = 4, o = 6, e = 2).  Else
 * ALN_E_UNSUPPORTED.  A first pass keeps fewer diagonals per row; a pair
 * whose range outgrows them is recomputed and flagged ALN_F_WIDENED. */
enum { ALN_FULL = 0, ALN_BAND = 1, ALN_XDROP = 2, ALN_ZDROP = 3, ALN_SEARCH = 4 };
/* score width: AUTO lets the library choose (packed int16 where it applies,
 * with an automatic int32 re-run of any pair that could have overflowed) */
enum { ALN_W_AUTO = 0, ALN_W_I16 = 1, ALN_W_I32 = 2 };

/* per-pair result status */
enum {
  ALN_R_OK = 0,
  ALN_R_UNREACHABLE = 1, /* GLOBAL + BAND: (M,N) not connected to (0,0)      */
  ALN_R_CIGAR_CAP = 2,   /* the pair's CIGAR did not fit its slot, or (XDROP
                            / ZDROP) its region was too wide for the
                            traceback window; score and end cell are valid */
  ALN_R_BAD_SYMBOL = 3,  /* a code >= alphabet; other fields undefined       */
  ALN_R_TOO_WIDE = 4,    /* XDROP / ZDROP: the surviving region spanned more
                            than the widest kernel window (2042 diagonals)   */
  ALN_R_INTERNAL = 5     /* a kernel's bounded internal wait expired (a defect
                            of the library); other fields undefined          */
};
/* per-pair result flags */
enum {
  ALN_F_I16_RERUN = 1,  /* the int16 pass could have saturated; the pair was
                           recomputed in int32 (the result is the int32 one) */
  ALN_F_WIDENED = 2     /* X-drop / Z-drop region, or a gap-affine SEARCH's
                           diagonal range, outgrew the first window; the
                           pair was recomputed with a wider one              */
};

enum { ALN_OP_I = 1, ALN_OP_D = 2, ALN_OP_EQ = 7, ALN_OP_X = 8 };

typedef struct aln_ctx aln_ctx;
typedef struct aln_plan aln_plan;

/* Scoring scheme.  matrix: host, alphabet*alphabet int32, row = query letter,
 * column = reference letter, every entry in [-127, 127].  gap_open and
 * gap_extend in [-1024, 0]. */
typedef struct {
  int32_t alphabet; /* 1..32 */
  const int32_t *matrix;
  int32_t gap_open;
  int32_t gap_extend;
} aln_scoring;

typedef struct {
  int32_t mode;       /* ALN_GLOBAL / ALN_LOCAL / ALN_EXTEND                  */
  int32_t prune;      /* ALN_FULL / ALN_BAND / ALN_XDROP or ALN_ZDROP (EXTEND
                         only) / ALN_SEARCH (GLOBAL, penalty scoring)        */
  int32_t band_w;     /* BAND half-width w >= 0                               */
  int32_t xdrop;      /* XDROP threshold X >= 0, or ZDROP threshold Z >= 0    */
  int32_t width;      /* ALN_W_*                                              */
  int32_t want_cigar; /* 1: produce a CIGAR.  Under XDROP / ZDROP the path runs
                         from the end cell back to (0,0) through evaluated,
                         unpruned cells (same preference order); it is
                         produced when every antidiagonal up to the end
                         cell's spans at most 250 diagonals of candidates,
                         else the pair reports ALN_R_CIGAR_CAP with score,
                         end cell and cells still valid                    */
} aln_params;

typedef struct {
  int32_t score;     /* INT32_MIN when status == ALN_R_UNREACHABLE            */
  int32_t q_end;     /* end cell as prefix lengths                            */
  int32_t r_end;
  int32_t q_begin;   /* where the traceback stopped (0,0 unless LOCAL)        */
  int32_t r_begin;
  int32_t status;    /* ALN_R_*                                               */
  int32_t flags;     /* ALN_F_*                                               */
  int32_t cigar_len; /* CIGAR words; 0 without want_cigar                     */
  int64_t cells;     /* interior cells (i >= 1, j >= 1) evaluated             */
  int64_t cigar_off; /* index of the first CIGAR word in d_cigar              */
} aln_result;        /* 48 bytes */

/* A batch of n pairs in device memory: codes concatenated, per-pair start
 * offsets (int64) and lengths (int32). */
typedef struct {
  int32_t n;
  const uint8_t *q;
  const int64_t *q_off;
  const int32_t *q_len;
  const uint8_t *r;
  const int64_t *r_off;
  const int32_t *r_len;
} aln_batch;

/* Device memory a plan needs.  workspace_bytes already includes
 * traceback_bytes (4 bits per computed cell when want_cigar). */
typedef struct {
  uint64_t workspace_bytes;
  uint64_t traceback_bytes;
  uint64_t cigar_words; /* room the caller must give d_cigar                  */
  int64_t cells;        /* interior cells the plan will evaluate (FULL, BAND) */
} aln_footprint;

/* Tile choices found by the autotuner (aln_autotune) for the three kernel
 * families whose tiling is free: rows per lane of the packed int16
 * Smith-Waterman kernel, rows per lane of the int32 full-matrix strips (0:
 * the planner's per-pair choice) and the X-drop kernel's starting window
 * (diagonals per lane, and extension sides per wavefront: 1 side over all
 * 64 lanes, 4 sides of 16 lanes each, or 16 sides of 4 lanes each).  Each
 * ms[] entry is the measured time of one candidate on the tuning batch (0:
 * not measured, negative: not runnable).  While `valid`, aln_plan_create uses the chosen tiles.
 * sw16_wide_pct sets when the packed kernel gives a pair-of-pairs a whole
 * 64-lane wavefront (64*R-row strips) instead of a 16-lane group: when the
 * task's serial column steps exceed that percent of the launch's balanced
 * load per wavefront slot (0: the default, 80; -1: never).  Tiles never
 * change results. */
typedef struct {
  int32_t valid;
  int32_t sw16_rows;      /* 4, 8, 12 or 16                                   */
  int32_t strip_rows;     /* 0 (per pair and batch), 2 (eight-wavefront
                             pipeline, 2 rows per lane), 4 (four-wavefront
                             pipeline, 4 rows), 8, 16, 24 or 32               */
  int32_t xdrop_rows;     /* 2, 4 or 8                                        */
  int32_t xdrop_sides;    /* 1, 4 (with xdrop_rows 8) or 16 (with xdrop_rows
                             4: 16 sides of 4 lanes, 64 cells per side and
                             antidiagonal; X-drop without CIGAR under
                             match / mismatch scoring, else as 4x1)       */
  int32_t sw16_wide_pct;  /* 0 (default 80), -1 (never) or 1..10000          */
  double sw16_ms[4];      /* candidates 16, 12, 8, 4 (each: best of the wide
                             thresholds 25, 40, 60, 80 it was timed with)    */
  double strip_ms[7];     /* candidates 0, 2, 4, 8, 16, 24, 32                */
  double xdrop_ms[4];     /* candidates 4x1, 4x16, 8x1, 8x4 (rows x sides)    */
  int32_t band_kernel;    /* static bands: 0 (by band width), 1 (antidiagonal
                             windows), strips with 4 rows per lane and one (2)
                             or four (3) wavefronts per pair, or with 2 rows
                             per lane and one (4) or four (5); pairs the strip
                             form cannot hold stay antidiagonal               */
  int32_t reserved;
  double band_ms[5];      /* candidates 1, 2, 3, 4, 5                        */
} aln_tuning;             /* 192 bytes */

/* ABI version of the loaded library (ALN_ABI_VERSION). */
int32_t aln_abi_version(void);

/* Create a context on HIP device `device`; the context owns scoring tables,
 * plans' staging memory, streams of the server and the autotune cache. */
aln_status aln_create(aln_ctx **ctx, int32_t device);

/* A context without a device, for planning only (capacity planning, host
 * tests of the planner): aln_set_scoring keeps the scheme on the host,
 * aln_plan_create / aln_fold_plan_create plan and report footprints,
 * aln_plan_describe lists the launches and tasks.  Every call that would
 * touch a device (execute, graph capture, autotune, server, probe) returns
 * ALN_E_DEVICE after its argument checks.  cus and lds_per_cu stand in for
 * the device's compute units and LDS bytes per CU (0: 256 and 160 KiB, an
 * MI355X).  Errors: ALN_E_INVAL (negative sizes), ALN_E_NOMEM. */
aln_status aln_create_host(aln_ctx **ctx, int32_t cus, int32_t lds_per_cu);
void aln_destroy(aln_ctx *ctx);
/* Message of the last failed call on ctx (empty string if none). */
const char *aln_last_error(const aln_ctx *ctx);

/* Copy a scoring scheme to the device; it stays resident until aln_destroy.
 * Returns its id in *scoring_id. */
aln_status aln_set_scoring(aln_ctx *ctx, const aln_scoring *sc,
                           int32_t *scoring_id);

/* Plan a batch from its host-side lengths: choose kernels and tile shapes
 * (bucketing pairs by length, longest work first), lay out the workspace and
 * report the footprint.  Host work only; allocates host memory for the plan. */
aln_status aln_plan_create(aln_ctx *ctx, int32_t scoring_id,
                           const aln_params *params, int32_t n,
                           const int32_t *q_len_host, const int32_t *r_len_host,
                           aln_plan **plan, aln_footprint *fp);

/* One kernel launch of a plan's fill (re-runs that depend on device results
 * -- widening, int32 re-runs -- and the walks are not listed). */
typedef struct {
  char family[24];  /* "sw16", "strip_i32", "diag_band", "band_strip",
                       "xdrop_lanes", "xdrop_lanes_tb", "xdrop_group", "xdrop",
                       "xdrop_tb", "zdrop", "zdrop_tb", "search",
                       "search_affine", "fold"                               */
  int32_t tile;     /* rows or window per lane (fold: triangle row stride)   */
  int32_t sides;    /* X-drop: sides per wavefront; sw16: 2 pairs per lane;
                       strips, band strips: wavefronts per pair; fold: bytes
                       per element                                           */
  int32_t first;    /* its tasks in the plan's task list                     */
  int32_t count;
} aln_launch_info;  /* 40 bytes */

/* One pair (sequence, for folding) as a launch runs it. */
typedef struct {
  int32_t launch;    /* index into the launches                              */
  int32_t pair;      /* index into the batch                                 */
  int64_t tb_off;    /* its traceback codes in the workspace's traceback
                        area (-1: none)                                      */
  int64_t tb_bytes;  /* bytes reserved for them                              */
  int64_t cigar_off; /* first word of its CIGAR slot (-1: no CIGAR)          */
  int32_t cigar_cap; /* words in the slot                                    */
  int32_t tile;      /* as the launch's, per task                            */
} aln_task_info;     /* 40 bytes */

/* Describe a plan: fills up to max_launches launches and up to max_tasks
 * tasks (either pointer may be null to count only), sets *n_launches (may
 * be null) and returns the number of tasks (a packed int16 task of two pairs
 * counts twice), or ALN_E_INVAL.  Host work only. */
int64_t aln_plan_describe(const aln_plan *plan, aln_launch_info *launches,
                          int32_t max_launches, int32_t *n_launches,
                          aln_task_info *tasks, int64_t max_tasks);
void aln_plan_destroy(aln_plan *plan);

/* Run a plan on a batch whose lengths equal those it was planned with.
 * d_ws: >= fp.workspace_bytes of device memory; d_res: n results;
 * d_cigar: >= fp.cigar_words words (may be NULL without want_cigar).
 * Enqueues everything on `stream`; allocates nothing. */
aln_status aln_execute(aln_ctx *ctx, aln_plan *plan, const aln_batch *batch,
                       void *d_ws, uint64_t ws_bytes, aln_result *d_res,
                       uint32_t *d_cigar, uint64_t cigar_words, void *stream);

/* Size of the fixed workspace aln_execute_noalloc uses on each GPU. */
#define ALN_NOALLOC_WORKSPACE_BYTES (64ull << 20)

/* aln_execute without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  The workspace is a fixed device array of
 * ALN_NOALLOC_WORKSPACE_BYTES per GPU, held from the first aln_create on that
 * GPU until the process ends.  The call allocates nothing (device, pinned or
 * host memory) and creates no HIP object; the plan must come from an earlier
 * aln_plan_create.  Errors: ALN_E_CAPACITY when the plan's
 * fp.workspace_bytes exceed the array (or d_cigar is too small), ALN_E_INVAL
 * while kernel timing (aln_set_profiling) is on, else as aln_execute.
 * Results equal aln_execute's.  Every call on one GPU shares that GPU's array
 * and leaves its contents behind (the kernels clear what they need cleared):
 * calls that overlap on one GPU -- other streams, other contexts, other
 * threads -- race and give undefined results, so serialise them. */
aln_status aln_execute_noalloc(aln_ctx *ctx, aln_plan *plan, const aln_batch *batch,
                               aln_result *d_res, uint32_t *d_cigar, uint64_t cigar_words,
                               void *stream);

/* The same kernels, one launch per pair (the per-pair baseline the batched
 * form is compared with).  Same arguments and results as aln_execute. */
aln_status aln_execute_per_pair(aln_ctx *ctx, aln_plan *plan,
                                const aln_batch *batch, void *d_ws,
                                uint64_t ws_bytes, aln_result *d_res,
                                uint32_t *d_cigar, uint64_t cigar_words,
                                void *stream);

/* Capture aln_execute with these exact arguments into a HIP graph held by the
 * plan (replacing any earlier capture), then launch it on `stream`.  Later
 * calls of aln_graph_launch replay it without host-side planning. */
aln_status aln_graph_capture(aln_ctx *ctx, aln_plan *plan,
                             const aln_batch *batch, void *d_ws,
                             uint64_t ws_bytes, aln_result *d_res,
                             uint32_t *d_cigar, uint64_t cigar_words,
                             void *stream);
aln_status aln_graph_launch(aln_ctx *ctx, aln_plan *plan, void *stream);

/* Autotuner: run every candidate tile of the kernel family this batch uses
 * (packed int16 SW, int32 strips or X-drop) on the batch itself -- pass a
 * sample of a large workload -- and keep the fastest in the context's
 * tuning (the other families' choices are kept).  Same arguments as
 * aln_plan_create plus the device batch; allocates and frees its own device
 * memory and synchronises `stream`.  Bands have nothing to tune (ALN_OK). */
aln_status aln_autotune(aln_ctx *ctx, int32_t scoring_id, const aln_params *params,
                        const aln_batch *batch, const int32_t *q_len_host,
                        const int32_t *r_len_host, void *stream);
/* Read or replace the context's tile choices (for example ones saved from
 * an earlier aln_autotune on the same device). */
aln_status aln_get_tuning(const aln_ctx *ctx, aln_tuning *tuning);
aln_status aln_set_tuning(aln_ctx *ctx, const aln_tuning *tuning);

/* Kernel timing for measurement tools.  While enabled (enable = 1), every
 * kernel launch of aln_execute is bracketed by HIP events on the launch
 * stream; aln_kernel_times() synchronises those events and returns, for each
 * kernel family, the summed milliseconds and launch count since the last
 * call (then resets).  names[k] receives a static string.  Returns the number
 * of families written (<= max).  Not for use during graph capture. */
aln_status aln_set_profiling(aln_ctx *ctx, int32_t enable);
int32_t aln_kernel_times(aln_ctx *ctx, const char **names, double *ms,
                         int64_t *launches, int32_t max);

/* VALU probe for measurement tools: keeps every SIMD of the device busy with
 * one instruction class (op: 0 v_add_u32, 1 v_max_i32, 2 v_max3_i32,
 * 3 v_cmp_gt_i32, 4 v_cndmask_b32, 5 v_pk_max_i16, 6 v_pk_add_u16,
 * 7 v_lshl_or_b32, 8 v_add3_u32, 9 v_mov_b32 with DPP, 10 v_max_i32 with DPP,
 * 11 v_add_u32 with an SDWA byte operand, 12 v_perm_b32, 13 v_alignbyte_b32,
 * 14 v_bfe_u32, 15 v_addc_co_u32): waves_per_simd (1..8) waves per SIMD, each
 * running iters x 32 such instructions over 8 independent register chains
 * (dependent != 0: one chain, to time their latency).  Writes out[0] the
 * launch's milliseconds, out[1] the mean shader-clock cycles of a wave's loop
 * (s_memtime), out[2] its mean 100 MHz ticks (s_memrealtime), out[3] waves,
 * out[4] wave instructions per wave, out[5] SIMDs.  Issue rate per SIMD =
 * out[4] * waves_per_simd / out[1] wave instructions per cycle; clock =
 * 0.1 GHz * out[1] / out[2].  Synchronises the device; allocates and frees
 * a small device buffer. */
aln_status aln_valu_probe(aln_ctx *ctx, int32_t op, int32_t dependent, int32_t waves_per_simd,
                          int32_t iters, double *out);

/* ------------------------------------------------------------------------
 * RNA folding: the RNA-folding recurrence of Sec. 3's example table
 * (Nussinov base-pair maximisation) over sequences x_0 .. x_{n-1} of codes
 * A, C, G, U = 0..3, for 0 <= i < j < n:
 *   F(i,j) = max( F(i+1,j), F(i,j-1), F(i+1,j-1) + in1(i,j),
 *                 max over i <= k < j of F(i,k) + F(k+1,j) ),
 * F(i,i) = 0, the empty interval = 0, in1(i,j) = pair[x_i*4 + x_j] when
 * j - i > min_loop, else 0.  The triangle is evaluated span t = j - i by
 * span.  With xdrop >= 0 the X-drop rule (Sec. 7.2) is transferred to it
 * (Sec. 9.5): past the warm-up (t > warmup) a cell scoring more than X below
 * the best score of the earlier spans is removed, and the next span is
 * evaluated only from one position before the first survivor (by i) to the
 * last; removed and unevaluated cells read as minus infinity.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t pair[16]; /* pairing scores, each 0..127                          */
  int32_t min_loop; /* >= 0                                                 */
  int32_t xdrop;    /* < 0: unpruned; else X                                */
  int32_t warmup;   /* spans t <= warmup are never pruned (>= 0)            */
  int32_t block;    /* threads per workgroup: 256, 512 or 1024; 0: about 16
                       wavefronts per CU (a tuning choice: results do not
                       depend on it)                                        */
} aln_fold_params;  /* 80 bytes */

typedef struct {
  int32_t n;          /* sequences                                          */
  const uint8_t *x;   /* device: codes, concatenated                        */
  const int64_t *off; /* device: start of each sequence                     */
  const int32_t *len; /* device: length of each sequence                    */
} aln_fold_batch;

typedef struct {
  int32_t score;    /* best surviving F (unpruned: F(0, n-1))                */
  int32_t i, j;     /* its interval: highest F, then the largest span, then
                       the smallest i                                       */
  int32_t full;     /* 1 when (0, n-1) was evaluated and kept               */
  int64_t cells;    /* cells evaluated with span >= 1                       */
  int64_t terms;    /* their bifurcation terms (a cell of span t has t)     */
  int32_t status;   /* ALN_R_OK, or ALN_R_BAD_SYMBOL (a code > 3)          */
  int32_t reserved;
} aln_fold_result;  /* 40 bytes */

/* Plan a folding batch from its host-side lengths: one workgroup per
 * sequence with the whole triangle in LDS (one byte per cell when every
 * score fits 0..253, else two), sequences grouped by LDS size and run
 * longest first.  Reports the workspace (the uploaded task list) in
 * fp->workspace_bytes and the unpruned cell count in fp->cells.
 * ALN_E_UNSUPPORTED when a sequence is longer than 511 nt, or longer than
 * 383 nt with scores that need two bytes (its triangle would not fit 160 KB
 * of LDS), or its scores could exceed 32767.  Destroy with
 * aln_plan_destroy. */
aln_status aln_fold_plan_create(aln_ctx *ctx, const aln_fold_params *params, int32_t n,
                                const int32_t *len_host, aln_plan **plan, aln_footprint *fp);
/* Run a folding plan on a batch with the lengths it was planned with.
 * d_ws: >= fp.workspace_bytes; d_res: n results.  Enqueues on `stream`;
 * allocates nothing. */
aln_status aln_fold_execute(aln_ctx *ctx, aln_plan *plan, const aln_fold_batch *batch,
                            void *d_ws, uint64_t ws_bytes, aln_fold_result *d_res,
                            void *stream);

/* ------------------------------------------------------------------------
 * Serving: continuous batching of single-pair requests on one device.
 *
 * A server owns a worker thread, `streams` HIP streams (default priority)
 * and one device allocation of `hbm_budget` bytes made at creation.  Each
 * submitted request is copied to host memory owned by the server.  Whenever
 * a stream is idle, the worker takes the oldest pending request whose class
 * (scoring and parameters) holds fewer than class_streams streams, together
 * with later pending requests of the same class (up to
 * max_batch_pairs pairs and max_batch_cells cells), plans them as one batch
 * (same planner and kernels as aln_execute) and admits the micro-batch once
 * the budget has a free block for its footprint: sequences + workspace
 * (traceback codes dominate) + results + CIGAR words.  Requests that arrive
 * while micro-batches run wait for the next free stream and memory;
 * micro-batches on different streams overlap on the device.  A pair's
 * result does not depend on which requests share its micro-batch.
 * Scorings must be set on the context before aln_server_create; the server
 * keeps its own device copies.  All aln_server_* calls are thread-safe.
 * ---------------------------------------------------------------------- */
typedef struct aln_server aln_server;

typedef struct {
  int32_t streams;         /* micro-batches in flight at once, 1..16          */
  int32_t max_batch_pairs; /* pairs per micro-batch, >= 1                     */
  uint64_t hbm_budget;     /* device bytes for admitted work; 0: half of the
                              free device memory at creation                 */
  int64_t max_batch_cells; /* M*N cap per micro-batch (0: none); the oldest
                              request is always taken                        */
  int32_t class_streams;   /* most streams one parameter class may hold at
                              once, so long jobs of one kind cannot starve
                              the others (0: streams / 4, at least 1)      */
  int32_t reserved;        /* 0                                              */
} aln_server_cfg;

typedef struct {
  int32_t scoring_id;   /* from aln_set_scoring, before aln_server_create     */
  aln_params params;    /* as for aln_plan_create                            */
  const uint8_t *q;     /* host memory, copied by aln_server_submit          */
  int32_t q_len;
  const uint8_t *r;
  int32_t r_len;
  uint64_t tag;         /* returned unchanged in the completion              */
} aln_request;

typedef struct {
  uint64_t id;          /* from aln_server_submit                            */
  uint64_t tag;
  aln_result result;    /* cigar_off indexes the `cigar` buffer of the poll
                           that returned this completion                     */
  int32_t error;        /* ALN_OK, or why the request was not run
                           (ALN_E_DEVICE, ALN_E_NOMEM, ALN_E_CAPACITY)       */
  int32_t batch_pairs;  /* pairs in the micro-batch that carried it          */
  uint64_t batch_id;
  double t_submit;      /* seconds on the server clock (aln_server_clock)   */
  double t_launch;      /* its micro-batch was enqueued                      */
  double t_done;        /* the worker saw the micro-batch finish             */
} aln_completion;       /* 104 bytes */

typedef struct {
  uint64_t submitted, completed, batches;
  uint64_t admission_waits;  /* times a ready micro-batch waited for memory   */
  uint64_t arena_bytes;      /* device budget in use by the server            */
  uint64_t peak_arena_bytes; /* most bytes held by micro-batches at once      */
  int64_t cells;             /* cells evaluated by completed requests         */
  int32_t peak_inflight;     /* most micro-batches on the device at once      */
  int32_t streams;
} aln_server_stats;          /* 64 bytes */

/* Create a server on ctx's device.  Errors: ALN_E_INVAL (configuration),
 * ALN_E_NOMEM (the budget cannot be reserved), ALN_E_DEVICE. */
aln_status aln_server_create(aln_ctx *ctx, const aln_server_cfg *cfg,
                             aln_server **srv);
/* Finish every submitted request, then release the server's resources.
 * Completions not yet polled are discarded. */
void aln_server_destroy(aln_server *srv);
/* Queue one pair.  The request is planned alone first: ALN_E_INVAL or
 * ALN_E_UNSUPPORTED for what aln_plan_create would reject, ALN_E_CAPACITY if
 * its footprint exceeds the whole budget.  *id receives the request id. */
aln_status aln_server_submit(aln_server *srv, const aln_request *req,
                             uint64_t *id);
/* Move up to `max` finished requests into out[], oldest first, waiting up to
 * wait_us microseconds if none is ready.  CIGAR words go to the caller's
 * host buffer cigar[0 .. cigar_cap); *cigar_used receives the words written.
 * Returns the number of completions, or ALN_E_CAPACITY if the next
 * completion's CIGAR alone does not fit in cigar_cap. */
int32_t aln_server_poll(aln_server *srv, aln_completion *out, int32_t max,
                        uint32_t *cigar, uint64_t cigar_cap,
                        uint64_t *cigar_used, int32_t wait_us);
/* Wait until every submitted request has finished (timeout_ms < 0: no limit).
 * ALN_E_CAPACITY if the time ran out. */
aln_status aln_server_drain(aln_server *srv, int32_t timeout_ms);
/* Seconds since the server was created (the clock of the completion times). */
double aln_server_clock(const aln_server *srv);
aln_status aln_server_get_stats(aln_server *srv, aln_server_stats *stats);
/* Message of the last failed call or worker error (empty string if none). */
const char *aln_server_last_error(aln_server *srv);

#ifdef __cplusplus
}
#endif
#endif
