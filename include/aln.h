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
enum { ALN_FULL = 0, ALN_BAND = 1, ALN_XDROP = 2 };
/* score width: AUTO lets the library choose (packed int16 where it applies,
 * with an automatic int32 re-run of any pair that could have overflowed) */
enum { ALN_W_AUTO = 0, ALN_W_I16 = 1, ALN_W_I32 = 2 };

/* per-pair result status */
enum {
  ALN_R_OK = 0,
  ALN_R_UNREACHABLE = 1, /* GLOBAL + BAND: (M,N) not connected to (0,0)      */
  ALN_R_CIGAR_CAP = 2,   /* the pair's CIGAR did not fit its slot           */
  ALN_R_BAD_SYMBOL = 3,  /* a code >= alphabet; other fields undefined       */
  ALN_R_TOO_WIDE = 4     /* XDROP: the surviving region spanned more than the
                            widest kernel window (2042 diagonals)            */
};
/* per-pair result flags */
enum {
  ALN_F_I16_RERUN = 1,  /* the int16 pass could have saturated; the pair was
                           recomputed in int32 (the result is the int32 one) */
  ALN_F_WIDENED = 2     /* X-drop region outgrew the first window; the pair
                           was recomputed with a wider one                    */
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
  int32_t prune;      /* ALN_FULL / ALN_BAND / ALN_XDROP (EXTEND only)        */
  int32_t band_w;     /* BAND half-width w >= 0                               */
  int32_t xdrop;      /* XDROP threshold X >= 0                               */
  int32_t width;      /* ALN_W_*                                              */
  int32_t want_cigar; /* 1: produce a CIGAR (FULL and BAND only)              */
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

/* ABI version of the loaded library (ALN_ABI_VERSION). */
int32_t aln_abi_version(void);

/* Create a context on HIP device `device`; the context owns scoring tables,
 * plans' staging memory, streams of the server and the autotune cache. */
aln_status aln_create(aln_ctx **ctx, int32_t device);
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
void aln_plan_destroy(aln_plan *plan);

/* Run a plan on a batch whose lengths equal those it was planned with.
 * d_ws: >= fp.workspace_bytes of device memory; d_res: n results;
 * d_cigar: >= fp.cigar_words words (may be NULL without want_cigar).
 * Enqueues everything on `stream`; allocates nothing. */
aln_status aln_execute(aln_ctx *ctx, aln_plan *plan, const aln_batch *batch,
                       void *d_ws, uint64_t ws_bytes, aln_result *d_res,
                       uint32_t *d_cigar, uint64_t cigar_words, void *stream);

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

/* Kernel timing for measurement tools.  While enabled (enable = 1), every
 * kernel launch of aln_execute is bracketed by HIP events on the launch
 * stream; aln_kernel_times() synchronises those events and returns, for each
 * kernel family, the summed milliseconds and launch count since the last
 * call (then resets).  names[k] receives a static string.  Returns the number
 * of families written (<= max).  Not for use during graph capture. */
aln_status aln_set_profiling(aln_ctx *ctx, int32_t enable);
int32_t aln_kernel_times(aln_ctx *ctx, const char **names, double *ms,
                         int64_t *launches, int32_t max);

#ifdef __cplusplus
}
#endif
#endif
