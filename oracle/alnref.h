/*
 * alnref.h -- CPU oracle for affine-gap (Gotoh H/E/F) pairwise alignment.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU path is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (paper: "Compiling Bioinformatics Recurrences"):
 *   - the alignment recurrence of Sec. 3 (sequence-alignment row of the
 *     example-recurrence table: three coupled arrays), written in Gotoh's
 *     H/E/F form with gap cost  open + L*extend  for a gap of length L;
 *   - over the full matrix, a static band (Sec. 7.1, prune axis
 *     -B <= diag(i,j) <= B, centred on the rectangle's diagonal when M != N),
 *     or X-drop dynamic pruning (Sec. 2, Sec. 5.2, Sec. 7.2) evaluated one
 *     antidiagonal k = i + j at a time (Sec. 6.2 shearing);
 *   - score, end cell, cells evaluated and (optionally) a CIGAR traceback.
 *
 * Integers only; all arithmetic in int64 with NEG = -2^60 as minus infinity.
 */
#ifndef ALNREF_H
#define ALNREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ALNREF_GLOBAL = 0, ALNREF_LOCAL = 1, ALNREF_EXTEND = 2 };
enum { ALNREF_FULL = 0, ALNREF_BAND = 1, ALNREF_XDROP = 2, ALNREF_ZDROP = 3 };

/* per-pair status */
enum {
  ALNREF_OK = 0,
  ALNREF_UNREACHABLE = 1, /* GLOBAL end cell (M,N) pruned away by the band */
  ALNREF_CIGAR_CAP = 2,   /* CIGAR longer than the caller's capacity        */
  ALNREF_BAD_SYMBOL = 3,  /* a code >= alphabet                              */
  ALNREF_INVAL = -1,      /* bad arguments                                   */
  ALNREF_NOMEM = -2       /* host allocation failed                          */
};

/* CIGAR word: (run_length << 4) | op, SAM op codes */
enum { ALNREF_OP_I = 1, ALNREF_OP_D = 2, ALNREF_OP_EQ = 7, ALNREF_OP_X = 8 };

typedef struct {
  int64_t score;    /* INT32_MIN when status == ALNREF_UNREACHABLE           */
  int32_t q_end;    /* end cell as prefix lengths (i = query, j = reference) */
  int32_t r_end;
  int32_t q_begin;  /* start cell of the traceback (LOCAL: first aligned-1)  */
  int32_t r_begin;
  int64_t cells;    /* interior cells (i>=1, j>=1) evaluated                  */
  int32_t status;
  int32_t cigar_len;/* number of CIGAR words written                         */
  int32_t span;     /* XDROP / ZDROP: widest candidate range, in diagonals
                       (2 * (last j - first j)), of antidiagonals 1 .. the end
                       cell's (q_end + r_end); 0 otherwise                   */
  int32_t reserved;
} alnref_out;

/*
 * Align query q (rows i = 1..M) against reference r (columns j = 1..N).
 *   matrix     alphabet*alphabet substitution scores, s(a,b) = matrix[a*alphabet+b]
 *              with a a query code and b a reference code
 *   gap_open, gap_extend   <= 0; a gap of length L scores gap_open + L*gap_extend
 *   mode       ALNREF_GLOBAL / LOCAL / EXTEND
 *   prune      ALNREF_FULL / BAND (band_w >= 0) / XDROP or ZDROP (threshold X or Z in
 *              xdrop >= 0, EXTEND only)
 *   cigar      NULL for score only; else room for cigar_cap words (XDROP / ZDROP:
 *              the path from the end cell back to (0,0) through evaluated,
 *              unpruned cells, chosen by the same preference order)
 * Returns the status (also stored in out->status).
 */
int alnref_align(const int32_t *matrix, int32_t alphabet, int32_t gap_open,
                 int32_t gap_extend, int32_t mode, int32_t prune,
                 int32_t band_w, int32_t xdrop, const uint8_t *q, int32_t M,
                 const uint8_t *r, int32_t N, uint32_t *cigar,
                 int32_t cigar_cap, alnref_out *out);

/*
 * Batch driver: n independent pairs over nthreads host threads (one pair per
 * task).  Sequences are concatenated; q_off/r_off are start offsets.  When
 * cigar != NULL pair p writes at cigar + cigar_off[p] with room cigar_cap[p].
 * Returns 0, or ALNREF_INVAL / ALNREF_NOMEM for a bad call.
 */
int alnref_align_batch(const int32_t *matrix, int32_t alphabet,
                       int32_t gap_open, int32_t gap_extend, int32_t mode,
                       int32_t prune, int32_t band_w, int32_t xdrop, int32_t n,
                       const uint8_t *q, const int64_t *q_off,
                       const int32_t *q_len, const uint8_t *r,
                       const int64_t *r_off, const int32_t *r_len,
                       uint32_t *cigar, const int64_t *cigar_off,
                       const int32_t *cigar_cap, alnref_out *out,
                       int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
