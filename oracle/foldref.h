/*
 * foldref.h -- CPU oracle for Nussinov RNA folding with optional X-drop
 * pruning transferred from alignment.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference that the GPU
 * folding kernel is checked against.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (paper: "Compiling Bioinformatics Recurrences"):
 *   - the RNA-folding row of the example-recurrence table (Sec. 3): over a
 *     sequence x_0 .. x_{n-1},
 *         F(i,j) = max( F(i+1,j), F(i,j-1), F(i+1,j-1) + in1(i,j),
 *                       max_{i <= k < j} F(i,k) + F(k+1,j) ),
 *     F(i,i) = 0 and the empty interval F(i+1,i) = 0, evaluated one span
 *     t = j - i at a time (the triangle's wavefronts);
 *   - optionally the X-drop pruning of Sec. 7.2 transferred to it (Sec. 9.5):
 *     past a warm-up of the first spans (t <= warmup) a cell scoring more than
 *     X below the best score of the earlier wavefronts is removed, and the
 *     next wavefront is evaluated only from one position before the first
 *     survivor to the last survivor.
 *
 * Integers only; int64 arithmetic with NEG = -2^60 as minus infinity.
 */
#ifndef FOLDREF_H
#define FOLDREF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t score;  /* best surviving F                                      */
  int32_t i, j;   /* its interval (largest span, then smallest i, on ties) */
  int64_t cells;  /* cells evaluated with span t >= 1                       */
  int64_t terms;  /* bifurcation terms of those cells (span t: t terms each) */
  int32_t full;   /* 1 when the whole sequence (0, n-1) was evaluated and kept */
  int32_t status; /* 0, or -1 (bad arguments) / -2 (allocation failed)      */
} foldref_out;

/*
 * Fold x[0..n-1] (codes 0..3 = A, C, G, U).
 *   pair       4x4 pairing scores, in1(i,j) = pair[x_i*4 + x_j] when j - i >
 *              min_loop, else 0
 *   xdrop      < 0: no pruning; else the threshold X
 *   warmup     spans t <= warmup are never pruned
 * Returns the status (also in out->status).
 */
int foldref_fold(const int32_t *pair, int32_t min_loop, int32_t xdrop, int32_t warmup,
                 const uint8_t *x, int32_t n, foldref_out *out);

/* n sequences (concatenated, start offsets off[], lengths len[]) on nthreads
 * host threads.  Returns 0 or -1 / -2. */
int foldref_fold_batch(const int32_t *pair, int32_t min_loop, int32_t xdrop, int32_t warmup,
                       int32_t n, const uint8_t *x, const int64_t *off, const int32_t *len,
                       foldref_out *out, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
