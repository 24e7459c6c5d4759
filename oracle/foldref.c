/*
 * foldref.c -- CPU oracle for Nussinov RNA folding, unpruned or with X-drop
 * pruning transferred from alignment.
 *
 * TEST INFRASTRUCTURE ONLY (see foldref.h).  A plain n x n int64 table,
 * filled one span t = j - i at a time; no blocking, no vectorisation.
 *
 * Recurrence (Sec. 3, RNA-folding row of the example-recurrence table), for
 * 0 <= i < j < n:
 *     F(i,j) = max( F(i+1,j), F(i,j-1), F(i+1,j-1) + in1(i,j),
 *                   max over i <= k < j of F(i,k) + F(k+1,j) )
 * with F(i,i) = 0 and the empty interval F(i+1,i) = 0.  in1(i,j) is the
 * pairing score of x_i with x_j when j - i > min_loop, else 0.
 *
 * Every term of the recurrence reads an interval strictly shorter than
 * (i,j), so the cells of one span t are independent: they form the
 * wavefronts the table is traversed by (with the rows flipped, i' = n-1-i,
 * a cell depends on (i'-1,j), (i',j-1), (i'-1,j-1) exactly like an alignment
 * cell, and span t is its antidiagonal).
 *
 * X-drop transferred to it (Sec. 9.5 with the rule of Sec. 7.2), wavefront by
 * wavefront, positions p = i along wavefront t:
 *   1. t = 0: F(i,i) = 0 for every i; best = 0; survivors [lo, hi] = [0, n-1].
 *   2. t >= 1: candidates p in [lo - 1, hi] intersected with [0, n-1-t] (a
 *      cell at position p reads positions p and p+1 of wavefront t-1, so
 *      the region can widen by one position to the left per wavefront);
 *      when that range is empty the fold stops.
 *   3. Evaluate each candidate by the recurrence; a term that reads a cell
 *      never evaluated or pruned reads minus infinity.
 *   4. Prune (t > warmup only): a candidate whose value falls more than X
 *      below `best`, the best score of wavefronts 0 .. t-1, reads minus
 *      infinity from then on.
 *   5. best = max(best, survivors' values); [lo, hi] = first and last
 *      surviving positions; if none survives the fold stops.
 * The result is the best surviving cell: highest F, then the largest span,
 * then the smallest i (so an unpruned fold reports F(0, n-1) on (0, n-1)).
 */
#include "foldref.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define NEG (-(((int64_t)1) << 60))

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

int foldref_fold(const int32_t *pair, int32_t min_loop, int32_t xdrop, int32_t warmup,
                 const uint8_t *x, int32_t n, foldref_out *out) {
  if (!out) return -1;
  memset(out, 0, sizeof(*out));
  if (!pair || n < 0 || (n > 0 && !x) || min_loop < 0 || warmup < 0) {
    out->status = -1;
    return -1;
  }
  if (n == 0) return 0;
  for (int32_t p = 0; p < n; p++)
    if (x[p] > 3) {
      out->status = -1;
      return -1;
    }
  /* F[i*n + j] for i <= j; `alive` marks evaluated, unpruned cells */
  int64_t *F = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (size_t)n);
  uint8_t *alive = (uint8_t *)calloc((size_t)n * (size_t)n, 1);
  if (!F || !alive) {
    free(F);
    free(alive);
    out->status = -2;
    return -2;
  }
  /* value of interval (a, b): the empty interval (b = a - 1) is 0 */
#define VAL(a, b) ((b) < (a) ? (int64_t)0 : (alive[(size_t)(a) * n + (b)] ? F[(size_t)(a) * n + (b)] : NEG))
  for (int32_t i = 0; i < n; i++) {
    F[(size_t)i * n + i] = 0;
    alive[(size_t)i * n + i] = 1;
  }
  int64_t best = 0;
  int32_t bi = 0, bj = 0; /* best cell so far: F = 0 at the largest span 0, smallest i */
  int32_t lo = 0, hi = n - 1;
  int64_t cells = 0, terms = 0;
  for (int32_t t = 1; t < n; t++) {
    int32_t a = lo - 1, b = hi;
    if (a < 0) a = 0;
    if (b > n - 1 - t) b = n - 1 - t;
    if (a > b) break;
    const int prune = xdrop >= 0 && t > warmup;
    int32_t nlo = -1, nhi = -1;
    int64_t wbest = NEG;
    int32_t wi = 0;
    for (int32_t i = a; i <= b; i++) {
      const int32_t j = i + t;
      int64_t v = NEG;
      const int64_t down = VAL(i + 1, j), left = VAL(i, j - 1), inner = VAL(i + 1, j - 1);
      v = max2(v, down);
      v = max2(v, left);
      if (inner > NEG) {
        const int64_t s = (j - i > min_loop) ? (int64_t)pair[x[i] * 4 + x[j]] : 0;
        v = max2(v, inner + s);
      }
      for (int32_t k = i; k < j; k++) {
        const int64_t l = VAL(i, k), r = VAL(k + 1, j);
        if (l > NEG && r > NEG) v = max2(v, l + r);
      }
      cells++;
      terms += t;
      int keep = v > NEG;
      if (keep && prune && best - v > (int64_t)xdrop) keep = 0;
      F[(size_t)i * n + j] = v;
      alive[(size_t)i * n + j] = (uint8_t)keep;
      if (keep) {
        if (nlo < 0) nlo = i;
        nhi = i;
        if (v > wbest) { /* strict: the smallest i of this wavefront wins ties */
          wbest = v;
          wi = i;
        }
      }
    }
    if (nlo < 0) break;
    /* a later wavefront has the larger span, so it wins ties with the best */
    if (wbest >= best) {
      best = wbest;
      bi = wi;
      bj = wi + t;
    }
    lo = nlo;
    hi = nhi;
  }
#undef VAL
  out->score = best;
  out->i = bi;
  out->j = bj;
  out->cells = cells;
  out->terms = terms;
  out->full = (n == 1) || alive[(size_t)0 * n + (n - 1)];
  free(F);
  free(alive);
  return 0;
}

typedef struct {
  const int32_t *pair;
  int32_t min_loop, xdrop, warmup, n;
  const uint8_t *x;
  const int64_t *off;
  const int32_t *len;
  foldref_out *out;
  int32_t next;
  pthread_mutex_t mu;
} fold_job;

static void *fold_worker(void *arg) {
  fold_job *b = (fold_job *)arg;
  for (;;) {
    pthread_mutex_lock(&b->mu);
    const int32_t p = b->next++;
    pthread_mutex_unlock(&b->mu);
    if (p >= b->n) break;
    foldref_fold(b->pair, b->min_loop, b->xdrop, b->warmup, b->x + b->off[p], b->len[p],
                 &b->out[p]);
  }
  return NULL;
}

int foldref_fold_batch(const int32_t *pair, int32_t min_loop, int32_t xdrop, int32_t warmup,
                       int32_t n, const uint8_t *x, const int64_t *off, const int32_t *len,
                       foldref_out *out, int32_t nthreads) {
  if (n < 0 || !out || (n > 0 && (!off || !len))) return -1;
  if (nthreads < 1) nthreads = 1;
  fold_job b;
  b.pair = pair;
  b.min_loop = min_loop;
  b.xdrop = xdrop;
  b.warmup = warmup;
  b.n = n;
  b.x = x;
  b.off = off;
  b.len = len;
  b.out = out;
  b.next = 0;
  pthread_mutex_init(&b.mu, NULL);
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  if (!th) {
    pthread_mutex_destroy(&b.mu);
    return -2;
  }
  int started = 0;
  for (int t = 0; t < nthreads; t++)
    if (pthread_create(&th[t], NULL, fold_worker, &b) == 0)
      started++;
    else
      break;
  if (started == 0) fold_worker(&b);
  for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&b.mu);
  return 0;
}
