/* Host-only run of the CPU oracle (oracle/alnref.c, oracle/foldref.c) under
 * AddressSanitizer and UndefinedBehaviorSanitizer: random pairs of every
 * shape class (empty, one-letter, skewed, equal), every mode and pruning
 * rule, with and without CIGAR (and with a CIGAR slot one word too small),
 * bad symbols, the batch driver on several threads against single calls,
 * and folds of random sequences with and without X-drop.  Prints OK. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "alnref.h"
#include "foldref.h"

static uint64_t rng_state;
static uint64_t next64(void) { /* SplitMix64 */
  uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static int rnd(int n) { return n > 0 ? (int)(next64() % (uint64_t)n) : 0; }

static int fail(const char *what, int a, int b) {
  printf("FAIL %s %d %d\n", what, a, b);
  return 1;
}

int main(int argc, char **argv) {
  rng_state = argc > 1 ? (uint64_t)atoll(argv[1]) : 1u;
  enum { NP = 40 };
  for (int round = 0; round < 24; ++round) {
    const int A = round % 3 == 0 ? 20 : 4;
    int32_t mat[400];
    for (int a = 0; a < A; ++a)
      for (int b = 0; b < A; ++b) mat[a * A + b] = a == b ? 1 + rnd(5) : -1 - rnd(4);
    const int go = -rnd(6), ge = -1 - rnd(3);
    const int mode = round % 3, prune = mode == 2 ? round % 4 : round % 2;
    const int band_w = rnd(40), xdrop = rnd(60);
    int32_t ql[NP], rl[NP];
    int64_t qo[NP], ro[NP], co[NP];
    int32_t cap[NP];
    int64_t tq = 0, tr = 0, tc = 0;
    for (int p = 0; p < NP; ++p) {
      const int cls = rnd(5);
      ql[p] = cls == 0 ? 0 : cls == 1 ? 1 : rnd(300);
      rl[p] = cls == 0 ? rnd(3) : cls == 2 ? 1 : rnd(300);
      qo[p] = tq;
      ro[p] = tr;
      co[p] = tc;
      cap[p] = ql[p] + rl[p] + 1 - (p % 7 == 6); /* some slots one word short */
      if (cap[p] < 0) cap[p] = 0;
      tq += ql[p];
      tr += rl[p];
      tc += cap[p];
    }
    uint8_t *q = malloc((size_t)tq + 1), *r = malloc((size_t)tr + 1);
    for (int64_t k = 0; k < tq; ++k) q[k] = (uint8_t)rnd(A);
    for (int64_t k = 0; k < tr; ++k) r[k] = (uint8_t)rnd(A);
    if (tq > 5 && round % 5 == 4) q[tq / 2] = (uint8_t)A; /* a bad symbol */
    for (int p = 1; p < NP; p += 3) /* related pairs */
      for (int k = 0; k < ql[p] && k < rl[p]; ++k)
        if (rnd(10)) q[qo[p] + k] = r[ro[p] + k];
    uint32_t *cig = malloc(sizeof(uint32_t) * (size_t)(tc + 1));
    uint32_t *cig1 = malloc(sizeof(uint32_t) * (size_t)(tc + 1));
    alnref_out out[NP], one;
    for (int want = 0; want < 2; ++want) {
      if (alnref_align_batch(mat, A, go, ge, mode, prune, band_w, xdrop, NP, q, qo, ql, r, ro, rl,
                             want ? cig : NULL, want ? co : NULL, want ? cap : NULL, out, 3) < 0)
        return fail("batch", round, want);
      for (int p = 0; p < NP; ++p) {
        if (alnref_align(mat, A, go, ge, mode, prune, band_w, xdrop, q + qo[p], ql[p], r + ro[p],
                         rl[p], want ? cig1 + co[p] : NULL, want ? cap[p] : 0, &one) < 0)
          return fail("single", round, p);
        if (one.score != out[p].score || one.cells != out[p].cells ||
            one.status != out[p].status || one.cigar_len != out[p].cigar_len)
          return fail("batch differs from single", round, p);
        if (want && memcmp(cig + co[p], cig1 + co[p], sizeof(uint32_t) * (size_t)one.cigar_len))
          return fail("cigar differs", round, p);
      }
    }
    free(q);
    free(r);
    free(cig);
    free(cig1);
  }
  /* folding */
  int32_t pair[16] = {0};
  pair[0 * 4 + 3] = pair[3 * 4 + 0] = 1;
  pair[1 * 4 + 2] = pair[2 * 4 + 1] = 1;
  pair[2 * 4 + 3] = pair[3 * 4 + 2] = 1;
  for (int round = 0; round < 60; ++round) {
    const int n = round < 4 ? round : rnd(260);
    uint8_t *x = malloc((size_t)n + 1);
    for (int k = 0; k < n; ++k) x[k] = (uint8_t)rnd(4);
    foldref_out a, b;
    if (foldref_fold(pair, round % 4, -1, 15, x, n, &a) != 0) return fail("fold", round, n);
    if (foldref_fold(pair, round % 4, rnd(5), rnd(20), x, n, &b) != 0)
      return fail("fold xdrop", round, n);
    if (b.score > a.score || b.cells > a.cells) return fail("pruned fold above unpruned", round, n);
    if (n > 2) {
      x[n / 2] = 7;
      if (foldref_fold(pair, 0, -1, 15, x, n, &a) != -1) return fail("bad code accepted", round, n);
    }
    free(x);
  }
  printf("OK\n");
  return 0;
}
