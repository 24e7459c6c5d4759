/*
 * alnref.c -- CPU oracle for affine-gap (Gotoh H/E/F) pairwise alignment.
 *
 * TEST INFRASTRUCTURE ONLY (see alnref.h).  Plain row-major dynamic
 * programming in int64; no blocking, no vectorisation, no reordering beyond
 * what the definitions below state.
 *
 * Notation follows the paper's problem statement (Sec. 2): the query q lies
 * on the vertical axis with rows i = 1..M, the reference r on the horizontal
 * axis with columns j = 1..N; cell (i,j) scores the prefixes q[1..i], r[1..j].
 *
 * Recurrence (Sec. 3, sequence-alignment row of the example-recurrence table:
 * a match array plus two gap arrays coupled through max).  It is written here
 * in Gotoh's H/E/F form, with a gap of length L costing  o + L*e  (o = open,
 * e = extend, both <= 0):
 *     E(i,j) = max(E(i,j-1) + e, H(i,j-1) + o + e)     horizontal move (D)
 *     F(i,j) = max(F(i-1,j) + e, H(i-1,j) + o + e)     vertical move   (I)
 *     H(i,j) = max(H(i-1,j-1) + s(q_i, r_j), E(i,j), F(i,j))
 * LOCAL adds 0 to the H max (Smith-Waterman).
 *
 * Base cases are index conditions (Sec. 5.2, conditional definitions):
 *     GLOBAL/EXTEND: H(0,0)=0; H(0,j)=E(0,j)=o+j*e, F(0,j)=NEG (j>=1);
 *                    H(i,0)=F(i,0)=o+i*e, E(i,0)=NEG (i>=1)
 *     LOCAL:         H(0,j)=H(i,0)=0; E and F on the boundary = NEG.
 *
 * Pruning (Sec. 7):
 *   FULL   every cell 0<=i<=M, 0<=j<=N.
 *   BAND   static prune axis (Sec. 7.1): row i keeps c(i)-w <= j <= c(i)+w with
 *          c(i) = floor(i*N/M); for M = N this is exactly -w <= diag(i,j) <= w.
 *          Out-of-band cells (boundary cells included) are NEG.
 *   XDROP  dynamic pruning evaluated antidiagonal by antidiagonal (Sec. 2,
 *          Sec. 5.2, Sec. 6.2, Sec. 7.2): a cell whose H falls more than X
 *          below the best score of the antidiagonals before it is set to
 *          NEG, and the next antidiagonal is evaluated only between the first
 *          and last surviving cells (plus one step right).
 *   ZDROP  the same antidiagonal procedure with the Z-drop condition of
 *          Sec. 9.3 (named in Sec. 7.2): a cell is set to NEG when the best
 *          score of the antidiagonals before it exceeds its H by more than
 *          Z + |diag(i,j) - diag_best|, diag = j - i, diag_best the diagonal
 *          of that best cell.
 */
#include "alnref.h"

#include <limits.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define NEG (-(((int64_t)1) << 60))
#define IS_NEG(v) ((v) <= NEG / 2)

static int64_t max2(int64_t a, int64_t b) { return a > b ? a : b; }

/* ------------------------------------------------------------------ */
/* Row-range storage: row i holds columns lo[i]..hi[i]; the rest read NEG. */
/* FULL uses lo = 0, hi = N for every row.                                  */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t M, N;
  int32_t *lo, *hi;
  int64_t *off;     /* start of row i in the value arrays */
  int64_t *H, *E, *F;
} rowstore;

static void rs_free(rowstore *s) {
  free(s->lo); free(s->hi); free(s->off);
  free(s->H); free(s->E); free(s->F);
}

/* band centre for row i: floor(i*N/M) */
static int64_t band_centre(int64_t i, int32_t M, int32_t N) {
  return (i * (int64_t)N) / (int64_t)M;
}

static int rs_alloc(rowstore *s, int32_t M, int32_t N, int band, int32_t w) {
  memset(s, 0, sizeof(*s));
  s->M = M; s->N = N;
  s->lo = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
  s->hi = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
  s->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(M + 2));
  if (!s->lo || !s->hi || !s->off) { rs_free(s); return -1; }
  int64_t total = 0;
  for (int32_t i = 0; i <= M; i++) {
    int64_t lo = 0, hi = N;
    if (band && M > 0) {
      int64_t c = band_centre(i, M, N);
      lo = c - w; hi = c + w;
      if (lo < 0) lo = 0;
      if (hi > N) hi = N;
    }
    s->lo[i] = (int32_t)lo;
    s->hi[i] = (int32_t)hi;
    s->off[i] = total;
    if (hi >= lo) total += hi - lo + 1;
  }
  s->off[M + 1] = total;
  size_t bytes = sizeof(int64_t) * (size_t)(total > 0 ? total : 1);
  s->H = (int64_t *)malloc(bytes);
  s->E = (int64_t *)malloc(bytes);
  s->F = (int64_t *)malloc(bytes);
  if (!s->H || !s->E || !s->F) { rs_free(s); return -1; }
  return 0;
}

static int rs_in(const rowstore *s, int64_t i, int64_t j) {
  if (i < 0 || i > s->M || j < 0 || j > s->N) return 0;
  return j >= s->lo[i] && j <= s->hi[i];
}

static int64_t rs_get(const rowstore *s, const int64_t *A, int64_t i, int64_t j) {
  if (!rs_in(s, i, j)) return NEG;
  return A[s->off[i] + (j - s->lo[i])];
}

static void rs_set(rowstore *s, int64_t *A, int64_t i, int64_t j, int64_t v) {
  A[s->off[i] + (j - s->lo[i])] = v;
}

/* end-cell order: higher score first, then smaller i, then smaller j */
static int better(int64_t sc, int64_t i, int64_t j, int64_t bsc, int64_t bi,
                  int64_t bj) {
  if (sc != bsc) return sc > bsc;
  if (i != bi) return i < bi;
  return j < bj;
}

/* ------------------------------------------------------------------ */
/* CIGAR assembly: ops are produced end->start, emitted start->end.     */
/* ------------------------------------------------------------------ */
typedef struct {
  uint8_t *ops; /* reversed op sequence */
  int64_t n, cap;
} opbuf;

static int ob_push(opbuf *b, uint8_t op) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? b->cap * 2 : 256;
    uint8_t *p = (uint8_t *)realloc(b->ops, (size_t)nc);
    if (!p) return -1;
    b->ops = p; b->cap = nc;
  }
  b->ops[b->n++] = op;
  return 0;
}

/* run-length encode the forward op sequence; returns words or -1 on overflow */
static int32_t ob_emit(const opbuf *b, uint32_t *cigar, int32_t cap) {
  int32_t w = 0;
  int64_t k = b->n - 1;
  while (k >= 0) {
    uint8_t op = b->ops[k];
    uint32_t run = 0;
    while (k >= 0 && b->ops[k] == op) { run++; k--; }
    if (w >= cap) return -1;
    cigar[w++] = (run << 4) | op;
  }
  return w;
}

/* ------------------------------------------------------------------ */
/* Traceback (Sec. 2: the optimal path through the matrix), shared by the  */
/* row-major fill and the antidiagonal X-drop / Z-drop fill.  get(ctx, w,  */
/* i, j) returns H (w = 0), E (w = 1) or F (w = 2) of a stored cell and    */
/* NEG for any cell that was not evaluated or was pruned.  In each state   */
/* the first option whose equality holds is taken:                         */
/*   H: (LOCAL and H == 0 -> stop), diagonal, then E, then F;              */
/*   E/F: open (from H) before extend;                                     */
/* on row 0 the path runs left (D) and on column 0 up (I) to (0,0).        */
/* ------------------------------------------------------------------ */
typedef int64_t (*cell_get)(const void *ctx, int which, int64_t i, int64_t j);

static int traceback(cell_get get, const void *ctx, const int32_t *mat, int32_t A, int64_t o,
                     int64_t e, int local, const uint8_t *q, const uint8_t *r, int64_t ei,
                     int64_t ej, uint32_t *cigar, int32_t cigar_cap, alnref_out *out) {
  opbuf ob = {0, 0, 0};
  int64_t i = ei, j = ej;
  int state = 0; /* 0 = H, 1 = E, 2 = F */
  int rc = 0;
  for (;;) {
    if (state == 0) {
      if (i == 0 && j == 0) break;
      int64_t hv = get(ctx, 0, i, j);
      if (local && hv == 0) break;
      if (i == 0) { rc |= ob_push(&ob, ALNREF_OP_D); j--; continue; }
      if (j == 0) { rc |= ob_push(&ob, ALNREF_OP_I); i--; continue; }
      int64_t sub = mat[(int64_t)q[i - 1] * A + r[j - 1]];
      int64_t hd = get(ctx, 0, i - 1, j - 1);
      if (!IS_NEG(hd) && hv == hd + sub) {
        rc |= ob_push(&ob, q[i - 1] == r[j - 1] ? ALNREF_OP_EQ : ALNREF_OP_X);
        i--; j--;
      } else if (hv == get(ctx, 1, i, j)) {
        state = 1;
      } else {
        state = 2;
      }
    } else if (state == 1) {
      rc |= ob_push(&ob, ALNREF_OP_D);
      int64_t ev = get(ctx, 1, i, j);
      int64_t hl = get(ctx, 0, i, j - 1);
      if (!IS_NEG(hl) && ev == hl + o + e) state = 0;
      j--;
    } else {
      rc |= ob_push(&ob, ALNREF_OP_I);
      int64_t fv = get(ctx, 2, i, j);
      int64_t hu = get(ctx, 0, i - 1, j);
      if (!IS_NEG(hu) && fv == hu + o + e) state = 0;
      i--;
    }
    if (rc) break;
  }
  if (rc) { free(ob.ops); return ALNREF_NOMEM; }
  out->q_begin = (int32_t)i;
  out->r_begin = (int32_t)j;
  int32_t nw = ob_emit(&ob, cigar, cigar_cap);
  free(ob.ops);
  if (nw < 0) {
    out->cigar_len = 0;
    out->status = ALNREF_CIGAR_CAP;
    return ALNREF_CIGAR_CAP;
  }
  out->cigar_len = nw;
  return ALNREF_OK;
}

static int64_t rows_get(const void *ctx, int which, int64_t i, int64_t j) {
  const rowstore *s = (const rowstore *)ctx;
  return rs_get(s, which == 0 ? s->H : (which == 1 ? s->E : s->F), i, j);
}

/* ------------------------------------------------------------------ */
/* FULL and BAND: row-major fill of the whole (or banded) matrix.        */
/* ------------------------------------------------------------------ */
static int align_rows(const int32_t *mat, int32_t A, int64_t o, int64_t e,
                      int32_t mode, int band, int32_t w, const uint8_t *q,
                      int32_t M, const uint8_t *r, int32_t N, uint32_t *cigar,
                      int32_t cigar_cap, alnref_out *out) {
  rowstore s;
  if (rs_alloc(&s, M, N, band, w) != 0) return ALNREF_NOMEM;
  const int local = (mode == ALNREF_LOCAL);

  int64_t best = NEG, bi = 0, bj = 0;
  int64_t cells = 0;
  for (int64_t i = 0; i <= M; i++) {
    for (int64_t j = s.lo[i]; j <= s.hi[i]; j++) {
      int64_t h, ev, fv;
      if (i == 0 && j == 0) {
        h = 0; ev = NEG; fv = NEG;
      } else if (i == 0) {
        if (local) { h = 0; ev = NEG; }
        else { h = o + j * e; ev = h; }
        fv = NEG;
      } else if (j == 0) {
        if (local) { h = 0; fv = NEG; }
        else { h = o + i * e; fv = h; }
        ev = NEG;
      } else {
        int64_t sub = mat[(int64_t)q[i - 1] * A + r[j - 1]];
        ev = max2(rs_get(&s, s.E, i, j - 1) + e, rs_get(&s, s.H, i, j - 1) + o + e);
        fv = max2(rs_get(&s, s.F, i - 1, j) + e, rs_get(&s, s.H, i - 1, j) + o + e);
        h = max2(rs_get(&s, s.H, i - 1, j - 1) + sub, max2(ev, fv));
        if (local) h = max2(h, 0);
        cells++;
      }
      /* keep minus infinity pinned so that it can never drift upwards */
      if (IS_NEG(h)) h = NEG;
      if (IS_NEG(ev)) ev = NEG;
      if (IS_NEG(fv)) fv = NEG;
      rs_set(&s, s.H, i, j, h);
      rs_set(&s, s.E, i, j, ev);
      rs_set(&s, s.F, i, j, fv);
      if (mode != ALNREF_GLOBAL && !IS_NEG(h) && better(h, i, j, best, bi, bj)) {
        best = h; bi = i; bj = j;
      }
    }
  }

  out->cells = cells;
  int64_t ei, ej;
  if (mode == ALNREF_GLOBAL) {
    ei = M; ej = N;
    int64_t hv = rs_get(&s, s.H, M, N);
    if (IS_NEG(hv)) {
      out->score = INT32_MIN;
      out->q_end = M; out->r_end = N;
      out->q_begin = 0; out->r_begin = 0;
      out->status = ALNREF_UNREACHABLE;
      rs_free(&s);
      return ALNREF_UNREACHABLE;
    }
    out->score = hv;
  } else {
    ei = bi; ej = bj;
    out->score = best;
  }
  out->q_end = (int32_t)ei;
  out->r_end = (int32_t)ej;
  out->q_begin = 0;
  out->r_begin = 0;

  if (cigar) {
    int rc = traceback(rows_get, &s, mat, A, o, e, local, q, r, ei, ej, cigar, cigar_cap, out);
    if (rc != ALNREF_OK) {
      rs_free(&s);
      return rc;
    }
  }
  rs_free(&s);
  out->status = ALNREF_OK;
  return ALNREF_OK;
}

/* ------------------------------------------------------------------ */
/* XDROP (EXTEND only): antidiagonal k = i + j, position m = j (Sec. 6.2). */
/* Three antidiagonal buffers indexed by j hold k, k-1 and k-2; entries   */
/* outside an antidiagonal's candidate range, or pruned, read NEG.         */
/* ------------------------------------------------------------------ */
typedef struct {
  int64_t *H, *E, *F;
  int64_t lo, hi; /* candidate range of this antidiagonal (lo > hi: none) */
} adiag;

static int64_t ad_get(const adiag *a, const int64_t *A, int64_t j) {
  if (j < a->lo || j > a->hi) return NEG;
  return A[j];
}

/* Every antidiagonal kept for the traceback: antidiagonal k holds the
 * candidates lo[k]..hi[k] (in j) at off[k] in the value arrays; cells outside
 * them, pruned cells and antidiagonals after the last one read NEG. */
typedef struct {
  int64_t nk;              /* antidiagonals stored: 0 .. nk-1 */
  int64_t *lo, *hi, *off;  /* per antidiagonal, room for M+N+1 */
  int64_t *H, *E, *F;
  int64_t used, cap;
} adstore;

static void as_free(adstore *s) {
  free(s->lo); free(s->hi); free(s->off); free(s->H); free(s->E); free(s->F);
}

static int as_push(adstore *s, const adiag *a, int64_t k) {
  int64_t n = a->hi >= a->lo ? a->hi - a->lo + 1 : 0;
  if (s->used + n > s->cap) {
    int64_t nc = s->cap ? s->cap : 1024;
    while (nc < s->used + n) nc *= 2;
    int64_t *h = (int64_t *)realloc(s->H, sizeof(int64_t) * (size_t)nc);
    if (h) s->H = h;
    int64_t *e2 = (int64_t *)realloc(s->E, sizeof(int64_t) * (size_t)nc);
    if (e2) s->E = e2;
    int64_t *f = (int64_t *)realloc(s->F, sizeof(int64_t) * (size_t)nc);
    if (f) s->F = f;
    if (!h || !e2 || !f) return -1;
    s->cap = nc;
  }
  s->lo[k] = a->lo; s->hi[k] = a->hi; s->off[k] = s->used;
  for (int64_t j = a->lo; j <= a->hi; j++) {
    s->H[s->used + j - a->lo] = a->H[j];
    s->E[s->used + j - a->lo] = a->E[j];
    s->F[s->used + j - a->lo] = a->F[j];
  }
  s->used += n;
  s->nk = k + 1;
  return 0;
}

static int64_t xs_get(const void *ctx, int which, int64_t i, int64_t j) {
  const adstore *s = (const adstore *)ctx;
  int64_t k = i + j;
  if (i < 0 || j < 0 || k >= s->nk || j < s->lo[k] || j > s->hi[k]) return NEG;
  const int64_t *A = which == 0 ? s->H : (which == 1 ? s->E : s->F);
  return A[s->off[k] + j - s->lo[k]];
}

/* zdrop = 0: X-drop with threshold X; zdrop = 1: Z-drop with Z = X. */
static int align_xdrop(const int32_t *mat, int32_t Al, int64_t o, int64_t e,
                       int64_t X, int zdrop, const uint8_t *q, int32_t M,
                       const uint8_t *r, int32_t N, uint32_t *cigar,
                       int32_t cigar_cap, alnref_out *out) {
  adstore st;
  memset(&st, 0, sizeof(st));
  if (cigar) {
    st.lo = (int64_t *)malloc(sizeof(int64_t) * (size_t)(M + N + 1));
    st.hi = (int64_t *)malloc(sizeof(int64_t) * (size_t)(M + N + 1));
    st.off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(M + N + 1));
    if (!st.lo || !st.hi || !st.off) { as_free(&st); return ALNREF_NOMEM; }
  }
  adiag buf[3];
  for (int t = 0; t < 3; t++) {
    buf[t].H = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    buf[t].E = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    buf[t].F = (int64_t *)malloc(sizeof(int64_t) * (size_t)(N + 1));
    buf[t].lo = 1; buf[t].hi = 0;
    if (!buf[t].H || !buf[t].E || !buf[t].F) {
      for (int u = 0; u <= t; u++) { free(buf[u].H); free(buf[u].E); free(buf[u].F); }
      as_free(&st);
      return ALNREF_NOMEM;
    }
  }
  /* k = 0: the single cell (0,0) */
  adiag *cur = &buf[0], *p1 = &buf[1], *p2 = &buf[2];
  cur->lo = 0; cur->hi = 0;
  cur->H[0] = 0; cur->E[0] = NEG; cur->F[0] = NEG;
  int rc = 0;
  if (cigar) rc |= as_push(&st, cur, 0);
  int64_t best = 0, bi = 0, bj = 0; /* best_{k-1}: running max through k-1 */
  int64_t lo = 0, hi = 0;           /* surviving range of the last antidiagonal */
  int64_t cells = 0;
  /* widest candidate range so far, in diagonals (d = 2j - k spans 2(hi-lo)),
   * and its value when the best cell was last found */
  int64_t span = 0, best_span = 0;

  for (int64_t k = 1; k <= (int64_t)M + N; k++) {
    adiag *t = p2; p2 = p1; p1 = cur; cur = t; /* rotate: cur <- k */
    int64_t clo = lo > k - M ? lo : k - M;
    int64_t chi = hi + 1;
    if (chi > k) chi = k;
    if (chi > N) chi = N;
    if (clo > chi) break;
    cur->lo = clo; cur->hi = chi;
    if (2 * (chi - clo) > span) span = 2 * (chi - clo);
    int64_t nlo = -1, nhi = -1;
    int64_t kbest = NEG, kbi = 0, kbj = 0;
    for (int64_t j = clo; j <= chi; j++) {
      int64_t i = k - j;
      int64_t h, ev, fv;
      if (i == 0) {
        h = o + j * e; ev = h; fv = NEG;
      } else if (j == 0) {
        h = o + i * e; fv = h; ev = NEG;
      } else {
        int64_t sub = mat[(int64_t)q[i - 1] * Al + r[j - 1]];
        ev = max2(ad_get(p1, p1->E, j - 1) + e, ad_get(p1, p1->H, j - 1) + o + e);
        fv = max2(ad_get(p1, p1->F, j) + e, ad_get(p1, p1->H, j) + o + e);
        h = max2(ad_get(p2, p2->H, j - 1) + sub, max2(ev, fv));
        cells++;
      }
      if (IS_NEG(h)) h = NEG;
      if (IS_NEG(ev)) ev = NEG;
      if (IS_NEG(fv)) fv = NEG;
      /* conditional definition: pruned when more than X below best_{k-1}
       * (Z-drop: more than Z + |diag(i,j) - diag_best_{k-1}| below it) */
      int64_t limit = X;
      if (zdrop) {
        const int64_t dd = (j - i) - (bj - bi);
        limit += dd < 0 ? -dd : dd;
      }
      if (IS_NEG(h) || best - h > limit) {
        h = NEG; ev = NEG; fv = NEG;
      } else {
        if (nlo < 0) nlo = j;
        nhi = j;
        if (better(h, i, j, kbest, kbi, kbj)) { kbest = h; kbi = i; kbj = j; }
      }
      cur->H[j] = h; cur->E[j] = ev; cur->F[j] = fv;
    }
    if (cigar && !rc) rc |= as_push(&st, cur, k);
    if (nlo < 0) break; /* every candidate pruned: the extension stops */
    if (better(kbest, kbi, kbj, best, bi, bj)) {
      best = kbest; bi = kbi; bj = kbj;
      best_span = span;
    }
    lo = nlo; hi = nhi;
  }
  for (int t = 0; t < 3; t++) { free(buf[t].H); free(buf[t].E); free(buf[t].F); }
  out->score = best;
  out->q_end = (int32_t)bi;
  out->r_end = (int32_t)bj;
  out->q_begin = 0;
  out->r_begin = 0;
  out->cells = cells;
  out->cigar_len = 0;
  out->span = (int32_t)best_span;
  if (rc) { as_free(&st); return ALNREF_NOMEM; }
  if (cigar) {
    /* the path from the end cell back to (0,0), through stored cells only */
    int trc = traceback(xs_get, &st, mat, Al, o, e, 0, q, r, bi, bj, cigar, cigar_cap, out);
    as_free(&st);
    if (trc != ALNREF_OK) return trc;
  }
  out->status = ALNREF_OK;
  return ALNREF_OK;
}

int alnref_align(const int32_t *matrix, int32_t alphabet, int32_t gap_open,
                 int32_t gap_extend, int32_t mode, int32_t prune,
                 int32_t band_w, int32_t xdrop, const uint8_t *q, int32_t M,
                 const uint8_t *r, int32_t N, uint32_t *cigar,
                 int32_t cigar_cap, alnref_out *out) {
  if (!out) return ALNREF_INVAL;
  memset(out, 0, sizeof(*out));
  if (!matrix || alphabet < 1 || alphabet > 256 || M < 0 || N < 0 ||
      (M > 0 && !q) || (N > 0 && !r) || gap_open > 0 || gap_extend > 0 ||
      mode < ALNREF_GLOBAL || mode > ALNREF_EXTEND || prune < ALNREF_FULL ||
      prune > ALNREF_ZDROP || (prune == ALNREF_BAND && band_w < 0) ||
      ((prune == ALNREF_XDROP || prune == ALNREF_ZDROP) &&
       (xdrop < 0 || mode != ALNREF_EXTEND)) ||
      (cigar && cigar_cap < 0)) {
    out->status = ALNREF_INVAL;
    return ALNREF_INVAL;
  }
  for (int32_t i = 0; i < M; i++)
    if (q[i] >= alphabet) { out->status = ALNREF_BAD_SYMBOL; return ALNREF_BAD_SYMBOL; }
  for (int32_t j = 0; j < N; j++)
    if (r[j] >= alphabet) { out->status = ALNREF_BAD_SYMBOL; return ALNREF_BAD_SYMBOL; }
  int rc;
  if (prune == ALNREF_XDROP || prune == ALNREF_ZDROP)
    rc = align_xdrop(matrix, alphabet, gap_open, gap_extend, xdrop, prune == ALNREF_ZDROP,
                     q, M, r, N, cigar, cigar_cap, out);
  else
    rc = align_rows(matrix, alphabet, gap_open, gap_extend, mode,
                    prune == ALNREF_BAND, band_w, q, M, r, N, cigar, cigar_cap, out);
  out->status = rc;
  return rc;
}

/* ------------------------------------------------------------------ */
/* Batch driver: one pair per task, tasks handed out by a shared counter. */
/* ------------------------------------------------------------------ */
typedef struct {
  const int32_t *matrix;
  int32_t alphabet, o, e, mode, prune, w, x, n;
  const uint8_t *q, *r;
  const int64_t *q_off, *r_off, *cigar_off;
  const int32_t *q_len, *r_len, *cigar_cap;
  uint32_t *cigar;
  alnref_out *out;
  int64_t next;
  pthread_mutex_t mu;
} batch_job;

static void *batch_worker(void *arg) {
  batch_job *b = (batch_job *)arg;
  for (;;) {
    pthread_mutex_lock(&b->mu);
    int64_t p = b->next++;
    pthread_mutex_unlock(&b->mu);
    if (p >= b->n) break;
    uint32_t *cg = b->cigar ? b->cigar + b->cigar_off[p] : NULL;
    int32_t cap = b->cigar ? b->cigar_cap[p] : 0;
    alnref_align(b->matrix, b->alphabet, b->o, b->e, b->mode, b->prune, b->w,
                 b->x, b->q + b->q_off[p], b->q_len[p], b->r + b->r_off[p],
                 b->r_len[p], cg, cap, &b->out[p]);
  }
  return NULL;
}

int alnref_align_batch(const int32_t *matrix, int32_t alphabet,
                       int32_t gap_open, int32_t gap_extend, int32_t mode,
                       int32_t prune, int32_t band_w, int32_t xdrop, int32_t n,
                       const uint8_t *q, const int64_t *q_off,
                       const int32_t *q_len, const uint8_t *r,
                       const int64_t *r_off, const int32_t *r_len,
                       uint32_t *cigar, const int64_t *cigar_off,
                       const int32_t *cigar_cap, alnref_out *out,
                       int32_t nthreads) {
  if (n < 0 || !out || (n > 0 && (!q_off || !q_len || !r_off || !r_len)) ||
      (cigar && (!cigar_off || !cigar_cap)))
    return ALNREF_INVAL;
  if (nthreads < 1) nthreads = 1;
  batch_job b;
  b.matrix = matrix; b.alphabet = alphabet; b.o = gap_open; b.e = gap_extend;
  b.mode = mode; b.prune = prune; b.w = band_w; b.x = xdrop; b.n = n;
  b.q = q; b.r = r; b.q_off = q_off; b.r_off = r_off; b.cigar_off = cigar_off;
  b.q_len = q_len; b.r_len = r_len; b.cigar_cap = cigar_cap; b.cigar = cigar;
  b.out = out; b.next = 0;
  pthread_mutex_init(&b.mu, NULL);
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  if (!th) { pthread_mutex_destroy(&b.mu); return ALNREF_NOMEM; }
  int started = 0;
  for (int t = 0; t < nthreads; t++)
    if (pthread_create(&th[t], NULL, batch_worker, &b) == 0) started++;
    else break;
  if (started == 0) batch_worker(&b);
  for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&b.mu);
  return 0;
}
