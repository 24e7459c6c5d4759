"""Pins for the CPU oracle: checks against things other than the oracle itself.

* brute-force enumeration of every alignment (score, end cell) and of every
  H/E/F state path (CIGAR tie-break) on tiny pairs, for all three modes;
* closed forms: identical sequences, empty sequences, band cell counts and the
  per-antidiagonal band bounds of the paper's static-pruning example (Sec. 7.1);
* special cases that reduce to textbook algorithms: unit-cost scoring is minus
  the Levenshtein distance (the edit-distance recurrence of Sec. 2), a zero gap
  open is linear-gap Needleman-Wunsch;
* invariants: score symmetry, SW >= EXTEND >= NW, SW >= 0, CIGAR rescoring,
  band limits (band covering the matrix = full), X-drop limits (X -> infinity =
  full EXTEND), and agreement with an independent antidiagonal-order
  evaluation (the schedule-invariance property of Sec. 6).
"""
import numpy as np
import pytest

import oracle
from tests import brute


def rand_seq(rng, n, A):
    return [int(x) for x in rng.integers(0, A, size=n)]


def dna_matrix(match, mismatch):
    m = np.full((4, 4), mismatch, dtype=np.int32)
    np.fill_diagonal(m, match)
    return m


def rand_matrix(rng, A, symmetric=False):
    m = rng.integers(-5, 6, size=(A, A)).astype(np.int32)
    if symmetric:
        m = np.triu(m) + np.triu(m, 1).T
    return m


SCORINGS = [
    # (matrix builder, open, extend)
    (lambda rng: dna_matrix(2, -4), -4, -2),          # configs 1 and 4
    (lambda rng: dna_matrix(1, -2), -2, -1),          # config 3
    (lambda rng: rand_matrix(rng, 4), -3, -1),        # asymmetric 4x4
    (lambda rng: rand_matrix(rng, 5), -5, -2),        # asymmetric 5-letter
    (lambda rng: dna_matrix(2, -1), 0, -1),           # linear gap
    (lambda rng: dna_matrix(3, -3), -1, 0),           # zero extend
]


def cigar_pairs(words):
    return [(op, n) for op, n in oracle.alnref.decode_cigar(words)]


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("sc", range(len(SCORINGS)))
def test_global_score_vs_enumeration(sc):
    rng = np.random.default_rng(100 + sc)
    build, o, e = SCORINGS[sc]
    for _ in range(12):
        S = build(rng)
        A = S.shape[0]
        M, N = int(rng.integers(0, 6)), int(rng.integers(0, 6))
        q, r = rand_seq(rng, M, A), rand_seq(rng, N, A)
        got = oracle.align(S, o, e, q, r, mode=oracle.GLOBAL)
        assert got["score"] == brute.global_best(q, r, S.tolist(), o, e)
        assert (got["q_end"], got["r_end"]) == (M, N)
        assert got["cells"] == M * N


@pytest.mark.parametrize("sc", range(len(SCORINGS)))
def test_local_score_vs_enumeration(sc):
    rng = np.random.default_rng(200 + sc)
    build, o, e = SCORINGS[sc]
    for _ in range(6):
        S = build(rng)
        A = S.shape[0]
        M, N = int(rng.integers(0, 5)), int(rng.integers(0, 5))
        q, r = rand_seq(rng, M, A), rand_seq(rng, N, A)
        got = oracle.align(S, o, e, q, r, mode=oracle.LOCAL)
        exp = brute.local_best(q, r, S.tolist(), o, e)
        assert (got["score"], got["q_end"], got["r_end"]) == exp


@pytest.mark.parametrize("sc", range(len(SCORINGS)))
def test_extend_score_vs_enumeration(sc):
    rng = np.random.default_rng(300 + sc)
    build, o, e = SCORINGS[sc]
    for _ in range(8):
        S = build(rng)
        A = S.shape[0]
        M, N = int(rng.integers(0, 6)), int(rng.integers(0, 6))
        q, r = rand_seq(rng, M, A), rand_seq(rng, N, A)
        got = oracle.align(S, o, e, q, r, mode=oracle.EXTEND)
        exp = brute.extend_best(q, r, S.tolist(), o, e)
        assert (got["score"], got["q_end"], got["r_end"]) == exp


@pytest.mark.parametrize("mode", [oracle.GLOBAL, oracle.LOCAL, oracle.EXTEND])
@pytest.mark.parametrize("sc", range(len(SCORINGS)))
def test_cigar_tie_break_vs_state_paths(mode, sc):
    """The traceback returns, among optimal H/E/F state paths ending at the end
    cell, the one whose backward label sequence is lexicographically smallest
    (stop < diagonal < E < F in state H; open < extend in E and F)."""
    rng = np.random.default_rng(400 + 10 * mode + sc)
    build, o, e = SCORINGS[sc]
    for _ in range(6):
        S = build(rng)
        A = S.shape[0]
        M, N = int(rng.integers(0, 5)), int(rng.integers(0, 5))
        # low-entropy sequences make ties common
        q, r = rand_seq(rng, M, min(A, 2)), rand_seq(rng, N, min(A, 2))
        got = oracle.align(S, o, e, q, r, mode=mode, want_cigar=True)
        end = (got["q_end"], got["r_end"])
        val, cig, begin = brute.preferred_path(q, r, S.tolist(), o, e, end,
                                               local=(mode == oracle.LOCAL))
        assert val == got["score"]
        assert cigar_pairs(got["cigar"]) == cig
        assert (got["q_begin"], got["r_begin"]) == begin


# ---------------------------------------------------------------- closed forms
def test_identical_sequences_closed_form():
    """With every diagonal entry above every off-diagonal entry and gaps <= 0,
    aligning x with itself scores sum_i s(x_i, x_i) in all modes, ending at
    (L, L) when every diagonal entry is positive."""
    rng = np.random.default_rng(7)
    for trial in range(20):
        A = 20 if trial % 2 else 4
        S = rng.integers(-4, 4, size=(A, A)).astype(np.int32)
        S = np.triu(S) + np.triu(S, 1).T
        np.fill_diagonal(S, rng.integers(4, 12, size=A))
        L = int(rng.integers(1, 60))
        x = rand_seq(rng, L, A)
        total = int(sum(S[c, c] for c in x))
        for mode in (oracle.GLOBAL, oracle.LOCAL, oracle.EXTEND):
            got = oracle.align(S, -11, -1, x, x, mode=mode, want_cigar=True)
            assert got["score"] == total
            assert (got["q_end"], got["r_end"]) == (L, L)
            assert cigar_pairs(got["cigar"]) == [("=", L)]


def test_dna_identical_is_len_times_match():
    S = dna_matrix(2, -4)
    rng = np.random.default_rng(8)
    x = rand_seq(rng, 1000, 4)
    assert oracle.align(S, -4, -2, x, x)["score"] == 2000


@pytest.mark.parametrize("mode", [oracle.GLOBAL, oracle.EXTEND, oracle.LOCAL])
def test_empty_sequences(mode):
    S = dna_matrix(2, -4)
    o, e = -4, -2
    for M, N in [(0, 0), (0, 5), (7, 0)]:
        q, r = [1] * M, [2] * N
        got = oracle.align(S, o, e, q, r, mode=mode, want_cigar=True)
        if mode == oracle.GLOBAL:
            exp = 0 if M + N == 0 else o + (M + N) * e
            assert got["score"] == exp
            ops = [] if M + N == 0 else [("I" if M else "D", M + N)]
            assert cigar_pairs(got["cigar"]) == ops
        else:
            assert (got["score"], got["q_end"], got["r_end"]) == (0, 0, 0)
            assert len(got["cigar"]) == 0


# ---------------------------------------------------------------- special cases
def levenshtein(a, b):
    """Wagner-Fischer edit distance (unit cost), written independently."""
    prev = list(range(len(b) + 1))
    for i in range(1, len(a) + 1):
        cur = [i] + [0] * len(b)
        for j in range(1, len(b) + 1):
            cur[j] = min(prev[j] + 1, cur[j - 1] + 1,
                         prev[j - 1] + (0 if a[i - 1] == b[j - 1] else 1))
        prev = cur
    return prev[-1]


def test_unit_cost_is_minus_levenshtein():
    """Match 0, mismatch -1, open 0, extend -1 turns the affine recurrence into
    the unit-cost edit-distance recurrence of Sec. 2 (negated)."""
    rng = np.random.default_rng(9)
    S = dna_matrix(0, -1)
    for _ in range(60):
        q = rand_seq(rng, int(rng.integers(0, 40)), 4)
        r = rand_seq(rng, int(rng.integers(0, 40)), 4)
        assert oracle.align(S, 0, -1, q, r)["score"] == -levenshtein(q, r)


def linear_nw(q, r, S, g):
    M, N = len(q), len(r)
    H = [[0] * (N + 1) for _ in range(M + 1)]
    for i in range(1, M + 1):
        H[i][0] = i * g
    for j in range(1, N + 1):
        H[0][j] = j * g
    for i in range(1, M + 1):
        for j in range(1, N + 1):
            H[i][j] = max(H[i - 1][j - 1] + S[q[i - 1]][r[j - 1]],
                          H[i - 1][j] + g, H[i][j - 1] + g)
    return H[M][N]


def test_zero_open_is_linear_gap_nw():
    rng = np.random.default_rng(10)
    for _ in range(40):
        S = rand_matrix(rng, 4)
        q = rand_seq(rng, int(rng.integers(0, 30)), 4)
        r = rand_seq(rng, int(rng.integers(0, 30)), 4)
        g = -int(rng.integers(1, 4))
        assert oracle.align(S, 0, g, q, r)["score"] == linear_nw(q, r, S.tolist(), g)


# ---------------------------------------------------------------- invariants
def rescore_cigar(cig, q, r, S, o, e, qb, rb):
    i, j, total = qb, rb, 0
    for op, n in cig:
        if op in "=X":
            for _ in range(n):
                assert (q[i] == r[j]) == (op == "=")
                total += S[q[i]][r[j]]
                i += 1; j += 1
        elif op == "I":
            total += o + n * e; i += n
        else:
            total += o + n * e; j += n
    return total, i, j


def test_symmetry_chain_and_rescoring():
    rng = np.random.default_rng(11)
    for trial in range(40):
        A = 20 if trial % 2 else 4
        S = rand_matrix(rng, A, symmetric=True)
        o, e = -int(rng.integers(0, 12)), -int(rng.integers(0, 3))
        q = rand_seq(rng, int(rng.integers(0, 50)), A)
        r = rand_seq(rng, int(rng.integers(0, 50)), A)
        res = {}
        for mode in (oracle.GLOBAL, oracle.LOCAL, oracle.EXTEND):
            a = oracle.align(S, o, e, q, r, mode=mode, want_cigar=True)
            b = oracle.align(S, o, e, r, q, mode=mode)
            assert a["score"] == b["score"]
            res[mode] = a
            sc, i, j = rescore_cigar(cigar_pairs(a["cigar"]), q, r, S.tolist(), o, e,
                                     a["q_begin"], a["r_begin"])
            assert sc == a["score"]
            assert (i, j) == (a["q_end"], a["r_end"])
        assert (res[oracle.LOCAL]["score"] >= res[oracle.EXTEND]["score"]
                >= res[oracle.GLOBAL]["score"])
        assert res[oracle.LOCAL]["score"] >= 0
        assert (res[oracle.GLOBAL]["q_begin"], res[oracle.GLOBAL]["r_begin"]) == (0, 0)


def test_bad_symbol_and_invalid_args():
    S = dna_matrix(2, -4)
    assert oracle.align(S, -4, -2, [0, 4], [0])["status"] == oracle.BAD_SYMBOL
    assert oracle.align(S, -4, -2, [0], [9])["status"] == oracle.BAD_SYMBOL
    assert oracle.align(S, 4, -2, [0], [0])["status"] < 0           # open > 0
    assert oracle.align(S, -4, -2, [0], [0], mode=oracle.GLOBAL,
                        prune=oracle.XDROP, xdrop=10)["status"] < 0  # XDROP needs EXTEND
    got = oracle.align(S, -4, -2, [0] * 20, [0] * 20, want_cigar=True, cigar_cap=0)
    assert got["status"] == oracle.CIGAR_CAP


# ---------------------------------------------------------------- band
def band_allowed(M, N, w):
    def f(i, j):
        if M == 0:
            return True
        c = (i * N) // M
        return c - w <= j <= c + w
    return f


def test_band_vs_enumeration():
    rng = np.random.default_rng(12)
    S = dna_matrix(2, -4)
    for _ in range(40):
        M, N = int(rng.integers(0, 7)), int(rng.integers(0, 7))
        w = int(rng.integers(0, 4))
        q, r = rand_seq(rng, M, 4), rand_seq(rng, N, 4)
        got = oracle.align(S, -4, -2, q, r, prune=oracle.BAND, band_w=w)
        exp = brute.global_best(q, r, S.tolist(), -4, -2, allowed=band_allowed(M, N, w))
        if exp is None:
            assert got["status"] == oracle.UNREACHABLE
        else:
            assert got["status"] == oracle.OK and got["score"] == exp


def test_band_covering_matrix_is_full_and_band_is_lower_bound():
    rng = np.random.default_rng(13)
    S = dna_matrix(1, -2)
    for _ in range(30):
        M, N = int(rng.integers(1, 80)), int(rng.integers(1, 80))
        q, r = rand_seq(rng, M, 4), rand_seq(rng, N, 4)
        for mode in (oracle.GLOBAL, oracle.LOCAL, oracle.EXTEND):
            full = oracle.align(S, -2, -1, q, r, mode=mode, want_cigar=True)
            wide = oracle.align(S, -2, -1, q, r, mode=mode, prune=oracle.BAND,
                                band_w=max(M, N), want_cigar=True)
            for k in ("score", "q_end", "r_end", "cells"):
                assert full[k] == wide[k]
            assert np.array_equal(full["cigar"], wide["cigar"])
            w = int(rng.integers(0, 10))
            nb = oracle.align(S, -2, -1, q, r, mode=mode, prune=oracle.BAND, band_w=w)
            if nb["status"] == oracle.OK:
                assert nb["score"] <= full["score"]


def test_band_cell_count_closed_form_square():
    """For M = N the band is -w <= j - i <= w; its interior cell count is
    M(2w+1) - w(w+1) (w < M), and on antidiagonal k its positions m = j are
    max(0,k-M,ceil((k-w)/2)) <= m <= min(N,k,floor((k+w)/2)) (Sec. 7.1)."""
    S = dna_matrix(1, -2)
    rng = np.random.default_rng(14)
    for _ in range(20):
        M = int(rng.integers(1, 120))
        w = int(rng.integers(0, M))
        q, r = rand_seq(rng, M, 4), rand_seq(rng, M, 4)
        got = oracle.align(S, -2, -1, q, r, prune=oracle.BAND, band_w=w)
        assert got["cells"] == M * (2 * w + 1) - w * (w + 1)
        per_k = 0
        for k in range(0, 2 * M + 1):
            lo = max(0, k - M, -((w - k) // 2))      # ceil((k-w)/2)
            hi = min(M, k, (k + w) // 2)
            per_k += sum(1 for m in range(lo, hi + 1) if 1 <= k - m and m >= 1)
        assert per_k == got["cells"]


def test_band_cell_count_closed_form_twice_as_wide():
    """For N = 2M the band centre is c(i) = 2i, so row i keeps
    [max(1, 2i - w), min(2M, 2i + w)]: 2w + 1 cells less what the matrix
    clips.  The top rows lose w + 1 - 2i each while 2i <= w, the bottom rows
    w - 2u (u = M - i) while 2u < w, so for w < M the count is
    M(2w+1) - a(w - a) - b(w - b + 1), a = floor(w/2), b = ceil(w/2)."""
    S = dna_matrix(1, -2)
    rng = np.random.default_rng(15)
    for M in (1, 2, 5, 17, 40, 93):
        for w in sorted({0, 1, 2, 3, M // 2, M - 1} & set(range(M))):
            q, r = rand_seq(rng, M, 4), rand_seq(rng, 2 * M, 4)
            got = oracle.align(S, -2, -1, q, r, prune=oracle.BAND, band_w=w)
            a, b = w // 2, (w + 1) // 2
            assert got["cells"] == M * (2 * w + 1) - a * (w - a) - b * (w - b + 1), (M, w)


# ---------------------------------------------------------------- x-drop
def xdrop_dict(q, r, S, o, e, X, zdrop=False, detail=None):
    """Second, independent implementation of the X-drop rule: cells kept in a
    dict keyed by (i, j); a missing key is minus infinity.  Antidiagonal k's
    candidates are j in [lo, hi+1] of the previous antidiagonal's survivors,
    clipped to the matrix; a candidate is pruned when best - H > X with best
    the running maximum over earlier antidiagonals.  With zdrop the limit is
    X + |(j - i) - (j_best - i_best)| (the Z-drop condition, Sec. 9.3)."""
    M, N = len(q), len(r)
    Hd, Ed, Fd = {(0, 0): 0}, {}, {}
    best, end = 0, (0, 0)
    lo = hi = 0
    cells = 0
    spans = {}
    for k in range(1, M + N + 1):
        js = [j for j in range(max(lo, k - M), min(hi + 1, k, N) + 1)]
        if not js:
            break
        spans[k] = 2 * (js[-1] - js[0])
        alive = []
        kbest = None
        for j in js:
            i = k - j
            if i == 0:
                h = o + j * e; ev = h; fv = None
            elif j == 0:
                h = o + i * e; fv = h; ev = None
            else:
                cells += 1
                c1 = [x for x in (Ed.get((i, j - 1)), ) if x is not None]
                c2 = [x for x in (Hd.get((i, j - 1)), ) if x is not None]
                cand_e = [x + e for x in c1] + [x + o + e for x in c2]
                ev = max(cand_e) if cand_e else None
                c3 = [x for x in (Fd.get((i - 1, j)), ) if x is not None]
                c4 = [x for x in (Hd.get((i - 1, j)), ) if x is not None]
                cand_f = [x + e for x in c3] + [x + o + e for x in c4]
                fv = max(cand_f) if cand_f else None
                cand_h = [x for x in (ev, fv) if x is not None]
                if (i - 1, j - 1) in Hd:
                    cand_h.append(Hd[(i - 1, j - 1)] + S[q[i - 1]][r[j - 1]])
                h = max(cand_h) if cand_h else None
            limit = X + (abs((j - i) - (end[1] - end[0])) if zdrop else 0)
            if h is None or best - h > limit:
                continue
            Hd[(i, j)] = h
            if ev is not None:
                Ed[(i, j)] = ev
            if fv is not None:
                Fd[(i, j)] = fv
            alive.append(j)
            if kbest is None or (h, -i, -j) > (kbest[0], -kbest[1], -kbest[2]):
                kbest = (h, i, j)
        if not alive:
            break
        # the surviving cells form one contiguous run of candidates or not;
        # the domain keeps only its first and last survivors
        if kbest[0] > best or (kbest[0] == best and (kbest[1], kbest[2]) < end):
            best, end = kbest[0], (kbest[1], kbest[2])
        lo, hi = min(alive), max(alive)
    if detail is not None:
        detail["kept"] = set(Hd)
        detail["span"] = max([spans[k] for k in spans if k <= end[0] + end[1]], default=0)
    return best, end, cells


def test_xdrop_vs_dict_implementation():
    rng = np.random.default_rng(15)
    for trial in range(150):
        S = dna_matrix(2, -4) if trial % 3 else rand_matrix(rng, 4)
        o, e = -4, -2
        X = int(rng.integers(0, 30))
        M, N = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        base = rand_seq(rng, max(M, N), 4)
        q = base[:M] if trial % 2 else rand_seq(rng, M, 4)
        r = [c if rng.random() > 0.15 else int(rng.integers(0, 4)) for c in base[:N]]
        got = oracle.align(S, o, e, q, r, mode=oracle.EXTEND, prune=oracle.XDROP, xdrop=X)
        best, end, cells = xdrop_dict(q, r, S.tolist(), o, e, X)
        assert (got["score"], (got["q_end"], got["r_end"]), got["cells"]) == (best, end, cells)


def test_xdrop_infinite_x_is_full_extend():
    rng = np.random.default_rng(16)
    S = dna_matrix(2, -4)
    for _ in range(30):
        M, N = int(rng.integers(0, 70)), int(rng.integers(0, 70))
        q, r = rand_seq(rng, M, 4), rand_seq(rng, N, 4)
        full = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND)
        xd = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND, prune=oracle.XDROP,
                          xdrop=1 << 30)
        assert (xd["score"], xd["q_end"], xd["r_end"]) == (
            full["score"], full["q_end"], full["r_end"])
        assert xd["cells"] == M * N
        small = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND, prune=oracle.XDROP,
                             xdrop=int(rng.integers(0, 20)))
        assert small["score"] <= full["score"]
        assert small["cells"] <= M * N


def test_xdrop_identical_sequences():
    """On identical sequences the odd antidiagonals hold only cells one gap off
    the main diagonal, scoring best + o + e; so X >= -(o+e) reaches the corner
    with score len*match, while X < -(o+e) prunes all of antidiagonal 1 and the
    extension stops at (0,0) having evaluated no interior cell."""
    S = dna_matrix(2, -4)
    rng = np.random.default_rng(17)
    x = rand_seq(rng, 300, 4)
    for X in (6, 10, 100):
        got = oracle.align(S, -4, -2, x, x, mode=oracle.EXTEND, prune=oracle.XDROP, xdrop=X)
        assert (got["score"], got["q_end"], got["r_end"]) == (600, 300, 300)
    for X in (0, 5):
        got = oracle.align(S, -4, -2, x, x, mode=oracle.EXTEND, prune=oracle.XDROP, xdrop=X)
        assert (got["score"], got["q_end"], got["r_end"], got["cells"]) == (0, 0, 0, 0)


# ---------------------------------------------------------------- z-drop
def test_zdrop_vs_dict_implementation():
    rng = np.random.default_rng(25)
    for trial in range(150):
        S = dna_matrix(2, -4) if trial % 3 else rand_matrix(rng, 4)
        o, e = -4, -2
        Z = int(rng.integers(0, 30))
        M, N = int(rng.integers(0, 40)), int(rng.integers(0, 40))
        base = rand_seq(rng, max(M, N), 4)
        q = base[:M] if trial % 2 else rand_seq(rng, M, 4)
        r = [c if rng.random() > 0.15 else int(rng.integers(0, 4)) for c in base[:N]]
        if trial % 5 == 0 and N > 12:  # a long insertion: where the distance term matters
            r = r[:N // 3] + rand_seq(rng, 10, 4) + r[N // 3:]
        got = oracle.align(S, o, e, q, r, mode=oracle.EXTEND, prune=oracle.ZDROP, xdrop=Z)
        best, end, cells = xdrop_dict(q, r, S.tolist(), o, e, Z, zdrop=True)
        assert (got["score"], (got["q_end"], got["r_end"]), got["cells"]) == (best, end, cells)


def test_zdrop_infinite_z_is_full_extend():
    rng = np.random.default_rng(26)
    S = dna_matrix(2, -4)
    for _ in range(30):
        M, N = int(rng.integers(0, 70)), int(rng.integers(0, 70))
        q, r = rand_seq(rng, M, 4), rand_seq(rng, N, 4)
        full = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND)
        zd = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND, prune=oracle.ZDROP,
                          xdrop=1 << 30)
        assert (zd["score"], zd["q_end"], zd["r_end"], zd["cells"]) == (
            full["score"], full["q_end"], full["r_end"], M * N)


def test_zdrop_identical_sequences():
    """On identical sequences the best cell stays on the main diagonal and the
    odd antidiagonals hold cells one diagonal off it scoring best + o + e, so
    Z-drop keeps them for Z + 1 >= -(o+e), one less than X-drop needs: with
    o + e = -6, Z = 5 reaches the corner where X = 5 stops at (0,0)."""
    S = dna_matrix(2, -4)
    rng = np.random.default_rng(27)
    x = rand_seq(rng, 300, 4)
    for Z in (5, 10, 100):
        got = oracle.align(S, -4, -2, x, x, mode=oracle.EXTEND, prune=oracle.ZDROP, xdrop=Z)
        assert (got["score"], got["q_end"], got["r_end"]) == (600, 300, 300)
    for Z in (0, 4):
        got = oracle.align(S, -4, -2, x, x, mode=oracle.EXTEND, prune=oracle.ZDROP, xdrop=Z)
        assert (got["score"], got["q_end"], got["r_end"], got["cells"]) == (0, 0, 0, 0)
    xd = oracle.align(S, -4, -2, x, x, mode=oracle.EXTEND, prune=oracle.XDROP, xdrop=5)
    assert (xd["score"], xd["cells"]) == (0, 0)


def test_zdrop_survives_a_long_gap_that_xdrop_cuts():
    """A 40-base insertion in the reference after 60 matching bases, then 60
    more (a and b over letters 0-1, the insertion all letter 3, so nothing
    matches by chance): crossing it costs o + 40e = -84 below the best so far.
    X-drop with X = 60 stops at (60, 60) with 120 (a gap cell L deep falls
    4 + 2L below it, pruned from L = 29); Z-drop with Z = 60 crosses it (the
    limit on diagonal d is 60 + d, and 4 + 2d exceeds it only beyond d = 56)
    and ends at the far corner with 120 matches minus the gap."""
    S = dna_matrix(2, -4)
    rng = np.random.default_rng(28)
    a = [int(c) for c in rng.integers(0, 2, 60)]
    b = [int(c) for c in rng.integers(0, 2, 60)]
    ins = [3] * 40
    q, r = a + b, a + ins + b
    xd = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND, prune=oracle.XDROP, xdrop=60)
    zd = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND, prune=oracle.ZDROP, xdrop=60)
    full = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND)
    assert xd["score"] == 120 and (xd["q_end"], xd["r_end"]) == (60, 60)
    assert (zd["score"], zd["q_end"], zd["r_end"]) == (full["score"], full["q_end"], full["r_end"])
    assert full["score"] == 240 - 4 - 2 * 40 and (full["q_end"], full["r_end"]) == (120, 160)


# ---------------------------------------------------------------- schedule invariance
def antidiagonal_fill(q, r, S, o, e, mode):
    """Evaluate H/E/F in antidiagonal order k = i + j (Sec. 6.2 shear,
    m = j, i = k - m) and return (score, end)."""
    M, N = len(q), len(r)
    NEG = -(1 << 60)
    H = {}
    E = {}
    F = {}
    local = mode == oracle.LOCAL
    best = (NEG, 0, 0)
    for k in range(M + N + 1):
        for m in range(max(0, k - M), min(N, k) + 1):
            i, j = k - m, m
            if i == 0 and j == 0:
                h, ev, fv = 0, NEG, NEG
            elif i == 0:
                h, ev, fv = (0, NEG, NEG) if local else (o + j * e, o + j * e, NEG)
            elif j == 0:
                h, ev, fv = (0, NEG, NEG) if local else (o + i * e, NEG, o + i * e)
            else:
                ev = max(E[(i, j - 1)] + e, H[(i, j - 1)] + o + e)
                fv = max(F[(i - 1, j)] + e, H[(i - 1, j)] + o + e)
                h = max(H[(i - 1, j - 1)] + S[q[i - 1]][r[j - 1]], ev, fv)
                if local:
                    h = max(h, 0)
            H[(i, j)], E[(i, j)], F[(i, j)] = h, ev, fv
            if (h, -i, -j) > (best[0], -best[1], -best[2]):
                best = (h, i, j)
    if mode == oracle.GLOBAL:
        return H[(M, N)], (M, N)
    return best[0], (best[1], best[2])


def test_schedule_invariance_antidiagonal_order():
    rng = np.random.default_rng(18)
    for trial in range(30):
        S = rand_matrix(rng, 4)
        q = rand_seq(rng, int(rng.integers(0, 25)), 4)
        r = rand_seq(rng, int(rng.integers(0, 25)), 4)
        for mode in (oracle.GLOBAL, oracle.LOCAL, oracle.EXTEND):
            got = oracle.align(S, -3, -1, q, r, mode=mode)
            sc, end = antidiagonal_fill(q, r, S.tolist(), -3, -1, mode)
            assert got["score"] == sc
            assert (got["q_end"], got["r_end"]) == end


def test_batch_driver_matches_single_calls():
    rng = np.random.default_rng(19)
    S = dna_matrix(2, -4)
    n = 40
    ql = rng.integers(0, 60, size=n).astype(np.int32)
    rl = rng.integers(0, 60, size=n).astype(np.int32)
    q = rng.integers(0, 4, size=int(ql.sum())).astype(np.uint8)
    r = rng.integers(0, 4, size=int(rl.sum())).astype(np.uint8)
    qo = np.concatenate([[0], np.cumsum(ql)[:-1]]).astype(np.int64)
    ro = np.concatenate([[0], np.cumsum(rl)[:-1]]).astype(np.int64)
    for mode, prune in [(0, 0), (1, 0), (2, 0), (0, 1), (2, 2)]:
        b = oracle.align_batch(S, -4, -2, q, qo, ql, r, ro, rl, mode=mode,
                               prune=prune, band_w=5, xdrop=20,
                               want_cigar=(prune != 2), nthreads=4)
        for p in range(n):
            s = oracle.align(S, -4, -2, q[qo[p]:qo[p] + ql[p]], r[ro[p]:ro[p] + rl[p]],
                             mode=mode, prune=prune, band_w=5, xdrop=20,
                             want_cigar=(prune != 2))
            for k in ("score", "q_end", "r_end", "cells", "status"):
                assert int(b[k][p]) == s[k]
            if prune != 2:
                c = b["cigar"][b["cigar_off"][p]: b["cigar_off"][p] + b["cigar_len"][p]]
                assert np.array_equal(c, s["cigar"])


# ---------------------------------------------------------------- x-drop / z-drop traceback
def rescore(cig, q, r, S, o, e):
    """Score of a CIGAR from (0,0), written out independently of the oracle."""
    i = j = 0
    total = 0
    for op, n in cig:
        if op in "=X":
            for _ in range(n):
                total += S[q[i]][r[j]]
                i += 1
                j += 1
        elif op == "I":
            total += o + n * e
            i += n
        else:
            total += o + n * e
            j += n
    return total, i, j


@pytest.mark.parametrize("prune", ["XDROP", "ZDROP"])
def test_dynamic_prune_cigar_infinite_threshold_is_full_extend(prune):
    """With a threshold no cell can fall below, the stored antidiagonal region
    is the whole matrix: the CIGAR equals the row-major full-matrix one."""
    rng = np.random.default_rng(51)
    S = dna_matrix(2, -4)
    for _ in range(40):
        M, N = int(rng.integers(0, 60)), int(rng.integers(0, 60))
        base = rand_seq(rng, max(M, N), 4)
        q = base[:M]
        r = [c if rng.random() > 0.2 else int(rng.integers(0, 4)) for c in base[:N]]
        full = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND, want_cigar=True)
        dyn = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND,
                           prune=getattr(oracle, prune), xdrop=1 << 30, want_cigar=True)
        assert dyn["status"] == oracle.OK
        assert (dyn["score"], dyn["q_end"], dyn["r_end"]) == (
            full["score"], full["q_end"], full["r_end"])
        assert np.array_equal(dyn["cigar"], full["cigar"])


@pytest.mark.parametrize("zdrop", [False, True])
def test_dynamic_prune_cigar_is_preferred_path_through_kept_cells(zdrop):
    """Brute force on tiny pairs: among all state paths from the end cell to
    (0,0) through cells the dictionary implementation keeps, the optimal ones
    score the extension's score, and the CIGAR is the one with the smallest
    backward label sequence (diag < E < F, open < extend)."""
    rng = np.random.default_rng(52 + zdrop)
    checked = 0
    for trial in range(400):
        S = dna_matrix(2, -4) if trial % 2 else rand_matrix(rng, 4)
        o, e = -4, -2
        X = int(rng.integers(0, 14))
        M, N = int(rng.integers(1, 7)), int(rng.integers(1, 7))
        base = rand_seq(rng, max(M, N), 4)
        q = base[:M]
        r = [c if rng.random() > 0.3 else int(rng.integers(0, 4)) for c in base[:N]]
        det = {}
        best, end, _ = xdrop_dict(q, r, S.tolist(), o, e, X, zdrop=zdrop, detail=det)
        got = oracle.align(S, o, e, q, r, mode=oracle.EXTEND,
                           prune=oracle.ZDROP if zdrop else oracle.XDROP, xdrop=X,
                           want_cigar=True)
        assert (got["score"], (got["q_end"], got["r_end"])) == (best, end)
        assert got["span"] == det["span"]
        if end == (0, 0):
            assert len(got["cigar"]) == 0
            continue
        kept = det["kept"]
        v, cig, begin = brute.preferred_path(q, r, S.tolist(), o, e, end, False,
                                             allowed=lambda i, j: (i, j) in kept)
        assert v == best and begin == (0, 0)
        assert cigar_pairs(got["cigar"]) == cig, (q, r, X, zdrop)
        checked += 1
    assert checked > 100


@pytest.mark.parametrize("prune", ["XDROP", "ZDROP"])
def test_dynamic_prune_cigar_rescores_and_consumes_the_end_cell(prune):
    rng = np.random.default_rng(54)
    S = dna_matrix(2, -4)
    for _ in range(60):
        L = int(rng.integers(20, 400))
        ref = rand_seq(rng, L, 4)
        q = [c if rng.random() > 0.15 else int(rng.integers(0, 4)) for c in ref]
        if rng.random() < 0.5:
            at = int(rng.integers(0, L))
            q = q[:at] + rand_seq(rng, int(rng.integers(5, 40)), 4) + q[at:]
        q = q + rand_seq(rng, 30, 4)
        r = ref + rand_seq(rng, 30, 4)
        X = int(rng.integers(10, 120))
        got = oracle.align(S, -4, -2, q, r, mode=oracle.EXTEND, prune=getattr(oracle, prune),
                           xdrop=X, want_cigar=True)
        sc, i, j = rescore(cigar_pairs(got["cigar"]), q, r, S.tolist(), -4, -2)
        assert (sc, i, j) == (got["score"], got["q_end"], got["r_end"])
        assert (got["q_begin"], got["r_begin"]) == (0, 0)
