"""Pins of the folding oracle (oracle/foldref.c) to things other than itself.

The RNA-folding recurrence (the example-recurrence table of Sec. 3) is the
Nussinov base-pair maximisation: F(0, n-1) is the largest total pairing score
of a set of non-crossing base pairs.  So the unpruned oracle is pinned by
brute-force enumeration of every non-crossing structure of tiny sequences and
by closed forms; the X-drop transfer (Sec. 9.5) by its limits (X far above
every score, sequences that never leave the warm-up) and by a second,
independently written implementation of the rule."""
import functools
import itertools

import numpy as np
import pytest

import oracle

A, C, G, U = 0, 1, 2, 3
COMP = {A: U, U: A, C: G, G: C}


def pair_table(weights):
    """4x4 pairing scores from {(a, b): w} (symmetric)."""
    P = np.zeros((4, 4), dtype=np.int32)
    for (a, b), w in weights.items():
        P[a, b] = w
        P[b, a] = w
    return P


# canonical pairs plus the G-U wobble, one point each (the reading the
# workload uses), and a weighted variant (G-C 3, A-U 2, G-U 1)
UNIT = pair_table({(A, U): 1, (C, G): 1, (G, U): 1})
WEIGHTED = pair_table({(A, U): 2, (C, G): 3, (G, U): 1})
TABLES = {"unit": UNIT, "weighted": WEIGHTED}


def brute_force(x, P, min_loop):
    """Largest total score over every set of non-crossing pairs (i, j) with
    j - i > min_loop and a positive pairing score, by enumeration."""
    n = len(x)

    @functools.lru_cache(maxsize=None)
    def structures(i, j):
        # every structure on x[i..j] as a frozenset of pairs
        if i >= j:
            return [frozenset()]
        out = list(structures(i + 1, j))  # x_i unpaired
        for k in range(i + min_loop + 1, j + 1):
            if P[x[i], x[k]] > 0:
                for s1 in structures(i + 1, k - 1):
                    for s2 in structures(k + 1, j):
                        out.append(s1 | s2 | {(i, k)})
        return out

    best = 0
    for s in structures(0, n - 1):
        # non-crossing by construction; recheck it independently
        for (a, b), (c, d) in itertools.combinations(sorted(s), 2):
            assert not (a < c < b < d), (a, b, c, d)
        best = max(best, sum(int(P[x[a], x[b]]) for a, b in s))
    return best


@pytest.mark.parametrize("table", sorted(TABLES))
@pytest.mark.parametrize("min_loop", [0, 1, 3])
def test_unpruned_equals_brute_force(table, min_loop):
    P = TABLES[table]
    rng = np.random.default_rng(100 + min_loop)
    for trial in range(40):
        n = int(rng.integers(1, 11))
        x = tuple(int(v) for v in rng.integers(0, 4, size=n))
        got = oracle.fold(P, x, min_loop=min_loop)
        assert got["status"] == 0
        assert got["score"] == brute_force(x, P, min_loop), (x, got)
        assert (got["i"], got["j"]) == (0, n - 1)
        assert got["cells"] == n * (n - 1) // 2
        assert got["terms"] == n * (n * n - 1) // 6  # sum over spans t of (n - t) t
        assert got["full"] == 1


def test_closed_forms():
    # a perfect hairpin: x followed by its reverse complement pairs every base
    rng = np.random.default_rng(7)
    for k in (1, 5, 40, 120):
        x = [int(v) for v in rng.integers(0, 4, size=k)]
        seq = x + [COMP[v] for v in reversed(x)]
        assert oracle.fold(UNIT, seq)["score"] == k
    # G^k, a loop of h+1 A's, C^k: exactly k G-C pairs, nothing else can pair
    for k, h in ((3, 0), (7, 3), (20, 5)):
        seq = [G] * k + [A] * (h + 1) + [C] * k
        assert oracle.fold(UNIT, seq, min_loop=h)["score"] == k
        assert oracle.fold(WEIGHTED, seq, min_loop=h)["score"] == 3 * k
        # with a loop of h - 1 the innermost G and C are too close to pair, so
        # one G is left over
        if h >= 1:
            seq2 = [G] * k + [A] * (h - 1) + [C] * k
            assert oracle.fold(UNIT, seq2, min_loop=h)["score"] == k - 1
    # letters that cannot pair with each other fold to 0
    for n in (1, 2, 50):
        assert oracle.fold(UNIT, [A] * n)["score"] == 0
        assert oracle.fold(UNIT, [C] * n)["score"] == 0
    # the empty and one-letter sequences
    assert oracle.fold(UNIT, [])["score"] == 0
    one = oracle.fold(UNIT, [G])
    assert (one["score"], one["cells"], one["i"], one["j"]) == (0, 0, 0, 0)


def dict_fold(x, P, min_loop, X, warmup):
    """The X-drop rule on the folding recurrence, written independently:
    surviving cells in a dictionary keyed by interval, wavefronts by span."""
    n = len(x)
    if n == 0:
        return 0, 0, 0, 0, 0
    kept = {(i, i): 0 for i in range(n)}

    def get(a, b):
        if b == a - 1:
            return 0
        return kept.get((a, b))

    best, bcell = 0, (0, 0)
    first, last = 0, n - 1
    cells = terms = 0
    for t in range(1, n):
        cand = range(max(first - 1, 0), min(last, n - 1 - t) + 1)
        if len(cand) == 0:
            break
        new = {}
        for i in cand:
            j = i + t
            opts = []
            for v in (get(i + 1, j), get(i, j - 1)):
                if v is not None:
                    opts.append(v)
            inner = get(i + 1, j - 1)
            if inner is not None:
                opts.append(inner + (int(P[x[i], x[j]]) if j - i > min_loop else 0))
            for k in range(i, j):
                a, b = get(i, k), get(k + 1, j)
                if a is not None and b is not None:
                    opts.append(a + b)
            cells += 1
            terms += j - i
            if not opts:
                continue
            v = max(opts)
            if X is not None and t > warmup and best - v > X:
                continue
            new[(i, j)] = v
        if not new:
            break
        kept.update(new)
        top = max(new.values())
        if top >= best:
            best = top
            bcell = min(c for c, v in new.items() if v == top)
        first = min(i for i, _ in new)
        last = max(i for i, _ in new)
    return best, bcell[0], bcell[1], cells, terms


@pytest.mark.parametrize("X", [0, 1, 2, 5])
@pytest.mark.parametrize("warmup", [0, 3, 15])
def test_xdrop_matches_independent_implementation(X, warmup):
    rng = np.random.default_rng(1000 + 10 * X + warmup)
    for trial in range(12):
        n = int(rng.integers(1, 70))
        x = [int(v) for v in rng.integers(0, 4, size=n)]
        ml = int(rng.integers(0, 4))
        P = TABLES["weighted" if trial % 3 == 0 else "unit"]
        got = oracle.fold(P, x, min_loop=ml, xdrop=X, warmup=warmup)
        exp = dict_fold(x, P, ml, X, warmup)
        assert (got["score"], got["i"], got["j"], got["cells"], got["terms"]) == exp, \
            (n, X, warmup, ml)


def test_xdrop_limits():
    rng = np.random.default_rng(3)
    for n in (2, 17, 90, 300):
        x = [int(v) for v in rng.integers(0, 4, size=n)]
        full = oracle.fold(UNIT, x, min_loop=3)
        # X above every score: nothing is pruned
        big = oracle.fold(UNIT, x, min_loop=3, xdrop=10 ** 9, warmup=0)
        assert (big["score"], big["i"], big["j"], big["cells"]) == \
            (full["score"], full["i"], full["j"], full["cells"])
        # a warm-up covering every span: nothing is pruned either
        wu = oracle.fold(UNIT, x, min_loop=3, xdrop=0, warmup=n)
        assert (wu["score"], wu["cells"]) == (full["score"], full["cells"])
        # pruning can only lose score and cells
        for X in (0, 1, 2, 8):
            p = oracle.fold(UNIT, x, min_loop=3, xdrop=X, warmup=15)
            assert p["score"] <= full["score"]
            assert p["cells"] <= full["cells"]


def test_batch_matches_single_calls():
    rng = np.random.default_rng(5)
    lens = rng.integers(0, 120, size=40).astype(np.int32)
    xs = [rng.integers(0, 4, size=int(L)).astype(np.uint8) for L in lens]
    off = np.zeros(len(xs), dtype=np.int64)
    off[1:] = np.cumsum(lens[:-1])
    cat = np.concatenate(xs)
    for X in (oracle.NO_XDROP, 2):
        res = oracle.fold_batch(UNIT, cat, off, lens, min_loop=3, xdrop=X, warmup=15, nthreads=4)
        for p, x in enumerate(xs):
            one = oracle.fold(UNIT, x, min_loop=3, xdrop=X, warmup=15)
            assert (int(res["score"][p]), int(res["i"][p]), int(res["j"][p]),
                    int(res["cells"][p])) == (one["score"], one["i"], one["j"], one["cells"])


def test_bad_codes_rejected():
    assert oracle.fold(UNIT, [0, 1, 4])["status"] == -1
