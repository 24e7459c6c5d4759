"""GPU parity of the score-major search schedule (Sec. 6.3) against the CPU
oracle, for unit edit costs and for gap-affine penalties: the score equals
the oracle's full-matrix global score under the same scoring (for unit costs
minus the edit distance, the oracle itself pinned to an independent
Levenshtein), the end cell is (M, N), and `cells` equals the number of
(score, diagonal) entries of the widening domain, sum over s = 0..S of
(min(s // e, N) + min(s // e, M) + 1) with e the gap-extension penalty."""
import numpy as np
import pytest

from paper_2607_06225_amd import workloads as W
from tests.parity import compare, oracle_batch, search_cells

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2607_06225_amd import aln
    assert torch.cuda.is_available()
    c = aln.Context(0)
    yield c
    c.close()


def run(ctx, batch, **kw):
    from paper_2607_06225_amd import aln
    print(f"[gpu] {batch.name} n={batch.n} search {kw}", flush=True)
    return aln.align(ctx, batch, **kw)


def check(batch, res):
    return compare(batch, res, None, oracle_batch(batch))


def pairs(rng, lengths, div):
    st = W.Stream(int(rng.integers(1, 1 << 30)), 15)
    qs, rs = [], []
    for M, N in lengths:
        ref = rng.integers(0, 4, size=N).astype(np.uint8)
        q = W.mutate(ref, div, 2, 1, 1, 4, st)[:M] if div < 1 else \
            rng.integers(0, 4, size=M).astype(np.uint8)
        if len(q) < M:
            q = np.concatenate([q, rng.integers(0, 4, size=M - len(q)).astype(np.uint8)])
        qs.append(q)
        rs.append(ref)
    return qs, rs


def sbatch(qs, rs, name):
    return W.pack_pairs(qs, rs, W.dna_matrix(0, -1), 0, -1, W.GLOBAL, W.SEARCH, name=name)


@pytest.mark.parametrize("div", [0.0, 0.01, 0.05, 0.3, 1.0])
def test_search_edit_distance(ctx, div):
    rng = np.random.default_rng(900 + int(100 * div))
    lengths = [(0, 0), (0, 5), (5, 0), (1, 1), (1, 70), (70, 1), (63, 64), (64, 63),
               (65, 129)] + [(int(rng.integers(1, 2500)), int(rng.integers(1, 2500)))
                             for _ in range(40)]
    if div < 0.5:  # similar lengths, as for related sequences
        lengths = lengths[:9] + [(L, L + int(rng.integers(-20, 21))) for L, _ in lengths[9:]]
        lengths = [(max(M, 0), max(N, 0)) for M, N in lengths]
    qs, rs = pairs(rng, lengths, div)
    b = sbatch(qs, rs, f"search_{div}")
    res, _ = run(ctx, b)
    assert check(b, res) == []


def test_search_long_pairs_and_indels(ctx):
    """Pairs of 4 kbp (the paper's largest table size) at 1% and 5%
    divergence, some with a 60-base insertion."""
    rng = np.random.default_rng(911)
    qs, rs = [], []
    for k in range(24):
        q, r = pairs(rng, [(4000, 4000)], 0.01 if k % 2 else 0.05)
        q, r = q[0], r[0]
        if k % 3 == 0:
            q = np.concatenate([q[:2000], rng.integers(0, 4, 60).astype(np.uint8), q[2000:]])
        qs.append(q)
        rs.append(r)
    b = sbatch(qs, rs, "search_4k")
    res, _ = run(ctx, b)
    assert check(b, res) == []


def test_search_matches_full_matrix_on_gpu(ctx):
    """The same pairs through the full-matrix strip path (unit-cost global
    alignment): identical scores."""
    rng = np.random.default_rng(913)
    qs, rs = pairs(rng, [(int(L), int(L) + 7) for L in rng.integers(100, 1500, 30)], 0.05)
    bs = sbatch(qs, rs, "search_vs_full")
    bf = W.pack_pairs(qs, rs, W.dna_matrix(0, -1), 0, -1, W.GLOBAL, W.FULL, name="full_unit")
    rs_, _ = run(ctx, bs)
    rf, _ = run(ctx, bf)
    assert np.array_equal(rs_["score"], rf["score"])


def test_search_maximum_rows(ctx):
    """The largest query the int16 row store holds (32 767 rows), in a batch
    whose longest query plus longest reference fills most of the LDS limit:
    scores equal the oracle's where no closed form exists, and the closed
    forms (identical sequences: 0; one side empty: the other's length)
    elsewhere; `cells` follows the domain's count."""
    rng = np.random.default_rng(919)
    L, N = 32767, 20000
    qs, rs = pairs(rng, [(L, 4000), (4000, 3991)], 0.005)
    same = rng.integers(0, 4, size=N).astype(np.uint8)
    qs += [same, rng.integers(0, 4, size=L).astype(np.uint8), np.zeros(0, np.uint8)]
    rs += [same.copy(), np.zeros(0, np.uint8), rng.integers(0, 4, size=N).astype(np.uint8)]
    b = sbatch(qs, rs, "search_max_rows")
    res, _ = run(ctx, b)
    assert list(res["status"]) == [0] * 5
    assert check(sbatch(qs[:2], rs[:2], "search_max_rows_head"), res[:2]) == []
    assert list(res["score"][2:]) == [0, -L, -N]
    for p in range(5):
        S = -int(res["score"][p])
        assert int(res["cells"][p]) == search_cells(S, len(qs[p]), len(rs[p]))
        assert (int(res["q_end"][p]), int(res["r_end"][p])) == (len(qs[p]), len(rs[p]))


def test_search_four_wavefronts_near_their_lds_limit(ctx):
    """Pairs whose two F rows and sequences still fit one CU's LDS (the batch's
    longest query plus longest reference about 31 000), so four wavefronts
    share each pair: scores, end cells and cells equal the oracle's."""
    rng = np.random.default_rng(923)
    qs, rs = pairs(rng, [(16000, 15990), (20000, 11000), (300, 310)], 0.01)
    b = sbatch(qs, rs, "search_group_limit")
    res, _ = run(ctx, b)
    assert check(b, res) == []


def test_search_per_pair_and_graph_match(ctx):
    rng = np.random.default_rng(917)
    qs, rs = pairs(rng, [(300, 310), (50, 60), (1200, 1190), (0, 9)], 0.1)
    b = sbatch(qs, rs, "search_pp")
    r1, _ = run(ctx, b)
    r2, _ = run(ctx, b, per_pair=True)
    r3, _ = run(ctx, b, graph=True)
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
    assert check(b, r1) == []


AFFINE = [(4, 6, 2), (2, 3, 1), (3, 0, 2), (1, 2, 1), (5, 1, 3)]  # (mismatch x, open o, extend e)


def abatch(qs, rs, pen, name):
    x, o, e = pen
    return W.pack_pairs(qs, rs, W.dna_matrix(0, -x), -o, -e, W.GLOBAL, W.SEARCH, name=name)


@pytest.mark.parametrize("pen", AFFINE)
@pytest.mark.parametrize("div", [0.02, 0.15, 1.0])
def test_search_gap_affine(ctx, pen, div):
    """Gap-affine penalties (match 0, mismatch x, a gap of length L costing
    o + L e): the score is minus the smallest penalty, equal to the oracle's
    full-matrix Gotoh global score under (0, -x, -o, -e); `cells` counts the
    (score, diagonal) entries with |d| <= s / e."""
    rng = np.random.default_rng(930 + int(100 * div) + 7 * pen[0] + pen[1])
    lengths = [(0, 0), (0, 5), (5, 0), (1, 1), (2, 9), (9, 2), (63, 64), (65, 129)] + \
              [(int(L), int(L) + int(rng.integers(-30, 31))) for L in rng.integers(30, 1500, 30)]
    lengths = [(max(M, 0), max(N, 0)) for M, N in lengths]
    qs, rs = pairs(rng, lengths, div)
    b = abatch(qs, rs, pen, f"search_affine_{pen}_{div}")
    res, _ = run(ctx, b)
    assert check(b, res) == []
    if pen == (4, 6, 2):
        # a first pass keeps a capped diagonal range (a few hundred diagonals
        # here); unrelated pairs outgrow it and are recomputed with full rows
        from paper_2607_06225_amd import aln
        widened = (res["flags"] & aln.F_WIDENED) != 0
        assert widened.any() if div == 1.0 else not widened.any()


def test_search_gap_affine_indels_and_graph(ctx):
    """Long indels (a single gap of 40-200 bases) under gap-affine penalties,
    per-pair and graph launches identical to the batch."""
    rng = np.random.default_rng(941)
    qs, rs = [], []
    for k in range(16):
        q, r = pairs(rng, [(int(rng.integers(400, 2000)),) * 2], 0.02)
        q, r = q[0], r[0]
        g = int(rng.integers(40, 200))
        at = int(rng.integers(10, len(q) - 10))
        ins = rng.integers(0, 4, g).astype(np.uint8)
        if k % 2:
            q = np.concatenate([q[:at], ins, q[at:]])
        else:
            r = np.concatenate([r[:at], ins, r[at:]])
        qs.append(q)
        rs.append(r)
    b = abatch(qs, rs, (4, 6, 2), "search_affine_indel")
    r1, _ = run(ctx, b)
    r2, _ = run(ctx, b, per_pair=True)
    r3, _ = run(ctx, b, graph=True)
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
    assert check(b, r1) == []


def test_search_rejects_what_it_does_not_compute(ctx):
    from paper_2607_06225_amd import aln
    ql = np.array([10], np.int32)
    sid_unit = ctx.set_scoring(W.dna_matrix(0, -1), 0, -1)
    sid_affine = ctx.set_scoring(W.dna_matrix(2, -4), -4, -2)
    for sid, mode, cig in ((sid_affine, W.GLOBAL, False), (sid_unit, W.LOCAL, False),
                           (sid_unit, W.GLOBAL, True)):
        with pytest.raises(aln.AlnError):
            ctx.plan(sid, ql, ql, mode, W.SEARCH, want_cigar=cig)
    with pytest.raises(aln.AlnError):  # rows beyond the int16 row store
        ctx.plan(sid_unit, np.array([32768], np.int32), ql, W.GLOBAL, W.SEARCH)
    sid_wide = ctx.set_scoring(W.dna_matrix(0, -4), -300, -2)
    with pytest.raises(aln.AlnError):  # gap-affine score rows beyond LDS
        ctx.plan(sid_wide, np.array([2000], np.int32), np.array([2000], np.int32), W.GLOBAL,
                 W.SEARCH)
    with pytest.raises(aln.AlnError):  # longest query + longest reference beyond LDS
        ctx.plan(sid_unit, np.array([30000, 10], np.int32), np.array([10, 30000], np.int32),
                 W.GLOBAL, W.SEARCH)
