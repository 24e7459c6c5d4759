"""GPU parity of the antidiagonal kernel (static band with CIGAR, X-drop
extension with window widening) against the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2607_06225_amd import workloads as W
from tests.parity import compare, oracle_batch

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
    print(f"[gpu] {batch.name} n={batch.n} mode={batch.mode} prune={batch.prune} {kw}",
          flush=True)
    return aln.align(ctx, batch, **kw)


def mutated_pairs(rng, lengths, A, rate=0.1):
    qs, rs = [], []
    st = W.Stream(int(rng.integers(1, 1 << 30)), 9)
    for M, N in lengths:
        ref = rng.integers(0, A, size=N).astype(np.uint8)
        q = W.mutate(ref, rate, 2, 1, 1, A, st)[:M] if M <= N + N // 2 else \
            rng.integers(0, A, size=M).astype(np.uint8)
        if len(q) < M:
            q = np.concatenate([q, rng.integers(0, A, size=M - len(q)).astype(np.uint8)])
        qs.append(q)
        rs.append(ref)
    return qs, rs


BAND_LENGTHS = [(0, 0), (0, 9), (7, 0), (1, 1), (5, 40), (40, 5), (63, 64), (100, 100),
                (129, 127), (300, 290), (500, 520), (700, 640), (1000, 1003), (33, 1000),
                (1000, 33), (2000, 1900), (1500, 1600)]


@pytest.mark.parametrize("mode", [W.GLOBAL, W.LOCAL, W.EXTEND])
@pytest.mark.parametrize("w", [0, 3, 17, 64, 300])
def test_band_edge_shapes_with_cigar(ctx, mode, w):
    rng = np.random.default_rng(1000 + 7 * mode + w)
    qs, rs = mutated_pairs(rng, BAND_LENGTHS, 4)
    b = W.pack_pairs(qs, rs, W.dna_matrix(1, -2), -2, -1, mode, W.BAND, band_w=w,
                     want_cigar=True, name=f"band_w{w}")
    res, cig = run(ctx, b)
    ores = oracle_batch(b)
    assert compare(b, res, cig, ores) == []


def test_band_protein_matrix(ctx):
    rng = np.random.default_rng(77)
    lengths = [(int(rng.integers(50, 400)), int(rng.integers(50, 400))) for _ in range(40)]
    qs, rs = mutated_pairs(rng, lengths, 20, rate=0.3)
    b = W.pack_pairs(qs, rs, W.protein_matrix(5), -11, -1, W.GLOBAL, W.BAND, band_w=40,
                     want_cigar=True, name="band_protein")
    res, cig = run(ctx, b)
    assert compare(b, res, cig, oracle_batch(b)) == []


def test_band_long_reads_sample(ctx):
    """Shortened long-read workload (2-20 kbp, 12% errors, w = 256) with CIGAR."""
    b = W.band_long(n=24, seed=313, min_len=2000, max_len=20000)
    res, cig = run(ctx, b)
    assert compare(b, res, cig, oracle_batch(b, nthreads=8)) == []


def test_band_long_reads_full_size_samples(ctx):
    """Four pairs drawn from the full-size long-read workload (10-100 kbp)."""
    b = W.band_long(n=4, seed=3030)
    res, cig = run(ctx, b)
    assert compare(b, res, cig, oracle_batch(b, nthreads=4)) == []


def xdrop_batch(rng, lengths, X, div=0.15, name="xd"):
    qs, rs = mutated_pairs(rng, lengths, 4, rate=div)
    return W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.EXTEND, W.XDROP, xdrop=X,
                        name=name)


XDROP_TILES = [(4, 1), (8, 4), (4, 16)]  # (window per lane, extension sides per wavefront)


def with_xdrop_tile(ctx, tile):
    ctx.set_tuning({"sw16_rows": 16, "strip_rows": 0, "xdrop_rows": tile[0],
                    "xdrop_sides": tile[1]})


@pytest.mark.parametrize("tile", XDROP_TILES)
@pytest.mark.parametrize("X", [0, 5, 20, 100, 400])
def test_xdrop_edge_shapes(ctx, X, tile):
    with_xdrop_tile(ctx, tile)
    rng = np.random.default_rng(500 + X)
    lengths = [(0, 0), (0, 5), (5, 0), (1, 1), (3, 50), (50, 3)] + \
              [(int(rng.integers(1, 800)), int(rng.integers(1, 800))) for _ in range(60)]
    b = xdrop_batch(rng, lengths, X, name=f"xd_X{X}")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


@pytest.mark.parametrize("tile", XDROP_TILES)
def test_xdrop_identical_and_unrelated(ctx, tile):
    with_xdrop_tile(ctx, tile)
    rng = np.random.default_rng(9)
    qs, rs = [], []
    for L in (10, 200, 1000, 3000):
        x = rng.integers(0, 4, size=L).astype(np.uint8)
        qs.append(x)
        rs.append(x.copy())
        qs.append(rng.integers(0, 4, size=L).astype(np.uint8))
        rs.append(rng.integers(0, 4, size=L).astype(np.uint8))
    b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.EXTEND, W.XDROP, xdrop=100,
                     name="xd_ident")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


@pytest.mark.parametrize("tile", XDROP_TILES)
def test_xdrop_widening_chain(ctx, tile):
    """A huge X keeps whole antidiagonals alive: regions wider than the first
    window, then 1024 diagonals, are recomputed with wider windows (flag
    WIDENED)."""
    from paper_2607_06225_amd import aln
    with_xdrop_tile(ctx, tile)
    rng = np.random.default_rng(10)
    lengths = [(100, 100), (400, 420), (900, 880), (60, 700)]
    b = xdrop_batch(rng, lengths, 10 ** 6, name="xd_wide")
    res, _ = run(ctx, b)
    ores = oracle_batch(b)
    assert compare(b, res, None, ores) == []
    assert int(res["flags"][1]) & aln.F_WIDENED
    assert int(res["flags"][2]) & aln.F_WIDENED


def test_xdrop_too_wide_reported_exactly(ctx):
    """With X far above any score the region is the whole rectangle, whose
    widest antidiagonal spans 2 min(M, N) diagonals.  Past the widest window
    (2042 diagonals) the pair must report TOO_WIDE with F_WIDENED, exactly
    there; every other pair of the batch stays bit-exact."""
    from paper_2607_06225_amd import aln
    with_xdrop_tile(ctx, XDROP_TILES[0])
    rng = np.random.default_rng(12)
    lengths = [(100, 100), (1200, 1200), (900, 880), (1030, 1040), (1021, 1300), (1022, 1022),
               (300, 2500)]
    b = xdrop_batch(rng, lengths, 10 ** 6, name="xd_too_wide")
    res, _ = run(ctx, b)
    wide = [2 * min(M, N) > 2042 for M, N in lengths]
    assert wide == [False, True, False, True, False, True, False]
    for k, w in enumerate(wide):
        if w:
            assert int(res["status"][k]) == aln.R_TOO_WIDE, k
            assert int(res["flags"][k]) & aln.F_WIDENED, k
        else:
            assert int(res["status"][k]) == aln.R_OK, k
    keep = [k for k, w in enumerate(wide) if not w]
    sub = b.subset(keep)
    assert compare(sub, res[keep], None, oracle_batch(sub)) == []


@pytest.mark.parametrize("tile", XDROP_TILES)
def test_xdrop_extension_workload_sample(ctx, tile):
    with_xdrop_tile(ctx, tile)
    b = W.xdrop_ext(n=1500, seed=4040)
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


def test_diag_per_pair_and_graph_match(ctx):
    rng = np.random.default_rng(11)
    qs, rs = mutated_pairs(rng, [(300, 310), (50, 60), (800, 790)], 4)
    for prune, mode, kw in ((W.BAND, W.GLOBAL, dict(band_w=32, want_cigar=True)),
                            (W.XDROP, W.EXTEND, dict(xdrop=50))):
        b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, mode, prune, name="diag_pp", **kw)
        r1, c1 = run(ctx, b)
        r2, c2 = run(ctx, b, per_pair=True)
        r3, c3 = run(ctx, b, graph=True)
        assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
        if c1 is not None:
            assert all(np.array_equal(x, y) for x, y in zip(c1, c2))
            assert all(np.array_equal(x, y) for x, y in zip(c1, c3))
