"""GPU parity of Z-drop extension (the X-drop procedure with the Z-drop
condition of Sec. 9.3) against the CPU oracle: both kernel forms (one
extension per wavefront, four per wavefront), degenerate sizes, pairs with a
long insertion or deletion, window widening, per-pair launches and graph
replay."""
import numpy as np
import pytest

from paper_2607_06225_amd import workloads as W
from tests.parity import compare, oracle_batch

pytestmark = pytest.mark.gpu

TILES = [(4, 1), (8, 4)]  # (diagonals per lane, extension sides per wavefront)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2607_06225_amd import aln
    assert torch.cuda.is_available()
    c = aln.Context(0)
    yield c
    c.close()


def with_tile(ctx, tile):
    ctx.set_tuning({"sw16_rows": 16, "strip_rows": 0, "xdrop_rows": tile[0],
                    "xdrop_sides": tile[1]})


def run(ctx, batch, **kw):
    from paper_2607_06225_amd import aln
    print(f"[gpu] {batch.name} n={batch.n} prune={batch.prune} Z={batch.xdrop} {kw}",
          flush=True)
    return aln.align(ctx, batch, **kw)


def diverged_pairs(rng, lengths, A=4, rate=0.15):
    st = W.Stream(int(rng.integers(1, 1 << 30)), 11)
    qs, rs = [], []
    for M, N in lengths:
        ref = rng.integers(0, A, size=N).astype(np.uint8)
        q = W.mutate(ref, rate, 2, 1, 1, A, st)[:M]
        if len(q) < M:
            q = np.concatenate([q, rng.integers(0, A, size=M - len(q)).astype(np.uint8)])
        qs.append(q)
        rs.append(ref)
    return qs, rs


def indel_pairs(rng, n, div=0.03):
    """Pairs whose query carries one long insertion (or whose reference
    carries one, a deletion) of 10-150 bases part-way along, on top of small
    divergence: the structural-variant case Z-drop is made for."""
    st = W.Stream(int(rng.integers(1, 1 << 30)), 12)
    qs, rs = [], []
    for k in range(n):
        L = int(rng.integers(200, 1500))
        ref = rng.integers(0, 4, size=L).astype(np.uint8)
        q = W.mutate(ref, div, 2, 1, 1, 4, st)
        g = int(rng.integers(10, 151))
        at = int(rng.integers(30, max(31, min(len(q), L) - 30)))
        ins = rng.integers(0, 4, size=g).astype(np.uint8)
        if k % 2 == 0:
            q = np.concatenate([q[:at], ins, q[at:]])
        else:
            ref = np.concatenate([ref[:at], ins, ref[at:]])
        qs.append(q)
        rs.append(ref)
    return qs, rs


def zbatch(qs, rs, Z, prune=W.ZDROP, name="zd"):
    return W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.EXTEND, prune, xdrop=Z,
                        name=name)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("Z", [0, 5, 20, 100, 400])
def test_zdrop_edge_shapes(ctx, Z, tile):
    with_tile(ctx, tile)
    rng = np.random.default_rng(700 + Z)
    lengths = [(0, 0), (0, 5), (5, 0), (1, 1), (3, 50), (50, 3)] + \
              [(int(rng.integers(1, 800)), int(rng.integers(1, 800))) for _ in range(60)]
    qs, rs = diverged_pairs(rng, lengths)
    b = zbatch(qs, rs, Z, name=f"zd_Z{Z}")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


@pytest.mark.parametrize("tile", TILES)
def test_zdrop_identical_and_unrelated(ctx, tile):
    with_tile(ctx, tile)
    rng = np.random.default_rng(19)
    qs, rs = [], []
    for L in (10, 200, 1000, 3000):
        x = rng.integers(0, 4, size=L).astype(np.uint8)
        qs += [x, rng.integers(0, 4, size=L).astype(np.uint8)]
        rs += [x.copy(), rng.integers(0, 4, size=L).astype(np.uint8)]
    b = zbatch(qs, rs, 100, name="zd_ident")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


@pytest.mark.parametrize("tile", TILES)
def test_zdrop_long_indels(ctx, tile):
    """Bit-exact under both rules on pairs with one long gap.  On this seeded
    sample Z-drop visits at least X-drop's cells and scores higher on some
    pairs (a property of the sample, not a theorem: a higher running best can
    also tighten later thresholds)."""
    with_tile(ctx, tile)
    rng = np.random.default_rng(23)
    qs, rs = indel_pairs(rng, 48)
    bz = zbatch(qs, rs, 100, name="zd_indel")
    bx = zbatch(qs, rs, 100, prune=W.XDROP, name="xd_indel")
    rz, _ = run(ctx, bz)
    rx, _ = run(ctx, bx)
    assert compare(bz, rz, None, oracle_batch(bz)) == []
    assert compare(bx, rx, None, oracle_batch(bx)) == []
    assert np.all(rz["cells"] >= rx["cells"])
    assert np.any(rz["score"] > rx["score"])


@pytest.mark.parametrize("tile", TILES)
def test_zdrop_protein_matrix(ctx, tile):
    with_tile(ctx, tile)
    rng = np.random.default_rng(29)
    lengths = [(int(rng.integers(20, 600)), int(rng.integers(20, 600))) for _ in range(40)]
    qs, rs = diverged_pairs(rng, lengths, A=20, rate=0.3)
    b = W.pack_pairs(qs, rs, W.protein_matrix(7), -11, -1, W.EXTEND, W.ZDROP, xdrop=60,
                     name="zd_protein")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


@pytest.mark.parametrize("tile", TILES)
def test_zdrop_widening_chain(ctx, tile):
    """A huge Z keeps whole antidiagonals alive: the region outgrows the first
    window and then 1024 diagonals and is recomputed wider (flag WIDENED)."""
    from paper_2607_06225_amd import aln
    with_tile(ctx, tile)
    rng = np.random.default_rng(31)
    qs, rs = diverged_pairs(rng, [(100, 100), (400, 420), (900, 880), (60, 700)])
    b = zbatch(qs, rs, 10 ** 6, name="zd_wide")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []
    assert int(res["flags"][1]) & aln.F_WIDENED
    assert int(res["flags"][2]) & aln.F_WIDENED


@pytest.mark.parametrize("tile", TILES)
def test_zdrop_extension_workload_sample(ctx, tile):
    with_tile(ctx, tile)
    b = W.zdrop_ext(n=1500, seed=4040)
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


def test_zdrop_per_pair_and_graph_match(ctx):
    rng = np.random.default_rng(37)
    qs, rs = indel_pairs(rng, 6)
    b = zbatch(qs, rs, 80, name="zd_pp")
    r1, _ = run(ctx, b)
    r2, _ = run(ctx, b, per_pair=True)
    r3, _ = run(ctx, b, graph=True)
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
    assert compare(b, r1, None, oracle_batch(b)) == []
