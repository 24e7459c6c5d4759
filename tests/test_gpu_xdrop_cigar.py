"""GPU parity of X-drop and Z-drop extension with CIGAR against the CPU
oracle: the score pass (either kernel form), the traceback pass over the
antidiagonals up to the end cell, and the walk.  Score, end cell and cells
are bit-exact for every pair; the CIGAR is bit-exact whenever every
antidiagonal up to the end cell spans at most 250 diagonals of candidates
(the oracle reports that span), and the pair reports CIGAR_CAP otherwise."""
import numpy as np
import pytest

import oracle
from paper_2607_06225_amd import workloads as W
from tests.parity import oracle_batch

pytestmark = pytest.mark.gpu

# (window per lane, extension sides per wavefront): for X-drop, (4, 16) is the
# sixteen-sides kernel writing 32-byte codes per antidiagonal, the others the
# one-side pass with codes; Z-drop always takes the one-side pass
TILES = [(4, 1), (8, 4), (4, 16)]
WINDOW_SPAN = 250          # widest candidate span the traceback window holds


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
    print(f"[gpu] {batch.name} n={batch.n} prune={batch.prune} X={batch.xdrop} cigar {kw}",
          flush=True)
    return aln.align(ctx, batch, **kw)


def check(batch, res, cig, ores):
    """Mismatch descriptions (empty when every pair meets the contract)."""
    bad = []
    for p in range(batch.n):
        g = res[p]
        exp = (int(ores["score"][p]), int(ores["q_end"][p]), int(ores["r_end"][p]),
               int(ores["cells"][p]))
        got = (int(g["score"]), int(g["q_end"]), int(g["r_end"]), int(g["cells"]))
        if exp != got:
            bad.append(f"pair {p}: gpu {got} oracle {exp}")
            continue
        wide = int(ores["span"][p]) > WINDOW_SPAN
        want = oracle.CIGAR_CAP if wide else int(ores["status"][p])
        if int(g["status"]) != want:
            bad.append(f"pair {p}: status gpu {int(g['status'])} want {want} "
                       f"(span {int(ores['span'][p])})")
            continue
        if want == oracle.OK:
            oc = ores["cigar"][ores["cigar_off"][p]: ores["cigar_off"][p] + ores["cigar_len"][p]]
            if not np.array_equal(np.asarray(oc, np.uint32), np.asarray(cig[p], np.uint32)):
                bad.append(f"pair {p} (M={batch.q_len[p]}, N={batch.r_len[p]}): cigar differs")
            if (int(g["q_begin"]), int(g["r_begin"])) != (0, 0):
                bad.append(f"pair {p}: begin {(int(g['q_begin']), int(g['r_begin']))}")
        if len(bad) >= 8:
            break
    return bad


def diverged_pairs(rng, lengths, A=4, rate=0.15):
    st = W.Stream(int(rng.integers(1, 1 << 30)), 13)
    qs, rs = [], []
    for M, N in lengths:
        ref = rng.integers(0, A, size=N).astype(np.uint8)
        q = W.mutate(ref, rate, 2, 1, 1, A, st)[:M]
        if len(q) < M:
            q = np.concatenate([q, rng.integers(0, A, size=M - len(q)).astype(np.uint8)])
        qs.append(q)
        rs.append(ref)
    return qs, rs


def cbatch(qs, rs, X, prune, name, matrix=None, go=-4, ge=-2):
    m = W.dna_matrix(2, -4) if matrix is None else matrix
    return W.pack_pairs(qs, rs, m, go, ge, W.EXTEND, prune, xdrop=X, want_cigar=True,
                        name=name)


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("prune", [W.XDROP, W.ZDROP])
@pytest.mark.parametrize("X", [0, 7, 30, 100])
def test_dynamic_prune_cigar_edge_shapes(ctx, X, prune, tile):
    with_tile(ctx, tile)
    rng = np.random.default_rng(800 + X + 7 * prune)
    lengths = [(0, 0), (0, 5), (5, 0), (1, 1), (3, 50), (50, 3), (2, 2)] + \
              [(int(rng.integers(1, 900)), int(rng.integers(1, 900))) for _ in range(50)]
    qs, rs = diverged_pairs(rng, lengths)
    b = cbatch(qs, rs, X, prune, f"xc_{prune}_{X}")
    res, cig = run(ctx, b)
    assert check(b, res, cig, oracle_batch(b)) == []


@pytest.mark.parametrize("prune", [W.XDROP, W.ZDROP])
def test_dynamic_prune_cigar_long_indels_and_protein(ctx, prune):
    rng = np.random.default_rng(61 + prune)
    st = W.Stream(61, 14)
    qs, rs = [], []
    for k in range(40):
        L = int(rng.integers(200, 2500))
        ref = rng.integers(0, 4, size=L).astype(np.uint8)
        q = W.mutate(ref, 0.04, 2, 1, 1, 4, st)
        g = int(rng.integers(10, 120))
        at = int(rng.integers(20, max(21, min(len(q), L) - 20)))
        ins = rng.integers(0, 4, size=g).astype(np.uint8)
        if k % 2:
            q = np.concatenate([q[:at], ins, q[at:]])
        else:
            ref = np.concatenate([ref[:at], ins, ref[at:]])
        qs.append(q)
        rs.append(ref)
    b = cbatch(qs, rs, 100, prune, "xc_indel")
    res, cig = run(ctx, b)
    assert check(b, res, cig, oracle_batch(b)) == []
    lengths = [(int(rng.integers(20, 500)), int(rng.integers(20, 500))) for _ in range(30)]
    qs, rs = diverged_pairs(rng, lengths, A=20, rate=0.3)
    bp = cbatch(qs, rs, 60, prune, "xc_protein", matrix=W.protein_matrix(7), go=-11, ge=-1)
    res, cig = run(ctx, bp)
    assert check(bp, res, cig, oracle_batch(bp)) == []


def test_dynamic_prune_cigar_wide_regions(ctx):
    """Huge thresholds: regions wider than the traceback window report
    CIGAR_CAP (score, end cell and cells exact); narrower ones are exact."""
    from paper_2607_06225_amd import aln
    rng = np.random.default_rng(67)
    qs, rs = diverged_pairs(rng, [(100, 100), (400, 420), (900, 880), (60, 700), (300, 40)])
    for prune in (W.XDROP, W.ZDROP):
        b = cbatch(qs, rs, 10 ** 6, prune, "xc_wide")
        res, cig = run(ctx, b)
        ores = oracle_batch(b)
        assert check(b, res, cig, ores) == []
        assert int(res["status"][2]) == aln.R_CIGAR_CAP
        assert int(res["status"][0]) == aln.R_OK


@pytest.mark.parametrize("tile", TILES)
def test_dynamic_prune_cigar_workload_sample(ctx, tile):
    with_tile(ctx, tile)
    b = W.xdrop_ext(n=800, seed=4041)
    b.want_cigar = True
    res, cig = run(ctx, b)
    ores = oracle_batch(b)
    assert check(b, res, cig, ores) == []
    assert int((res["status"] == 0).sum()) > 0.9 * b.n


def test_dynamic_prune_cigar_per_pair_and_graph_match(ctx):
    rng = np.random.default_rng(71)
    qs, rs = diverged_pairs(rng, [(300, 310), (50, 60), (800, 790), (120, 20)])
    b = cbatch(qs, rs, 50, W.XDROP, "xc_pp")
    r1, c1 = run(ctx, b)
    r2, c2 = run(ctx, b, per_pair=True)
    r3, c3 = run(ctx, b, graph=True)
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
    assert all(np.array_equal(x, y) for x, y in zip(c1, c2))
    assert all(np.array_equal(x, y) for x, y in zip(c1, c3))
    assert check(b, r1, c1, oracle_batch(b)) == []
