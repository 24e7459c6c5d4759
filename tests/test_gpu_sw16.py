"""GPU parity of the packed-int16 Smith-Waterman path (two pairs per lane,
int32 re-run of pairs that may saturate) against the CPU oracle."""
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
    print(f"[gpu] {batch.name} n={batch.n} {kw}", flush=True)
    return aln.align(ctx, batch, **kw)


def local_batch(matrix, go, ge, lengths, A, seed, ident=0.6, name="sw16_edge"):
    rng = np.random.default_rng(seed)
    qs, rs = [], []
    for M, N in lengths:
        base = rng.integers(0, A, size=max(M, N, 1)).astype(np.uint8)
        q = base[:M].copy()
        r = base[:N].copy()
        mut = rng.random(N) > ident
        r[mut] = rng.integers(0, A, size=int(mut.sum()))
        qs.append(q)
        rs.append(r)
    return W.pack_pairs(qs, rs, matrix, go, ge, W.LOCAL, W.FULL, name=name)


EDGE = [1, 2, 15, 16, 17, 127, 128, 129, 255, 256, 257, 383, 384, 385, 700, 1000, 2000]


@pytest.mark.parametrize("alpha", [4, 20])
def test_sw16_edge_shapes(ctx, alpha):
    rng = np.random.default_rng(5 + alpha)
    lengths = [(int(rng.choice(EDGE)), int(rng.choice(EDGE))) for _ in range(151)]
    lengths += [(0, 5), (5, 0), (0, 0)]
    if alpha == 4:
        mat, go, ge = W.dna_matrix(2, -4), -4, -2
    else:
        mat, go, ge = W.protein_matrix(11), -11, -1
    b = local_batch(mat, go, ge, lengths, alpha, 77 + alpha)
    res, _ = run(ctx, b)
    ores = oracle_batch(b)
    assert compare(b, res, None, ores) == []
    assert not np.any(res["flags"] & 1)


def test_sw16_protein_sample(ctx):
    b = W.sw_protein(n=4096, seed=909)
    res, _ = run(ctx, b)
    ores = oracle_batch(b)
    assert compare(b, res, None, ores) == []


def test_sw16_forced_overflow_reruns_in_int32(ctx):
    """Scores beyond int16: identical sequences with a large diagonal reach
    120 * L; such pairs are flagged and recomputed in int32."""
    mat = np.full((4, 4), -100, np.int32)
    np.fill_diagonal(mat, 120)
    rng = np.random.default_rng(3)
    qs, rs = [], []
    for L in (50, 250, 272, 273, 274, 300, 1000):
        x = rng.integers(0, 4, size=L).astype(np.uint8)
        qs.append(x)
        rs.append(x.copy())
    for _ in range(9):  # ordinary pairs sharing the launch
        qs.append(rng.integers(0, 4, size=200).astype(np.uint8))
        rs.append(rng.integers(0, 4, size=180).astype(np.uint8))
    b = W.pack_pairs(qs, rs, mat, -30, -5, W.LOCAL, W.FULL, name="sw16_overflow")
    res, _ = run(ctx, b)
    ores = oracle_batch(b)
    assert compare(b, res, None, ores) == []
    thresh = 32767 - 120
    for k in range(b.n):
        expect_flag = int(ores["score"][k]) >= thresh
        assert bool(res["flags"][k] & 1) == expect_flag, (k, int(ores["score"][k]))
    assert int(res["score"][6]) == 120 * 1000


def test_sw16_matches_int32_and_per_pair(ctx):
    from paper_2607_06225_amd import aln
    b = W.sw_protein(n=300, seed=31)
    r16, _ = run(ctx, b)
    r32, _ = run(ctx, b, width=aln.W_I32)
    rpp, _ = run(ctx, b, per_pair=True)
    rg, _ = run(ctx, b, graph=True)
    for r in (r32, rpp, rg):
        for k in ("score", "q_end", "r_end", "cells", "status"):
            assert np.array_equal(r16[k], r[k]), k


def test_sw16_graph_replays(ctx):
    import torch
    from paper_2607_06225_amd import aln
    b = W.sw_protein(n=200, seed=41)
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    plan = ctx.plan(sid, b.q_len, b.r_len, b.mode, b.prune)
    db = aln.DeviceBatch(b)
    buf = aln.Buffers(plan)
    s = torch.cuda.Stream()
    ctx.graph_capture(plan, db, buf.ws, buf.res, None, stream=s)
    s.synchronize()
    first = buf.results(b.n)
    ores = oracle_batch(b)
    assert compare(b, first, None, ores) == []
    for _ in range(3):
        buf.res.zero_()
        torch.cuda.synchronize()
        ctx.graph_launch(plan, stream=s)
        s.synchronize()
        assert np.array_equal(first, buf.results(b.n))
    plan.close()


def test_sw16_bad_symbol(ctx):
    mat = W.protein_matrix(2)
    qs = [np.array([1, 2, 3, 4], np.uint8), np.array([1, 25, 3], np.uint8)]
    rs = [np.array([1, 2, 3, 4], np.uint8), np.array([1, 2, 3], np.uint8)]
    b = W.pack_pairs(qs, rs, mat, -11, -1, W.LOCAL, W.FULL, name="sw16_bad")
    res, _ = run(ctx, b)
    ores = oracle_batch(b)
    assert int(res["status"][1]) == oracle.BAD_SYMBOL
    assert compare(b, res, None, ores) == []


@pytest.mark.parametrize("rows", [4, 8, 12, 16])
def test_sw16_every_row_tile_is_bit_exact(ctx, rows, monkeypatch):
    """Every rows-per-lane tile the tuner may pick gives the oracle's bytes."""
    monkeypatch.setenv("ALN_SW16_ROWS", str(rows))
    b = W.sw_protein(n=700, seed=100 + rows)
    res, _ = run(ctx, b)
    ores = oracle_batch(b)
    assert compare(b, res, None, ores) == []


EDGE_W = [1, 63, 64, 65, 255, 256, 257, 700, 1023, 1024, 1025, 1536, 2000]


@pytest.mark.parametrize("rows", [4, 16])
@pytest.mark.parametrize("wide_pct", [-1, 1, 0])
def test_sw16_narrow_and_wide_items_are_bit_exact(ctx, rows, wide_pct):
    """Work items on four 16-lane groups (wide_pct -1: every item), on one
    64-lane wavefront (wide_pct 1: every long task) and the planner's mix
    give the oracle's results, over lengths at and around the strip heights
    of both forms; per-pair launches (always wide) agree."""
    rng = np.random.default_rng(900 + rows)
    lengths = [(int(rng.choice(EDGE_W)), int(rng.choice(EDGE_W))) for _ in range(61)]
    lengths += [(2000, 2000), (1025, 3), (3, 1025), (1, 1), (0, 7)]
    b = local_batch(W.protein_matrix(11), -11, -1, lengths, 20, 950 + rows, name="sw16_items")
    ctx.set_tuning({"sw16_rows": rows, "strip_rows": 0, "xdrop_rows": 4, "sw16_wide_pct": wide_pct})
    try:
        res, _ = run(ctx, b)
        assert compare(b, res, None, oracle_batch(b)) == []
        sub = b.subset(np.arange(0, b.n, 5))
        rpp, _ = run(ctx, sub, per_pair=True)
        rb, _ = run(ctx, sub)
        for k in ("score", "q_end", "r_end", "cells", "status"):
            assert np.array_equal(rpp[k], rb[k]), k
    finally:
        ctx.set_tuning({"valid": False})
