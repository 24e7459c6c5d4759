"""GPU parity of the full-matrix path (strip kernel + traceback walk) against
the CPU oracle, through the C ABI.  Bit-exact: score, end cell, cells, begin
cell and CIGAR words."""
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
    print(f"[gpu] {batch.name} n={batch.n} mode={batch.mode} prune={batch.prune} "
          f"cigar={batch.want_cigar} {kw}", flush=True)
    return aln.align(ctx, batch, **kw)


def edge_batch(matrix, go, ge, mode, want_cigar, seed, lengths, A):
    rng = np.random.default_rng(seed)
    qs, rs = [], []
    for M, N in lengths:
        base = rng.integers(0, A, size=max(M, N)).astype(np.uint8)
        q = base[:M].copy()
        r = base[:N].copy()
        mut = rng.random(N) < 0.2
        r[mut] = rng.integers(0, A, size=int(mut.sum()))
        qs.append(q)
        rs.append(r)
    return W.pack_pairs(qs, rs, matrix, go, ge, mode, W.FULL, want_cigar=want_cigar,
                        name=f"edge_m{mode}_a{A}")


EDGE_LENGTHS = [(0, 0), (0, 7), (5, 0), (1, 1), (1, 70), (70, 1), (2, 3), (63, 64), (64, 63),
                (65, 65), (127, 129), (128, 128), (200, 31), (511, 513), (512, 512),
                (513, 100), (1023, 700), (1024, 1024), (1025, 333), (1536, 90), (1537, 257),
                (2048, 64), (2049, 130), (3000, 77), (4100, 50)]


@pytest.mark.parametrize("mode", [W.GLOBAL, W.LOCAL, W.EXTEND])
@pytest.mark.parametrize("alpha", [4, 20])
def test_full_edge_shapes(ctx, mode, alpha):
    if alpha == 4:
        mat, go, ge = W.dna_matrix(2, -4), -4, -2
    else:
        mat, go, ge = W.protein_matrix(7), -11, -1
    b = edge_batch(mat, go, ge, mode, True, 1000 + 10 * mode + alpha, EDGE_LENGTHS, alpha)
    res, cig = run(ctx, b)
    ores = oracle_batch(b)
    assert compare(b, res, cig, ores) == []


def test_nw_dna_1k_full_config(ctx):
    b = W.nw_dna_1k()
    res, cig = run(ctx, b)
    ores = oracle_batch(b)
    assert compare(b, res, cig, ores) == []


def test_per_pair_and_graph_match_batched(ctx):
    b = W.nw_dna_1k(n=24)
    r1, c1 = run(ctx, b)
    r2, c2 = run(ctx, b, per_pair=True)
    r3, c3 = run(ctx, b, graph=True)
    for r, c in ((r2, c2), (r3, c3)):
        assert np.array_equal(r1, r)
        assert all(np.array_equal(x, y) for x, y in zip(c1, c))


def test_graph_replays_are_identical(ctx):
    import torch
    from paper_2607_06225_amd import aln
    b = W.nw_dna_1k(n=16)
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    plan = ctx.plan(sid, b.q_len, b.r_len, b.mode, b.prune, want_cigar=True)
    db = aln.DeviceBatch(b)
    buf = aln.Buffers(plan)
    s = torch.cuda.Stream()
    ctx.graph_capture(plan, db, buf.ws, buf.res, buf.cigar, stream=s)
    s.synchronize()
    first = buf.results(b.n)
    ores = oracle_batch(b)
    assert compare(b, first, buf.cigars(first), ores) == []
    for _ in range(3):
        buf.res.zero_()
        buf.cigar.zero_()
        torch.cuda.synchronize()
        ctx.graph_launch(plan, stream=s)
        s.synchronize()
        again = buf.results(b.n)
        assert np.array_equal(first, again)
        assert compare(b, again, buf.cigars(again), ores) == []
    plan.close()


def test_bad_symbol_flagged(ctx):
    mat = W.dna_matrix(2, -4)
    qs = [np.array([0, 1, 2], np.uint8), np.array([0, 9, 2], np.uint8)]
    rs = [np.array([0, 1, 2], np.uint8), np.array([0, 1], np.uint8)]
    b = W.pack_pairs(qs, rs, mat, -4, -2, W.GLOBAL, W.FULL, want_cigar=True, name="badsym")
    res, cig = run(ctx, b)
    assert int(res["status"][0]) == 0 and int(res["score"][0]) == 6
    assert int(res["status"][1]) == oracle.BAD_SYMBOL


def test_sw_protein_sample_int32(ctx):
    """A slice of the protein local workload through the int32 strip kernel."""
    from paper_2607_06225_amd import aln
    b = W.sw_protein(n=512)
    res, cig = run(ctx, b, width=aln.W_I32)
    ores = oracle_batch(b)
    assert compare(b, res, cig, ores) == []


@pytest.mark.parametrize("cigar", [False, True])
def test_local_end_ties_across_pipeline_strips(ctx, cigar):
    """Equal best local scores in different 256-row strips, which different
    wavefronts of the strip pipeline evaluate: the end cell is the one with
    the smallest i, then the smallest j."""
    rng = np.random.default_rng(41)
    mat = W.dna_matrix(2, -4)
    qs, rs = [], []
    for gap in (200, 600, 1100):
        x = rng.integers(0, 4, size=100).astype(np.uint8)
        junk = rng.integers(0, 4, size=gap).astype(np.uint8)
        qs.append(np.concatenate([x, junk, x, junk, x]))
        rs.append(np.concatenate([x, rng.integers(0, 4, size=50).astype(np.uint8), x]))
    b = W.pack_pairs(qs, rs, mat, -4, -2, W.LOCAL, W.FULL, want_cigar=cigar, name="ties")
    res, cig = run(ctx, b)
    assert compare(b, res, cig, oracle_batch(b)) == []


@pytest.mark.parametrize("mode", [W.GLOBAL, W.LOCAL])
def test_strip_pipeline_forms(ctx, mode):
    """The strip pipeline (four wavefronts per pair, 4 rows per lane) on
    random shapes above 256 rows, with CIGARs: a few long pairs, and 400
    pairs (still below three quarters of a wavefront per SIMD)."""
    rng = np.random.default_rng(47 + mode)
    few = [(int(rng.integers(257, 2600)), int(rng.integers(1, 1100))) for _ in range(30)]
    many = [(int(rng.integers(257, 1400)), int(rng.integers(1, 600))) for _ in range(400)]
    for lengths in (few, many):
        b = edge_batch(W.dna_matrix(2, -4), -4, -2, mode, True, 4747, lengths, 4)
        res, cig = run(ctx, b)
        assert compare(b, res, cig, oracle_batch(b)) == []


@pytest.mark.parametrize("tile", [2, 4])
@pytest.mark.parametrize("mode", [W.GLOBAL, W.LOCAL, W.EXTEND])
def test_strip_pipeline_protein_tiles(ctx, tile, mode):
    """Both pipeline forms forced by the tuning (eight wavefronts of 2 rows,
    four of 4) on a 20-letter alphabet (query profile in LDS), with CIGARs;
    pairs too short for two strips fall back to one wavefront."""
    from paper_2607_06225_amd import aln
    rng = np.random.default_rng(53 + tile + mode)
    lengths = [(int(rng.integers(100, 1800)), int(rng.integers(1, 900))) for _ in range(40)]
    b = edge_batch(W.protein_matrix(5), -11, -1, mode, True, 5353, lengths, 20)
    ctx.set_tuning({"sw16_rows": 16, "strip_rows": tile, "xdrop_rows": 4})
    try:
        res, cig = run(ctx, b, width=aln.W_I32)
    finally:
        ctx.set_tuning({"valid": False})
    assert compare(b, res, cig, oracle_batch(b)) == []


def test_many_pairs_run_one_wavefront_each(ctx):
    """More full-matrix pairs than three quarters of the SIMDs: the planner
    keeps one wavefront per pair (multi-strip pairs included)."""
    rng = np.random.default_rng(43)
    lengths = [(int(rng.integers(200, 1400)), int(rng.integers(50, 400))) for _ in range(800)]
    b = edge_batch(W.dna_matrix(2, -4), -4, -2, W.GLOBAL, True, 4343, lengths, 4)
    res, cig = run(ctx, b)
    assert compare(b, res, cig, oracle_batch(b)) == []
