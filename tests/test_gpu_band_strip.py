"""GPU parity of the static band on strips (scores, end cells, cell counts and
CIGARs) against the CPU oracle, with each band kernel forced through the
tuning: 1 antidiagonal windows; strips of 4 rows per lane with one (2) or four
(3) wavefronts per pair; strips of 2 rows per lane with one (4) or four (5)."""
import numpy as np
import pytest

from paper_2607_06225_amd import workloads as W
from tests.parity import compare, oracle_batch

pytestmark = pytest.mark.gpu

KERNELS = [2, 3, 4, 5]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2607_06225_amd import aln
    assert torch.cuda.is_available()
    c = aln.Context(0)
    yield c
    c.close()


def with_band_kernel(ctx, k):
    ctx.set_tuning({"sw16_rows": 16, "strip_rows": 0, "xdrop_rows": 4, "xdrop_sides": 1,
                    "band_kernel": k})


def families(ctx, b):
    from paper_2607_06225_amd import aln
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    p = ctx.plan(sid, b.q_len, b.r_len, b.mode, b.prune, b.band_w, b.xdrop, aln.W_AUTO,
                 b.want_cigar)
    L, _ = p.describe()
    p.close()
    return sorted({(l["family"], l["sides"]) for l in L})


def run(ctx, batch, **kw):
    from paper_2607_06225_amd import aln
    print(f"[gpu] {batch.name} n={batch.n} mode={batch.mode} w={batch.band_w} {kw}", flush=True)
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


# shapes spanning one and several 256-row strips, ragged tails, elongated
# rectangles both ways (bands that leave the matrix, unreachable corners)
SHAPES = [(0, 0), (0, 9), (7, 0), (1, 1), (5, 40), (40, 5), (63, 64), (100, 100), (255, 256),
          (256, 255), (257, 300), (300, 290), (513, 520), (700, 640), (1000, 1003), (33, 1000),
          (1000, 33), (2000, 1900), (1500, 1600), (3000, 3100), (1024, 1024), (4000, 1000)]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("mode", [W.GLOBAL, W.LOCAL, W.EXTEND])
@pytest.mark.parametrize("w", [0, 3, 17, 64, 300, 700])
def test_strip_band_edge_shapes_with_cigar(ctx, kernel, mode, w):
    rng = np.random.default_rng(2000 + 11 * mode + w + kernel)
    qs, rs = mutated_pairs(rng, SHAPES, 4)
    b = W.pack_pairs(qs, rs, W.dna_matrix(1, -2), -2, -1, mode, W.BAND, band_w=w,
                     want_cigar=True, name=f"sband_w{w}_k{kernel}")
    with_band_kernel(ctx, kernel)
    fam = families(ctx, b)
    assert ("band_strip", 1 if kernel in (2, 4) else 4) in fam
    res, cig = run(ctx, b)
    assert compare(b, res, cig, oracle_batch(b)) == []


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("mode", [W.GLOBAL, W.LOCAL, W.EXTEND])
def test_strip_band_scores_only(ctx, kernel, mode):
    rng = np.random.default_rng(2100 + mode + kernel)
    qs, rs = mutated_pairs(rng, SHAPES, 4, rate=0.2)
    sc = [(W.dna_matrix(2, -4), -4, -2), (W.dna_matrix(1, -1), 0, -1), (W.dna_matrix(5, -3), -10, -1)]
    for k, (mat, go, ge) in enumerate(sc):
        b = W.pack_pairs(qs, rs, mat, go, ge, mode, W.BAND, band_w=[40, 130, 257][k],
                         want_cigar=False, name=f"sband_scores{k}")
        with_band_kernel(ctx, kernel)
        res, _ = run(ctx, b)
        assert compare(b, res, None, oracle_batch(b)) == []


@pytest.mark.parametrize("kernel", KERNELS)
def test_strip_band_protein_matrix(ctx, kernel):
    rng = np.random.default_rng(77 + kernel)
    lengths = [(int(rng.integers(50, 1400)), int(rng.integers(50, 1400))) for _ in range(40)]
    qs, rs = mutated_pairs(rng, lengths, 20, rate=0.3)
    for mode in (W.GLOBAL, W.LOCAL):
        b = W.pack_pairs(qs, rs, W.protein_matrix(5), -11, -1, mode, W.BAND, band_w=150,
                         want_cigar=True, name="sband_protein")
        with_band_kernel(ctx, kernel)
        res, cig = run(ctx, b)
        assert compare(b, res, cig, oracle_batch(b)) == []


@pytest.mark.parametrize("kernel", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("mode", [W.GLOBAL, W.LOCAL, W.EXTEND])
def test_strip_band_path_through_column_zero(ctx, kernel, mode):
    """Queries that are k unmatched letters and then the reference: the best
    path leaves column 0 at row k, so row k + 1 takes its diagonal from
    H(k, 0); k = 2 and 4 put that row on lane 1 of the 2- and 4-row strips."""
    rng = np.random.default_rng(4100 + 7 * mode + kernel)
    qs, rs = [], []
    for k in (1, 2, 3, 4, 5, 8):
        for N in (40, 300):
            ref = rng.integers(0, 3, size=N).astype(np.uint8)  # letters 0..2
            qs.append(np.concatenate([np.full(k, 3, np.uint8), ref]))
            rs.append(ref)
    b = W.pack_pairs(qs, rs, W.dna_matrix(5, -3), -10, -1, mode, W.BAND, band_w=20,
                     want_cigar=True, name=f"sband_col0_k{kernel}")
    with_band_kernel(ctx, kernel)
    res, cig = run(ctx, b)
    assert compare(b, res, cig, oracle_batch(b)) == []


@pytest.mark.parametrize("kernel,wmax", [(3, 890), (5, 954)])
def test_strip_band_widest_ring(ctx, kernel, wmax):
    """Bands whose strip range needs the largest ring (2048 columns) run on
    strips; one column more goes to the antidiagonal kernel."""
    rng = np.random.default_rng(91)
    qs, rs = mutated_pairs(rng, [(2600, 2600), (3000, 2900), (700, 650)], 4)
    with_band_kernel(ctx, kernel)
    # (2600, 2600): 2w + 2 + 64R - 1 columns, plus 10, fit 2048 up to w = 890
    # (R = 4) or 954 (R = 2); the antidiagonal fallback one wider has no
    # CIGAR form that wide
    for w, fam, cigar in ((wmax, "band_strip", True), (wmax + 1, "diag_band", False)):
        b = W.pack_pairs(qs, rs, W.dna_matrix(1, -2), -2, -1, W.GLOBAL, W.BAND, band_w=w,
                         want_cigar=cigar, name=f"sband_ring_w{w}")
        got = [f for f, _ in families(ctx, b)]
        assert fam in got
        res, cig = run(ctx, b)
        assert compare(b, res, cig if cigar else None, oracle_batch(b)) == []


@pytest.mark.parametrize("kernel", [1, 2, 3, 4, 5])
def test_band_long_reads_sample_each_kernel(ctx, kernel):
    """Shortened long-read workload (2-20 kbp, 12% errors, w = 256) with CIGAR."""
    b = W.band_long(n=24, seed=313 + kernel, min_len=2000, max_len=20000)
    with_band_kernel(ctx, kernel)
    res, cig = run(ctx, b)
    assert compare(b, res, cig, oracle_batch(b, nthreads=8)) == []


def test_strip_band_per_pair_and_graph_match(ctx):
    rng = np.random.default_rng(12)
    qs, rs = mutated_pairs(rng, [(3000, 3100), (50, 60), (800, 790), (1200, 1000)], 4)
    for kernel in KERNELS:
        with_band_kernel(ctx, kernel)
        b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.GLOBAL, W.BAND, band_w=200,
                         want_cigar=True, name="sband_pp")
        r1, c1 = run(ctx, b)
        r2, c2 = run(ctx, b, per_pair=True)
        r3, c3 = run(ctx, b, graph=True)
        assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
        assert all(np.array_equal(x, y) for x, y in zip(c1, c2))
        assert all(np.array_equal(x, y) for x, y in zip(c1, c3))
        assert compare(b, r1, c1, oracle_batch(b)) == []


def test_band_kernel_tuning_roundtrip(ctx):
    with_band_kernel(ctx, 2)
    assert ctx.tuning()["band_kernel"] == 2
    with pytest.raises(Exception):
        ctx.set_tuning({"sw16_rows": 16, "strip_rows": 0, "xdrop_rows": 4, "xdrop_sides": 1,
                        "band_kernel": 6})
    ctx.set_tuning({"valid": False})
