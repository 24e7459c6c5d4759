"""GPU parity of the sixteen-sides-per-wavefront X-drop kernel (four lanes
and 64 cells per side and antidiagonal, persistent work queue) against the
CPU oracle: score, end cell and cells evaluated, bit-exact.  Each test also
checks, through the kernel timers, which kernel ran."""
import numpy as np
import pytest

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


def run(ctx, b, expect_lanes=True, **kw):
    """Align with the default tiles; report whether the lanes kernel ran."""
    from paper_2607_06225_amd import aln
    print(f"[gpu] {b.name} n={b.n} X={b.xdrop} {kw}", flush=True)
    ctx.set_tuning({"valid": 0})
    ctx.set_profiling(True)
    try:
        res, cig = aln.align(ctx, b, **kw)
        fams = ctx.kernel_times()
    finally:
        ctx.set_profiling(False)
    if expect_lanes is not None and not kw.get("per_pair"):
        assert ("xdrop_lanes" in fams) == expect_lanes, fams
    return res, cig


def pairs(rng, lengths, rate=0.15, A=4):
    qs, rs = [], []
    st = W.Stream(int(rng.integers(1, 1 << 30)), 9)
    for M, N in lengths:
        ref = rng.integers(0, A, size=N).astype(np.uint8)
        q = W.mutate(ref, rate, 2, 1, 1, A, st)[:M]
        if len(q) < M:
            q = np.concatenate([q, rng.integers(0, A, size=M - len(q)).astype(np.uint8)])
        qs.append(q)
        rs.append(ref)
    return qs, rs


def batch(qs, rs, X, match=2, mismatch=-4, go=-4, ge=-2, A=4, name="lanes"):
    m = np.full((A, A), mismatch, dtype=np.int32)
    np.fill_diagonal(m, match)
    return W.pack_pairs(qs, rs, m, go, ge, W.EXTEND, W.XDROP, xdrop=X, name=name)


EDGE = [(0, 0), (0, 5), (5, 0), (1, 1), (1, 7), (7, 1), (2, 2), (3, 50), (50, 3), (31, 33),
        (64, 64), (65, 63), (127, 129)]


@pytest.mark.parametrize("X", [0, 1, 5, 20, 60, 131])
def test_lanes_edge_shapes(ctx, X):
    """X up to its limit for gap extension -2 (X < 128 + 2|e| = 132)."""
    rng = np.random.default_rng(900 + X)
    lengths = EDGE + [(int(rng.integers(1, 900)), int(rng.integers(1, 900))) for _ in range(80)]
    qs, rs = pairs(rng, lengths)
    b = batch(qs, rs, X, name=f"lanes_X{X}")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


SCORINGS = [  # match, mismatch, gap open, gap extend, X
    (1, -1, 0, -1, 40),
    (1, -3, -5, -2, 20),
    (2, -3, -5, -2, 131),
    (5, -4, -10, -1, 129),
    (100, -100, -20, -1, 129),
    (1, -2, 0, 0, 127),
    (3, 0, -1, -1, 60),
    (-1, -2, -1, -1, 10),
]


@pytest.mark.parametrize("sc", SCORINGS)
def test_lanes_scorings(ctx, sc):
    """Zero gap costs (ties between cells past the matrix edge and the cell
    they came from), zero mismatch, a negative match, byte-edge table values."""
    match, mismatch, go, ge, X = sc
    rng = np.random.default_rng(abs(hash(sc)) % (1 << 31))
    lengths = EDGE + [(int(rng.integers(1, 700)), int(rng.integers(1, 700))) for _ in range(60)]
    qs, rs = pairs(rng, lengths, rate=0.1)
    b = batch(qs, rs, X, match, mismatch, go, ge, name=f"lanes_sc{sc}")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


@pytest.mark.parametrize("A", [1, 2, 3])
def test_lanes_small_alphabets(ctx, A):
    rng = np.random.default_rng(40 + A)
    lengths = [(int(rng.integers(1, 500)), int(rng.integers(1, 500))) for _ in range(50)]
    qs, rs = pairs(rng, lengths, rate=0.2, A=A)
    b = batch(qs, rs, 30, A=A, name=f"lanes_A{A}")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


def test_lanes_window_slides_both_ways(ctx):
    """Long gaps move the surviving region to other diagonals: the window
    slides up (deletions from the query) and down (insertions)."""
    rng = np.random.default_rng(77)
    qs, rs = [], []
    for k in range(60):
        ref = rng.integers(0, 4, size=int(rng.integers(800, 2500))).astype(np.uint8)
        q = ref.copy()
        pos = 100
        while pos < len(q) - 60:
            g = int(rng.integers(3, 25))
            if rng.random() < 0.5:   # deletion from the query
                q = np.concatenate([q[:pos], q[pos + g:]])
            else:                    # insertion into the query
                q = np.concatenate([q[:pos], rng.integers(0, 4, size=g).astype(np.uint8),
                                    q[pos:]])
            pos += int(rng.integers(60, 200))
        sub = rng.random(len(q)) < 0.03
        q[sub] = (q[sub] + 1) % 4
        qs.append(q)
        rs.append(ref)
    for X in (60, 100, 131):
        b = batch(qs, rs, X, name=f"lanes_slide_X{X}")
        res, _ = run(ctx, b)
        assert compare(b, res, None, oracle_batch(b)) == []


@pytest.mark.parametrize("sc", [(1, -1, 0, -1, 129), (1, -2, 0, 0, 127)])
def test_lanes_region_wider_than_window_is_widened(ctx, sc):
    """Identical sequences under cheap gaps with X at its limit keep more
    than 64 cells per antidiagonal once they pass about 100 bases: the pair
    leaves for the wider kernel (flag WIDENED) and stays exact."""
    from paper_2607_06225_amd import aln
    match, mismatch, go, ge, X = sc
    rng = np.random.default_rng(5)
    qs, rs = [], []
    for L in (50, 300, 600, 2000):
        x = rng.integers(0, 4, size=L).astype(np.uint8)
        qs.append(x)
        rs.append(x.copy())
    qs2, rs2 = pairs(rng, [(400, 400)] * 5, rate=0.2)
    b = batch(qs + qs2, rs + rs2, X, match, mismatch, go, ge, name=f"lanes_widen{sc}")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []
    assert not int(res["flags"][0]) & aln.F_WIDENED
    assert all(int(f) & aln.F_WIDENED for f in res["flags"][1:4])


def test_lanes_many_tiny_pairs_and_repeat(ctx):
    """Thousands of tiny and empty pairs through the queue; a second run of
    the same plan (the queue resets itself) and per-pair launches agree."""
    from paper_2607_06225_amd import aln
    rng = np.random.default_rng(6)
    lengths = [(int(rng.integers(0, 9)), int(rng.integers(0, 9))) for _ in range(5000)]
    qs, rs = pairs(rng, lengths, rate=0.3)
    b = batch(qs, rs, 7, name="lanes_tiny")
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    db = aln.DeviceBatch(b)
    r1, _ = run(ctx, b, scoring_id=sid, dbatch=db)
    assert compare(b, r1, None, oracle_batch(b)) == []
    r2, _ = run(ctx, b, scoring_id=sid, dbatch=db)
    assert np.array_equal(r1, r2)
    sub = b.subset(np.arange(0, b.n, 97))
    rp, _ = run(ctx, sub, per_pair=True)
    rb, _ = run(ctx, sub)
    assert np.array_equal(rp, rb)


def test_lanes_bad_symbol(ctx):
    from paper_2607_06225_amd import aln
    rng = np.random.default_rng(8)
    qs, rs = pairs(rng, [(100, 100)] * 6)
    qs[1] = qs[1].copy()
    qs[1][50] = 4
    rs[4] = rs[4].copy()
    rs[4][0] = 9
    b = batch(qs, rs, 40, name="lanes_bad")
    res, _ = run(ctx, b)
    assert [int(s) for s in res["status"]] == [aln.R_OK, aln.R_BAD_SYMBOL, aln.R_OK, aln.R_OK,
                                                aln.R_BAD_SYMBOL, aln.R_OK]
    keep = [0, 2, 3, 5]
    sub = b.subset(keep)
    assert compare(sub, res[keep], None, oracle_batch(sub)) == []


def test_lanes_longest_pairs(ctx):
    """End cells use 16 bits: pairs up to 65535 per side run on the kernel;
    one longer pair sends the whole plan to the one-side kernel."""
    rng = np.random.default_rng(9)
    qs, rs = pairs(rng, [(65535, 65535), (40000, 65535), (65535, 20000), (3000, 3000)],
                   rate=0.02)
    b = batch(qs, rs, 25, name="lanes_long")
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []
    assert int(res["q_end"][0]) > 60000
    qs2, rs2 = pairs(rng, [(65536, 70000), (500, 500)], rate=0.02)
    b2 = batch(qs2, rs2, 25, name="lanes_too_long")
    res2, _ = run(ctx, b2, expect_lanes=False)
    assert compare(b2, res2, None, oracle_batch(b2)) == []


@pytest.mark.parametrize("case", ["x_over_limit", "cigar", "matrix", "zdrop_cigar", "alphabet5"])
def test_lanes_not_used_outside_its_arithmetic(ctx, case):
    """Plans the kernel cannot run exactly go to the one-side kernels."""
    rng = np.random.default_rng(10)
    lengths = [(int(rng.integers(1, 400)), int(rng.integers(1, 400))) for _ in range(40)]
    A = 5 if case == "alphabet5" else 4
    qs, rs = pairs(rng, lengths, rate=0.1, A=A)
    if case == "x_over_limit":
        b = batch(qs, rs, 132, name="lanes_X132")
    elif case == "cigar":
        b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.EXTEND, W.XDROP, xdrop=40,
                         want_cigar=True, name="lanes_cigar")
    elif case == "matrix":
        m = W.dna_matrix(2, -4)
        m[0, 1] = m[1, 0] = -3
        b = W.pack_pairs(qs, rs, m, -4, -2, W.EXTEND, W.XDROP, xdrop=40, name="lanes_mat")
    elif case == "zdrop_cigar":
        b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.EXTEND, W.ZDROP, xdrop=40,
                         want_cigar=True, name="lanes_zdrop_cigar")
    else:
        b = batch(qs, rs, 40, A=5, name="lanes_A5")
    res, cig = run(ctx, b, expect_lanes=False)
    assert compare(b, res, cig, oracle_batch(b)) == []


def run_z(ctx, b):
    """Z-drop scores with the sixteen-sides tile tuned: its Z-drop form runs."""
    from paper_2607_06225_amd import aln
    print(f"[gpu] {b.name} n={b.n} Z={b.xdrop}", flush=True)
    ctx.set_tuning({"sw16_rows": 16, "strip_rows": 0, "xdrop_rows": 4, "xdrop_sides": 16})
    ctx.set_profiling(True)
    try:
        res, _ = aln.align(ctx, b)
        fams = ctx.kernel_times()
    finally:
        ctx.set_profiling(False)
    assert "zdrop_lanes" in fams and "xdrop_lanes" not in fams, fams
    return res


@pytest.mark.parametrize("Z", [0, 3, 25, 100, 400])
def test_lanes_zdrop_matches_oracle(ctx, Z):
    """Z-drop on the sixteen-sides kernel: related and random pairs, lengths
    from 1 to 1 500 (regions wider than its window go on to the wider
    one-side kernels), two gap-open scores.  The extension score stays -2:
    at -1 a gap's cost equals the distance allowance, so a region never
    narrows and long pairs outgrow the widest window."""
    rng = np.random.default_rng(600 + Z)
    lengths = [(int(rng.integers(1, 1500)), int(rng.integers(1, 1500))) for _ in range(60)]
    qs, rs = pairs(rng, lengths, rate=0.12)
    qr = [rng.integers(0, 4, size=M).astype(np.uint8) for M, _ in lengths[:10]]
    for go, ge in ((-4, -2), (0, -2)):
        b = W.pack_pairs(qs + qr, rs + rs[:10], W.dna_matrix(2, -4), go, ge, W.EXTEND, W.ZDROP,
                         xdrop=Z, name=f"lanes_z{Z}_o{go}")
        res = run_z(ctx, b)
        assert compare(b, res, None, oracle_batch(b)) == []


def test_lanes_zdrop_workload_sample(ctx):
    b = W.zdrop_ext(n=4000, seed=4242)
    res = run_z(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


def test_lanes_extension_workload_sample(ctx):
    b = W.xdrop_ext(n=4000, seed=4141)
    res, _ = run(ctx, b)
    assert compare(b, res, None, oracle_batch(b)) == []


# ---------------------------------------------------------------- with CIGAR
def cigar_check(b, res, cig):
    from tests.test_gpu_xdrop_cigar import check
    return check(b, res, cig, oracle_batch(b, want_cigar=True))


def cbatch(qs, rs, X, match=2, mismatch=-4, go=-4, ge=-2, A=4, name="lanes_cigar"):
    m = np.full((A, A), mismatch, dtype=np.int32)
    np.fill_diagonal(m, match)
    return W.pack_pairs(qs, rs, m, go, ge, W.EXTEND, W.XDROP, xdrop=X, want_cigar=True,
                        name=name)


def families(ctx, b, **kw):
    from paper_2607_06225_amd import aln
    ctx.set_tuning({"valid": 0})
    ctx.set_profiling(True)
    try:
        res, cig = aln.align(ctx, b, **kw)
        fams = ctx.kernel_times()
    finally:
        ctx.set_profiling(False)
    return res, cig, fams


@pytest.mark.parametrize("X", [0, 7, 30, 100, 131])
def test_lanes_cigar_edge_shapes(ctx, X):
    rng = np.random.default_rng(1300 + X)
    lengths = EDGE + [(int(rng.integers(1, 900)), int(rng.integers(1, 900))) for _ in range(60)]
    qs, rs = pairs(rng, lengths)
    b = cbatch(qs, rs, X, name=f"lanes_cigar_X{X}")
    res, cig, fams = families(ctx, b)
    assert "xdrop_lanes_tb" in fams, fams
    assert cigar_check(b, res, cig) == []


@pytest.mark.parametrize("sc", SCORINGS)
def test_lanes_cigar_scorings(ctx, sc):
    match, mismatch, go, ge, X = sc
    rng = np.random.default_rng(abs(hash(("c",) + sc)) % (1 << 31))
    lengths = EDGE + [(int(rng.integers(1, 600)), int(rng.integers(1, 600))) for _ in range(40)]
    qs, rs = pairs(rng, lengths, rate=0.1)
    b = cbatch(qs, rs, X, match, mismatch, go, ge, name=f"lanes_cigar_sc{sc}")
    res, cig, fams = families(ctx, b)
    assert "xdrop_lanes_tb" in fams, fams
    assert cigar_check(b, res, cig) == []


def test_lanes_cigar_window_slides(ctx):
    rng = np.random.default_rng(78)
    qs, rs = [], []
    for k in range(40):
        ref = rng.integers(0, 4, size=int(rng.integers(600, 2000))).astype(np.uint8)
        q = ref.copy()
        pos = 80
        while pos < len(q) - 60:
            g = int(rng.integers(3, 25))
            if rng.random() < 0.5:
                q = np.concatenate([q[:pos], q[pos + g:]])
            else:
                q = np.concatenate([q[:pos], rng.integers(0, 4, size=g).astype(np.uint8),
                                    q[pos:]])
            pos += int(rng.integers(60, 200))
        sub = rng.random(len(q)) < 0.03
        q[sub] = (q[sub] + 1) % 4
        qs.append(q)
        rs.append(ref)
    for X in (60, 131):
        b = cbatch(qs, rs, X, name=f"lanes_cigar_slide_X{X}")
        res, cig, _ = families(ctx, b)
        assert cigar_check(b, res, cig) == []


@pytest.mark.parametrize("sc", [(1, -1, 0, -1, 129), (1, -2, 0, 0, 127)])
def test_lanes_cigar_overflow_goes_to_one_side_pass(ctx, sc):
    """Regions wider than 64 cells: the one-side pass recomputes the pair with
    its own codes (CIGAR up to a 250-diagonal span, CIGAR_CAP beyond), the
    rest keep the sixteen-sides kernel's codes; all as the oracle says."""
    from paper_2607_06225_amd import aln
    match, mismatch, go, ge, X = sc
    rng = np.random.default_rng(15)
    qs, rs = [], []
    for L in (50, 300, 600, 1500):
        x = rng.integers(0, 4, size=L).astype(np.uint8)
        qs.append(x)
        rs.append(x.copy())
    qs2, rs2 = pairs(rng, [(400, 400)] * 6, rate=0.2)
    b = cbatch(qs + qs2, rs + rs2, X, match, mismatch, go, ge, name=f"lanes_cigar_ovf{sc}")
    res, cig, fams = families(ctx, b)
    assert "xdrop_lanes_tb" in fams and "xdrop_tb" in fams, fams
    assert cigar_check(b, res, cig) == []
    assert all(int(f) & aln.F_WIDENED for f in res["flags"][1:4])


def test_lanes_cigar_per_pair_and_graph_match(ctx):
    rng = np.random.default_rng(16)
    qs, rs = pairs(rng, [(300, 310), (50, 60), (800, 790), (0, 4), (1, 1)])
    qi = rng.integers(0, 4, size=500).astype(np.uint8)
    qs.append(qi)
    rs.append(qi.copy())
    b = cbatch(qs, rs, 129, 1, -1, 0, -1, name="lanes_cigar_pp")
    r1, c1, _ = families(ctx, b)
    r2, c2, _ = families(ctx, b, per_pair=True)
    r3, c3, _ = families(ctx, b, graph=True)
    assert np.array_equal(r1, r2) and np.array_equal(r1, r3)
    assert all(np.array_equal(x, y) for x, y in zip(c1, c2))
    assert all(np.array_equal(x, y) for x, y in zip(c1, c3))
    assert cigar_check(b, r1, c1) == []


def test_lanes_cigar_workload_sample(ctx):
    b = W.xdrop_ext(n=1200, seed=4242)
    b.want_cigar = True
    res, cig, fams = families(ctx, b)
    assert "xdrop_lanes_tb" in fams, fams
    assert cigar_check(b, res, cig) == []
