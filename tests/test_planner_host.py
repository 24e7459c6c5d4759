"""Host-only tests of the planner through a context without a device
(aln_create_host): which kernel each configuration gets, and an
oracle-backed fake executor that checks the plan's partition of the batch and
its memory layout -- every pair runs exactly once, traceback regions and CIGAR
slots are disjoint, inside the footprint and large enough for the kernel's
layout and for the oracle's CIGAR, and the footprint's cell count is the
oracle's.  Calls that would touch a device are refused after their argument
checks (capacity errors first)."""
import ctypes

import numpy as np
import pytest

from paper_2607_06225_amd import aln
from paper_2607_06225_amd import workloads as W
from tests.parity import oracle_batch


@pytest.fixture(scope="module")
def hctx():
    c = aln.Context.host()
    yield c
    c.close()


def plan_of(ctx, b, want_cigar=None, **over):
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    kw = dict(mode=b.mode, prune=b.prune, band_w=b.band_w, xdrop=b.xdrop)
    kw.update(over)
    wc = b.want_cigar if want_cigar is None else want_cigar
    return ctx.plan(sid, b.q_len, b.r_len, kw["mode"], kw["prune"], kw["band_w"], kw["xdrop"],
                    aln.W_AUTO, wc)


def random_pairs(rng, lengths, A=4, rate=0.1):
    qs, rs = [], []
    st = W.Stream(int(rng.integers(1, 1 << 30)), 5)
    for M, N in lengths:
        ref = rng.integers(0, A, size=N).astype(np.uint8)
        q = W.mutate(ref, rate, 2, 1, 1, A, st)[:M]
        if len(q) < M:
            q = np.concatenate([q, rng.integers(0, A, size=M - len(q)).astype(np.uint8)])
        qs.append(q)
        rs.append(ref)
    return qs, rs


# ------------------------------------------------------------- kernel choice
def families(ctx, b, **kw):
    p = plan_of(ctx, b, **kw)
    L, _ = p.describe()
    p.close()
    return [l["family"] for l in L]


def test_kernel_choice_per_configuration(hctx):
    rng = np.random.default_rng(1)
    qs, rs = random_pairs(rng, [(300, 320), (50, 40), (900, 870)])
    dna = W.dna_matrix(2, -4)

    def pk(prune, mode=W.EXTEND, X=40, matrix=dna, go=-4, ge=-2, cigar=False, w=0):
        return W.pack_pairs(qs, rs, matrix, go, ge, mode, prune, band_w=w, xdrop=X,
                            want_cigar=cigar)

    assert families(hctx, pk(W.FULL, W.LOCAL)) == ["sw16"]
    # full-matrix pairs of several strips, few per SIMD: the four-wavefront
    # band strips with a band past the matrix; a one-strip pair: strip_i32
    assert set(families(hctx, pk(W.FULL, W.GLOBAL))) == {"strip_i32", "band_strip"}
    assert families(hctx, pk(W.BAND, W.GLOBAL, w=20)) == ["diag_band"]
    # wide bands (2w + 1 >= 256) run on strips, four wavefronts per pair
    # ((50, 40) lies wholly inside such bands: the full-matrix strips)
    assert families(hctx, pk(W.BAND, W.GLOBAL, w=127)) == ["strip_i32", "diag_band"]
    assert families(hctx, pk(W.BAND, W.GLOBAL, w=128)) == ["strip_i32", "band_strip"]
    # X-drop: the sixteen-sides kernel where its byte arithmetic holds
    assert families(hctx, pk(W.XDROP, X=131)) == ["xdrop_lanes"]
    assert families(hctx, pk(W.XDROP, X=132)) == ["xdrop"]          # X >= 128 + 2|e|
    assert families(hctx, pk(W.XDROP, X=131, ge=-1)) == ["xdrop"]   # limit 129 at e = -1
    prot = W.protein_matrix(3)
    qp, rp = random_pairs(rng, [(100, 90)], A=20)
    bp = W.pack_pairs(qp, rp, prot, -11, -1, W.EXTEND, W.XDROP, xdrop=30)
    assert families(hctx, bp) == ["xdrop"]                          # not match/mismatch
    assert families(hctx, pk(W.ZDROP)) == ["zdrop"]
    assert families(hctx, pk(W.ZDROP, cigar=True)) == ["zdrop_tb"]
    # the sixteen-sides kernel's Z-drop form when tuned
    hctx.set_tuning(dict(sw16_rows=16, strip_rows=0, xdrop_rows=4, xdrop_sides=16))
    try:
        assert families(hctx, pk(W.ZDROP)) == ["zdrop_lanes"]
    finally:
        hctx.set_tuning({"valid": False})
    assert families(hctx, pk(W.XDROP, cigar=True)) == ["xdrop_lanes_tb"]
    assert families(hctx, pk(W.XDROP, X=200, cigar=True)) == ["xdrop_tb"]
    assert families(hctx, pk(W.ZDROP, cigar=True)) == ["zdrop_tb"]
    e = W.pack_pairs(qs, rs, W.dna_matrix(0, -1), 0, -1, W.GLOBAL, aln.SEARCH)
    assert families(hctx, e) == ["search"]
    a = W.pack_pairs(qs, rs, W.dna_matrix(0, -4), -6, -2, W.GLOBAL, aln.SEARCH)
    assert families(hctx, a) == ["search_affine"]


def test_lanes_kernel_needs_side_lengths_below_2_16(hctx):
    b = W.pack_pairs([np.zeros(65535, np.uint8), np.zeros(10, np.uint8)],
                     [np.zeros(5, np.uint8), np.zeros(10, np.uint8)],
                     W.dna_matrix(2, -4), -4, -2, W.EXTEND, W.XDROP, xdrop=50)
    assert families(hctx, b) == ["xdrop_lanes"]
    b2 = W.pack_pairs([np.zeros(65536, np.uint8)], [np.zeros(5, np.uint8)],
                      W.dna_matrix(2, -4), -4, -2, W.EXTEND, W.XDROP, xdrop=50)
    assert families(hctx, b2) == ["xdrop"]


# ------------------------------------------------- oracle-backed fake executor
def tb_need(family, tile, sides, M, N, w=0):
    """Traceback bytes each kernel's layout writes for a pair (M, N)."""
    nk = M + N + 1
    bases = (nk + 63) // 64 * 64 * 4
    if family == "strip_i32":
        ns = -(-M // (64 * tile))
        return ns * (N + 63) * 64 * (tile // 2)
    if family == "band_strip":  # per strip and lane a window of Lw steps, aligned to a store piece
        ns = -(-M // (64 * tile))
        al = (64 if tile == 2 else 16) * 2 // tile
        span = min(2 * w + 2 + (tile - 1) * N // M, N)
        lw = (span + (al - 1) + al - 1) // al * al
        return ns * 64 * lw * (tile // 2)
    if family == "diag_band":
        return bases + ((M + N) // 2 + 1) * 64 * 8
    if family == "xdrop_lanes_tb":  # its own layout, and room for the one-side pass
        return max(bases + nk * 32, bases + ((M + N) // 2 + 1) * 64 * 2)
    if family in ("xdrop_tb", "zdrop_tb"):
        return bases + ((M + N) // 2 + 1) * 64 * 2
    raise AssertionError(family)


def fake_execute(ctx, b, want_cigar):
    """Plan b, then check the plan the way an executor would use it; the
    oracle stands in for the kernels (its CIGAR lengths and cell counts)."""
    p = plan_of(ctx, b, want_cigar=want_cigar)
    L, T = p.describe()
    # every pair once
    assert sorted(T["pair"].tolist()) == list(range(b.n))
    # every launch runs some of the tasks
    for k, l in enumerate(L):
        ids = np.nonzero(T["launch"] == k)[0]
        assert ids.size > 0
    if want_cigar:
        ores = oracle_batch(b, want_cigar=True)
        lo = T["tb_off"]
        hi = T["tb_off"] + T["tb_bytes"]
        order = np.argsort(lo)
        assert (lo >= 0).all() and (hi <= p.traceback_bytes).all()
        assert (hi[order][:-1] <= lo[order][1:]).all()          # disjoint
        c0, c1 = T["cigar_off"], T["cigar_off"] + T["cigar_cap"]
        order = np.argsort(c0)
        assert (c0 >= 0).all() and (c1 <= p.cigar_words).all()
        assert (c1[order][:-1] <= c0[order][1:]).all()
        for t in T:
            l = L[int(t["launch"])]
            M, N = int(b.q_len[t["pair"]]), int(b.r_len[t["pair"]])
            assert int(t["tb_bytes"]) >= tb_need(l["family"], int(t["tile"]), l["sides"], M, N,
                                                 int(b.band_w))
            assert int(t["cigar_cap"]) >= M + N + 1
            assert int(ores["cigar_len"][t["pair"]]) <= int(t["cigar_cap"])
        assert p.workspace_bytes >= p.traceback_bytes
    else:
        assert p.traceback_bytes == 0 and (T["tb_off"] == -1).all()
    if b.prune in (W.FULL, W.BAND):
        ores = oracle_batch(b, want_cigar=False)
        assert p.cells == int(ores["cells"].sum())
    p.close()
    return L, T


SHAPES = [(0, 0), (0, 7), (7, 0), (1, 1), (5, 40), (40, 5), (63, 64), (300, 290), (700, 640),
          (33, 1000), (1000, 33), (1500, 1600)]


@pytest.mark.parametrize("mode", [W.GLOBAL, W.LOCAL, W.EXTEND])
@pytest.mark.parametrize("cigar", [False, True])
def test_fake_executor_full_matrix(hctx, mode, cigar):
    rng = np.random.default_rng(10 + mode)
    qs, rs = random_pairs(rng, SHAPES)
    b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, mode, W.FULL, want_cigar=cigar)
    fake_execute(hctx, b, cigar)


@pytest.mark.parametrize("w", [0, 3, 17, 64, 300])
@pytest.mark.parametrize("cigar", [False, True])
def test_fake_executor_band(hctx, w, cigar):
    rng = np.random.default_rng(20 + w)
    qs, rs = random_pairs(rng, SHAPES)
    b = W.pack_pairs(qs, rs, W.dna_matrix(1, -2), -2, -1, W.GLOBAL, W.BAND, band_w=w,
                     want_cigar=cigar)
    fake_execute(hctx, b, cigar)


@pytest.mark.parametrize("prune,X", [(W.XDROP, 30), (W.XDROP, 131), (W.XDROP, 400),
                                     (W.ZDROP, 50)])
@pytest.mark.parametrize("cigar", [False, True])
def test_fake_executor_dynamic_pruning(hctx, prune, X, cigar):
    rng = np.random.default_rng(30 + X)
    qs, rs = random_pairs(rng, SHAPES)
    b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.EXTEND, prune, xdrop=X,
                     want_cigar=cigar)
    fake_execute(hctx, b, cigar)


def test_fake_executor_workload_shapes(hctx):
    for b in (W.sw_protein(n=600, seed=3), W.nw_dna_1k(n=12, seed=4), W.xdrop_ext(n=150, seed=5),
              W.band_long(n=2, seed=6, min_len=3000, max_len=6000)):
        fake_execute(hctx, b, False)
        if b.prune != W.FULL or b.mode != W.LOCAL:
            fake_execute(hctx, b, True)


def test_fold_plan_covers_every_sequence_once(hctx):
    fb = W.rna_fold(n=200, seed=9)
    p = aln.fold_plan(hctx, fb)
    L, T = p.describe()
    assert sorted(T["pair"].tolist()) == list(range(fb.n))
    for t in T:
        l = L[int(t["launch"])]
        assert l["family"] == "fold" and l["sides"] in (1, 2)
        assert l["tile"] >= int(fb.length[t["pair"]]) + 1
    assert p.cells == int(sum(int(n) * (int(n) - 1) // 2 for n in fb.length))
    p.close()


# ------------------------------------------- band cells: definition and oracle
def band_cells_by_definition(M, N, w):
    if M == 0 or N == 0:
        return 0
    if w >= max(M, N):
        return M * N
    i = np.arange(1, M + 1, dtype=np.int64)
    c = i * N // M
    lo = np.maximum(1, c - w)
    hi = np.minimum(N, c + w)
    return int(np.clip(hi - lo + 1, 0, None).sum())


@pytest.mark.parametrize("M,N,w", [(100, 100, 5), (100, 37, 5), (37, 100, 5), (1000, 3, 1),
                                   (3, 1000, 1), (640, 700, 64), (5000, 4000, 256),
                                   (4000, 5000, 256), (50, 60, 59), (60, 50, 59), (1, 9, 0),
                                   (9, 1, 0), (257, 1, 300), (2000, 1999, 0)])
def test_band_cells_m_ne_n_footprint_definition_and_oracle(hctx, M, N, w):
    """The footprint's band cells equal a direct count of the band's
    definition (row i keeps floor(iN/M) +- w, interior cells only) and the
    oracle's count, for M != N as well as M = N."""
    rng = np.random.default_rng(M * 7 + N + w)
    qs, rs = random_pairs(rng, [(M, N)])
    b = W.pack_pairs(qs, rs, W.dna_matrix(1, -2), -2, -1, W.GLOBAL, W.BAND, band_w=w)
    p = plan_of(hctx, b)
    ores = oracle_batch(b)
    assert p.cells == band_cells_by_definition(M, N, w) == int(ores["cells"][0])
    p.close()


# ------------------------------------------------- refused without a device
def test_device_calls_refused_after_argument_checks(hctx):
    rng = np.random.default_rng(40)
    qs, rs = random_pairs(rng, [(100, 90), (30, 40)])
    b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.GLOBAL, W.FULL, want_cigar=True)
    p = plan_of(hctx, b)
    lib = hctx.lib
    fake = 1 << 40  # never dereferenced: every check here precedes device access
    batch = aln._Batch(b.n, fake, fake, fake, fake, fake, fake)
    ex = lambda ws_bytes, cig_words: lib.aln_execute(  # noqa: E731
        hctx.handle, p.handle, ctypes.byref(batch), fake, ws_bytes, fake, fake, cig_words, None)
    assert ex(p.workspace_bytes - 1, p.cigar_words) == aln.E_CAPACITY
    assert ex(p.workspace_bytes, p.cigar_words - 1) == aln.E_CAPACITY
    assert ex(p.workspace_bytes, p.cigar_words) == aln.E_DEVICE
    assert lib.aln_execute_per_pair(hctx.handle, p.handle, ctypes.byref(batch), fake,
                                    p.workspace_bytes, fake, fake, p.cigar_words,
                                    None) == aln.E_DEVICE
    assert lib.aln_graph_launch(hctx.handle, p.handle, None) == aln.E_INVAL  # nothing captured
    wrong = aln._Batch(b.n + 1, fake, fake, fake, fake, fake, fake)
    assert lib.aln_execute(hctx.handle, p.handle, ctypes.byref(wrong), fake, p.workspace_bytes,
                           fake, fake, p.cigar_words, None) == aln.E_INVAL
    params = aln._Params(b.mode, b.prune, 0, 0, aln.W_AUTO, 0)
    ql = np.ascontiguousarray(b.q_len, dtype=np.int32)
    rl = np.ascontiguousarray(b.r_len, dtype=np.int32)
    assert lib.aln_autotune(hctx.handle, 0, ctypes.byref(params), ctypes.byref(batch),
                            ql.ctypes.data, rl.ctypes.data, None) == aln.E_DEVICE
    p.close()


def test_plan_errors_on_host_context(hctx):
    rng = np.random.default_rng(41)
    qs, rs = random_pairs(rng, [(100, 90)])
    b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.EXTEND, W.XDROP, xdrop=-1)
    with pytest.raises(aln.AlnError, match=r"\(-1\)"):
        plan_of(hctx, b)
    b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.GLOBAL, W.XDROP, xdrop=10)
    with pytest.raises(aln.AlnError, match=r"\(-1\)"):
        plan_of(hctx, b)
    b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.GLOBAL, W.BAND, band_w=-1)
    with pytest.raises(aln.AlnError, match=r"\(-1\)"):
        plan_of(hctx, b)
    # search needs penalties and GLOBAL without CIGAR
    b = W.pack_pairs(qs, rs, W.dna_matrix(2, -4), -4, -2, W.GLOBAL, aln.SEARCH)
    with pytest.raises(aln.AlnError, match=r"\(-5\)"):
        plan_of(hctx, b)
    # folding limits are planning errors as well
    P = np.zeros((4, 4), dtype=np.int32)
    P[1, 2] = P[2, 1] = 3
    for pair, L in ((W.rna_pair_table(), 512), (P, 384)):
        fb = W.pack_fold([np.zeros(L, dtype=np.uint8)], pair, name="too_long")
        with pytest.raises(aln.AlnError, match=r"\(-5\)"):
            aln.fold_plan(hctx, fb)


def test_empty_batch_plans(hctx):
    b = W.pack_pairs([], [], W.dna_matrix(2, -4), -4, -2, W.GLOBAL, W.FULL)
    p = plan_of(hctx, b)
    L, T = p.describe()
    assert T.size == 0 and p.cells == 0
    p.close()


def test_band_kernel_forced_by_tuning():
    """The tuned band kernel overrides the width rule; pairs the strips cannot
    hold (a strip range beyond 2038 columns) stay on antidiagonal windows."""
    c = aln.Context.host()
    try:
        rng = np.random.default_rng(5)
        qs, rs = random_pairs(rng, [(3000, 3000), (100, 90)])
        base = dict(sw16_rows=16, strip_rows=0, xdrop_rows=4, xdrop_sides=1)

        def fams(w, k):
            c.set_tuning(dict(base, band_kernel=k))
            b = W.pack_pairs(qs, rs, W.dna_matrix(1, -2), -2, -1, W.GLOBAL, W.BAND, band_w=w)
            p = plan_of(c, b)
            L, T = p.describe()
            p.close()
            # a one-strip pair wholly inside the band runs on the full-matrix strips
            return sorted((l["family"], l["sides"]) for l in L if l["family"] != "strip_i32")

        assert fams(20, 1) == [("diag_band", 1)]
        assert fams(20, 2) == [("band_strip", 1)]
        assert fams(20, 3) == [("band_strip", 4)]
        assert fams(20, 4) == [("band_strip", 1)]
        assert fams(20, 5) == [("band_strip", 4)]
        assert fams(300, 1) == [("diag_band", 1)]
        # (3000, 3000) at w = 890 needs 2 * 890 + 2 + 255 + 10 = 2047 ring columns
        assert fams(890, 3) == [("band_strip", 4)]
        assert fams(891, 3) == [("diag_band", 1)]
        # 2 rows a lane: 2 * 954 + 2 + 127 + 10 = 2047
        assert fams(954, 5) == [("band_strip", 4)]
        assert fams(955, 5) == [("diag_band", 1)]
        with pytest.raises(aln.AlnError):
            c.set_tuning(dict(base, band_kernel=6))
    finally:
        c.close()
