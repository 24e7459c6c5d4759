"""aln_execute_noalloc (the entry point that uses the library's fixed per-GPU
workspace instead of a caller allocation) against aln_execute, through the C
ABI: results and CIGAR words must be identical, on two calls in a row with
the second batch smaller than the first, for each kernel family; a plan whose
workspace exceeds the fixed array is refused with ALN_E_CAPACITY."""
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


def _run_both(ctx, batch):
    """The same plan through aln_execute (caller workspace) and through
    aln_execute_noalloc; returns both (results, cigars)."""
    import torch
    from paper_2607_06225_amd import aln
    sid = ctx.set_scoring(batch.matrix, batch.gap_open, batch.gap_extend)
    plan = ctx.plan(sid, batch.q_len, batch.r_len, batch.mode, batch.prune, batch.band_w,
                    batch.xdrop, aln.W_AUTO, batch.want_cigar)
    assert plan.workspace_bytes <= aln.NOALLOC_WORKSPACE_BYTES, plan.workspace_bytes
    db = aln.DeviceBatch(batch)
    ref = aln.Buffers(plan)
    ctx.execute(plan, db, ref.ws, ref.res, ref.cigar)
    got = aln.Buffers(plan)
    got.res.fill_(0xA5)  # stale bytes must not survive into the results
    ctx.execute_noalloc(plan, db, got.res, got.cigar)
    torch.cuda.synchronize()
    r_ref, r_got = ref.results(batch.n), got.results(batch.n)
    out = (r_ref, ref.cigars(r_ref)), (r_got, got.cigars(r_got))
    plan.close()
    return out


def _same(batch, a, b):
    (ra, ca), (rb, cb) = a, b
    assert np.array_equal(ra, rb), "results differ between aln_execute and aln_execute_noalloc"
    if ca is not None:
        for k in range(batch.n):
            assert np.array_equal(ca[k], cb[k]), f"pair {k}: CIGAR differs"


CASES = [
    ("nw_dna_1k", lambda: W.nw_dna_1k(n=48), lambda b: b.subset(np.arange(9))),
    ("sw_protein", lambda: W.sw_protein(n=600, seed=212), lambda b: b.subset(np.arange(77))),
    ("band_long", lambda: W.band_long(n=6, min_len=2000, max_len=5000, band_w=96),
     lambda b: b.subset(np.arange(2))),
    ("xdrop_ext", lambda: W.xdrop_ext(n=300, max_len=2000), lambda b: b.subset(np.arange(41))),
    ("xdrop_cigar", lambda: W.xdrop_cigar(n=120, max_len=1500), lambda b: b.subset(np.arange(30))),
    ("zdrop_ext", lambda: W.zdrop_ext(n=100, max_len=1500), lambda b: b.subset(np.arange(17))),
    ("edit_search", lambda: W.edit_search(n=256), lambda b: b.subset(np.arange(5))),
]


@pytest.mark.parametrize("name,make,shrink", CASES, ids=[c[0] for c in CASES])
def test_noalloc_matches_execute_twice(ctx, name, make, shrink):
    big = make()
    small = shrink(big)
    assert small.n < big.n
    for k, b in enumerate((big, small)):
        print(f"[gpu] noalloc {name} call {k + 1}: n={b.n}", flush=True)
        ref, got = _run_both(ctx, b)
        _same(b, ref, got)
    # the second (smaller) call also equals the oracle on a sample
    k = min(small.n, 8)
    sub = small.subset(np.arange(k))
    bad = compare(sub, got[0][:k], got[1][:k] if got[1] is not None else None,
                  oracle_batch(sub))
    assert not bad, bad


def test_noalloc_refuses_oversized_plan(ctx):
    from paper_2607_06225_amd import aln
    b = W.nw_dna_1k(n=256)  # 128 MB of traceback codes: beyond the fixed workspace
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    plan = ctx.plan(sid, b.q_len, b.r_len, b.mode, b.prune, 0, 0, aln.W_AUTO, True)
    assert plan.workspace_bytes > aln.NOALLOC_WORKSPACE_BYTES
    db = aln.DeviceBatch(b)
    buf = aln.Buffers(plan)
    with pytest.raises(aln.AlnError, match=r"\(-4\)"):
        ctx.execute_noalloc(plan, db, buf.res, buf.cigar)
    plan.close()
