"""GPU parity of the RNA-folding kernel (the folding recurrence, unpruned or
with X-drop transferred to it) against the CPU oracle, through the C ABI.
Bit-exact: score, best interval, cells and bifurcation terms evaluated and
whether the whole sequence was reached."""
import numpy as np
import pytest

import oracle
from paper_2607_06225_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2607_06225_amd import aln
    assert torch.cuda.is_available()
    c = aln.Context(0)
    yield c
    c.close()


def oracle_fold(fb):
    return oracle.fold_batch(fb.pair, fb.x, fb.off, fb.length, min_loop=fb.min_loop,
                             xdrop=fb.xdrop, warmup=fb.warmup, nthreads=16)


def check(ctx, fb):
    from paper_2607_06225_amd import aln
    print(f"[gpu] fold {fb.name} n={fb.n} max_len={int(fb.length.max()) if fb.n else 0} "
          f"X={fb.xdrop} warmup={fb.warmup} min_loop={fb.min_loop}", flush=True)
    got = aln.fold(ctx, fb)
    exp = oracle_fold(fb)
    bad = []
    for p in range(fb.n):
        g = tuple(int(got[k][p]) for k in ("score", "i", "j", "cells", "terms", "full"))
        e = tuple(int(exp[k][p]) for k in ("score", "i", "j", "cells", "terms", "full"))
        if g != e or int(got["status"][p]) != 0:
            bad.append(f"seq {p} (n={int(fb.length[p])}): gpu {g} status {int(got['status'][p])}"
                       f" oracle {e}")
    assert not bad, bad[:6]
    return got


EDGE = [0, 1, 2, 3, 4, 15, 16, 17, 18, 31, 63, 64, 65, 127, 128, 129, 200, 255, 256, 257, 300,
        401, 402, 403, 480, 500, 507]


def edge_batch(seed, lengths, **kw):
    st = W.Stream(seed, 3)
    xs = [(st.u64(L) & np.uint64(3)).astype(np.uint8) for L in lengths]
    return W.pack_fold(xs, W.rna_pair_table(), name=f"edge{seed}", **kw)


@pytest.mark.parametrize("xdrop", [-1, 0, 2, 5])
@pytest.mark.parametrize("warmup,min_loop", [(15, 3), (0, 0), (15, 0)])
def test_fold_edge_lengths(ctx, xdrop, warmup, min_loop):
    fb = edge_batch(11 + 7 * xdrop + warmup + min_loop, EDGE, min_loop=min_loop, xdrop=xdrop,
                    warmup=warmup)
    check(ctx, fb)


@pytest.mark.parametrize("xdrop", [-1, 1, 3, 40])
def test_fold_weighted_pairs_two_byte_scores(ctx, xdrop):
    """Weights up to 3 per pair push scores of long sequences past one byte:
    the two-byte triangle (and its LDS limit, 383 nt)."""
    P = np.zeros((4, 4), dtype=np.int32)
    for (a, b), w in (((0, 3), 2), ((1, 2), 3), ((2, 3), 1)):
        P[a, b] = P[b, a] = w
    st = W.Stream(77, 4)
    lengths = [5, 60, 170, 171, 250, 255, 256, 333, 382, 383]
    xs = [(st.u64(L) & np.uint64(3)).astype(np.uint8) for L in lengths]
    fb = W.pack_fold(xs, P, min_loop=3, xdrop=xdrop, warmup=15, name="weighted")
    check(ctx, fb)


def test_fold_hairpins_and_unpairable(ctx):
    rng = np.random.default_rng(4)
    comp = np.array([3, 2, 1, 0], dtype=np.uint8)  # A-U, C-G, G-C, U-A
    xs = []
    for k in (8, 40, 150, 250):
        x = rng.integers(0, 4, size=k).astype(np.uint8)
        xs.append(np.concatenate([x, comp[x[::-1]]]))
    xs.append(np.zeros(300, dtype=np.uint8))          # A only: nothing pairs
    xs.append(np.full(77, 1, dtype=np.uint8))          # C only
    fb = W.pack_fold(xs, W.rna_pair_table(), min_loop=0, xdrop=-1, warmup=15, name="hairpin")
    got = check(ctx, fb)
    assert list(got["score"][:4]) == [8, 40, 150, 250]
    assert list(got["score"][4:]) == [0, 0]


@pytest.mark.parametrize("xdrop", [-1, 2])
def test_fold_workload_sample(ctx, xdrop):
    fb = W.rna_fold(n=384, seed=8080, xdrop=xdrop)
    check(ctx, fb)


def test_fold_mixed_classes_in_one_batch(ctx):
    """Short and long sequences in one batch run in several launches (LDS
    classes); results stay in the caller's order."""
    rng = np.random.default_rng(9)
    lengths = list(rng.integers(1, 507, size=120))
    fb = edge_batch(5, lengths, min_loop=3, xdrop=2, warmup=15)
    check(ctx, fb)


def test_fold_bad_symbol(ctx):
    from paper_2607_06225_amd import aln
    xs = [np.array([0, 1, 2, 3], dtype=np.uint8), np.array([0, 4, 1], dtype=np.uint8),
          np.array([2, 2, 1, 1], dtype=np.uint8)]
    fb = W.pack_fold(xs, W.rna_pair_table(), name="bad")
    got = aln.fold(ctx, fb)
    assert list(got["status"]) == [aln.R_OK, aln.R_BAD_SYMBOL, aln.R_OK]
    exp = oracle_fold(fb.subset([0, 2]))
    assert [int(v) for v in got["score"][[0, 2]]] == [int(v) for v in exp["score"]]


def test_fold_limits_refused(ctx):
    """Past 511 nt, or past 383 nt when scores need two bytes, the plan is
    refused with ALN_E_UNSUPPORTED (the triangle would not fit LDS)."""
    from paper_2607_06225_amd import aln
    P = np.zeros((4, 4), dtype=np.int32)
    P[1, 2] = P[2, 1] = 3
    for pair, L in ((W.rna_pair_table(), 512), (P, 384)):
        fb = W.pack_fold([np.zeros(L, dtype=np.uint8)], pair, name="too_long")
        with pytest.raises(aln.AlnError, match=r"\(-5\)"):
            aln.fold_plan(ctx, fb)
