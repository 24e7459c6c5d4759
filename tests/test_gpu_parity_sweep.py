"""Seeded sweep of small mixed batches against the CPU oracle: every pruning
(full matrix, static band, X-drop, Z-drop), every mode the pruning takes, DNA
and protein scorings with and without gap-open costs, scores with and without
CIGARs, each under a random tile choice (packed int16 rows, strip rows and
pipelines, band kernels, X-drop windows), on lengths from empty through short
(one strip, one window) to a few strips and ragged tails.  Each case is one
batch, compared element by element (score, end cell, cell count, status,
begin cell and CIGAR words)."""
import numpy as np
import pytest

from paper_2607_06225_amd import workloads as W
from tests.parity import compare, oracle_batch

pytestmark = pytest.mark.gpu

N_CASES = 128

TILES_X = [(2, 1), (4, 1), (4, 16), (8, 1), (8, 4)]  # (xdrop_rows, xdrop_sides)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2607_06225_amd import aln
    assert torch.cuda.is_available()
    c = aln.Context(0)
    yield c
    c.close()


def lengths(rng, n):
    out = []
    for _ in range(n):
        u = rng.random()
        if u < 0.15:
            out.append(int(rng.integers(0, 8)))
        elif u < 0.6:
            out.append(int(rng.integers(8, 300)))
        else:
            out.append(int(rng.integers(300, 1300)))
    return out


def make_case(seed):
    rng = np.random.default_rng(seed)
    prune = [W.FULL, W.BAND, W.XDROP, W.ZDROP][seed % 4]
    if prune in (W.XDROP, W.ZDROP):
        mode = W.EXTEND
    else:
        mode = [W.GLOBAL, W.LOCAL, W.EXTEND][int(rng.integers(0, 3))]
    if rng.random() < 0.75:
        A = 4
        m = int(rng.choice([1, 2, 5]))
        mat = W.dna_matrix(m, -int(rng.choice([1, 3, 4])))
        go, ge = -int(rng.choice([0, 2, 4, 10])), -int(rng.choice([1, 2]))
    else:
        A = 20
        mat = W.protein_matrix(int(rng.integers(1, 100)))
        go, ge = -11, -1
    n = int(rng.integers(12, 33))
    ms, ns = lengths(rng, n), lengths(rng, n)
    qs, rs = [], []
    st = W.Stream(int(rng.integers(1, 1 << 30)), 3)
    for M, N in zip(ms, ns):
        ref = rng.integers(0, A, size=N).astype(np.uint8)
        if rng.random() < 0.7 and N > 0:  # a relative of the reference, cut or padded to M
            q = W.mutate(ref, float(rng.choice([0.02, 0.1, 0.25])), 2, 1, 1, A, st)[:M]
            if len(q) < M:
                q = np.concatenate([q, rng.integers(0, A, size=M - len(q)).astype(np.uint8)])
        else:
            q = rng.integers(0, A, size=M).astype(np.uint8)
        qs.append(q.astype(np.uint8))
        rs.append(ref)
    band_w = int(rng.choice([0, 1, 7, 40, 127, 128, 300, 2000]))
    xdrop = int(rng.choice([0, 5, 20, 60]))
    cigar = bool(rng.random() < 0.6)
    xr, xs = TILES_X[int(rng.integers(0, len(TILES_X)))]
    tuning = {"sw16_rows": int(rng.choice([4, 8, 12, 16])),
              "strip_rows": int(rng.choice([0, 2, 4, 8, 16, 24, 32])),
              "xdrop_rows": xr, "xdrop_sides": xs,
              "band_kernel": int(rng.integers(0, 6))}
    if tuning["band_kernel"] == 1 and cigar:
        band_w = min(band_w, 128)  # the antidiagonal kernel's CIGAR windows hold 1 018 diagonals
    b = W.pack_pairs(qs, rs, mat, go, ge, mode, prune, band_w=band_w, xdrop=xdrop,
                     want_cigar=cigar, name=f"sweep{seed}")
    return b, tuning


@pytest.mark.parametrize("seed", range(N_CASES))
def test_parity_sweep(ctx, seed):
    from paper_2607_06225_amd import aln
    b, tuning = make_case(7000 + seed)
    print(f"[gpu] sweep seed={7000 + seed} n={b.n} mode={b.mode} prune={b.prune} "
          f"w={b.band_w} x={b.xdrop} cigar={b.want_cigar} tiles={tuning}", flush=True)
    ctx.set_tuning(tuning)
    try:
        res, cig = aln.align(ctx, b)
    finally:
        ctx.set_tuning({"valid": False})
    assert compare(b, res, cig, oracle_batch(b)) == []
