"""GPU tests of the autotuner: it times every candidate tile of the kernel
family a batch uses, keeps the fastest, and plans built with any tile stay
bit-exact against the oracle."""
import numpy as np
import pytest

from paper_2607_06225_amd import workloads as W
from tests.parity import compare, oracle_batch

pytestmark = pytest.mark.gpu


@pytest.fixture()
def ctx():
    import torch
    from paper_2607_06225_amd import aln
    assert torch.cuda.is_available()
    c = aln.Context(0)
    yield c
    c.close()


def tune_and_check(ctx, b, family, tiles):
    from paper_2607_06225_amd import aln
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    db = aln.DeviceBatch(b)
    t = ctx.autotune(sid, db, b.mode, b.prune, b.band_w, b.xdrop, want_cigar=b.want_cigar)
    print(f"[gpu] {b.name}: {t}", flush=True)
    assert t["valid"]
    assert t[f"{family}_rows"] in tiles
    assert all(ms != 0.0 for ms in t[f"{family}_ms"].values())
    assert max(t[f"{family}_ms"].values()) > 0
    res, cig = aln.align(ctx, b, scoring_id=sid, dbatch=db)
    assert compare(b, res, cig, oracle_batch(b)) == []
    return t


def test_autotune_packed_sw(ctx):
    t = tune_and_check(ctx, W.sw_protein(n=3000, seed=61), "sw16", (4, 8, 12, 16))
    assert t["sw16_wide_pct"] in (25, 40, 60, 80)


def test_autotune_strips_with_cigar(ctx):
    tune_and_check(ctx, W.nw_dna_1k(n=64, seed=62), "strip", (0, 2, 4, 8, 16, 24, 32))


def test_autotune_xdrop(ctx):
    t = tune_and_check(ctx, W.xdrop_ext(n=3000, seed=63), "xdrop", (4, 8))
    assert (t["xdrop_rows"], t["xdrop_sides"]) in ((4, 1), (4, 16), (8, 1), (8, 4))


@pytest.mark.parametrize("tile,sides", [(2, 1), (8, 1), (8, 4), (4, 16)])
def test_every_xdrop_start_window_is_bit_exact(ctx, tile, sides):
    from paper_2607_06225_amd import aln
    b = W.xdrop_ext(n=1500, seed=70 + tile + sides)
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    ctx.set_tuning({"sw16_rows": 16, "strip_rows": 0, "xdrop_rows": tile, "xdrop_sides": sides})
    res, _ = aln.align(ctx, b, scoring_id=sid)
    assert compare(b, res, None, oracle_batch(b)) == []
    rp, _ = aln.align(ctx, b.subset(np.arange(0, b.n, 37)), scoring_id=sid, per_pair=True)
    rb, _ = aln.align(ctx, b.subset(np.arange(0, b.n, 37)), scoring_id=sid)
    assert np.array_equal(rp, rb)


@pytest.mark.parametrize("tile", [2, 4, 8, 24])
def test_every_fixed_strip_tile_is_bit_exact(ctx, tile):
    from paper_2607_06225_amd import aln
    b = W.nw_dna_1k(n=24, seed=80 + tile)
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    ctx.set_tuning({"sw16_rows": 16, "strip_rows": tile, "xdrop_rows": 4})
    res, cig = aln.align(ctx, b, scoring_id=sid)
    assert compare(b, res, cig, oracle_batch(b)) == []


def test_set_tuning_round_trip_and_validation(ctx):
    from paper_2607_06225_amd import aln
    ctx.set_tuning({"sw16_rows": 8, "strip_rows": 24, "xdrop_rows": 2, "sw16_wide_pct": 150})
    got = ctx.tuning()
    assert got["valid"] and (got["sw16_rows"], got["strip_rows"], got["xdrop_rows"],
                             got["sw16_wide_pct"]) == (8, 24, 2, 150)
    for bad in ({"sw16_rows": 5}, {"strip_rows": 12}, {"xdrop_rows": 16},
                {"xdrop_rows": 4, "xdrop_sides": 4}, {"xdrop_sides": 2},
                {"xdrop_rows": 8, "xdrop_sides": 16},
                {"sw16_wide_pct": -2}, {"sw16_wide_pct": 10001}):
        with pytest.raises(aln.AlnError):
            ctx.set_tuning(dict({"sw16_rows": 16, "strip_rows": 0, "xdrop_rows": 8,
                                 "xdrop_sides": 1}, **bad))


def test_autotune_band_kernel(ctx):
    """Bands: the tuner times the antidiagonal kernel and both strip forms."""
    from paper_2607_06225_amd import aln
    b = W.band_long(n=16, seed=64, min_len=2000, max_len=12000)
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    db = aln.DeviceBatch(b)
    t = ctx.autotune(sid, db, b.mode, b.prune, b.band_w, b.xdrop, want_cigar=True)
    print(f"[gpu] band tuning: {t}", flush=True)
    assert t["valid"] and t["band_kernel"] in (1, 2, 3, 4, 5)
    assert all(ms > 0 for ms in t["band_ms"].values())
    res, cig = aln.align(ctx, b, scoring_id=sid, dbatch=db)
    assert compare(b, res, cig, oracle_batch(b)) == []


def test_tuning_cache_reuses_choice(ctx, tmp_path):
    """A cached choice is applied without timing and plans the same kernels."""
    from paper_2607_06225_amd import aln
    b = W.sw_protein(n=2000, seed=65)
    sid = ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend)
    db = aln.DeviceBatch(b)
    path = str(tmp_path / "tuning.json")
    sc = (b.matrix, b.gap_open, b.gap_extend)
    t1 = ctx.autotune(sid, db, b.mode, b.prune, want_cigar=False, cache=path, scoring=sc)
    assert t1["cached"] is False
    ctx.set_tuning({"valid": False})
    t2 = ctx.autotune(sid, db, b.mode, b.prune, want_cigar=False, cache=path, scoring=sc)
    assert t2["cached"] is True
    for k in ("sw16_rows", "strip_rows", "xdrop_rows", "xdrop_sides", "sw16_wide_pct",
              "band_kernel"):
        assert t1[k] == t2[k], k
    res, _ = aln.align(ctx, b, scoring_id=sid, dbatch=db)
    assert compare(b, res, None, oracle_batch(b)) == []
