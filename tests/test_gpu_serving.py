"""GPU tests of the continuous-batching server: every result equals the
oracle's and is the same when the request runs alone as when it shares
micro-batches with a mix; admission waits for device memory; micro-batches
overlap on the device."""
import numpy as np
import pytest

from paper_2607_06225_amd import workloads as W
from tests.parity import compare, oracle_batch

pytestmark = pytest.mark.gpu

FIELDS = ("score", "q_end", "r_end", "q_begin", "r_begin", "status", "flags", "cigar_len",
          "cells", "error")


@pytest.fixture(scope="module")
def mix():
    """320 requests of the serving mix with long reads shortened to 1-10 kbp."""
    arrival, kinds, batches = W.serving_requests(320, qps=4000.0, seed=5150, scale_long=0.1)
    return arrival, kinds, batches


def make_ctx(batches):
    import torch
    from paper_2607_06225_amd import aln
    assert torch.cuda.is_available()
    ctx = aln.Context(0)
    sids = [ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend) for b in batches]
    return ctx, sids


def oracle_check(reqs, comps, cigs, batches):
    """Compare each completion with the oracle run on its own batch."""
    for k, b in enumerate(batches):
        idx = [i for i, rq in enumerate(reqs) if rq["kind"] == k]
        if not idx:
            continue
        pairs = [reqs[i]["pair"] for i in idx]
        sub = b.subset(pairs)
        ores = oracle_batch(sub)
        res = comps[idx]
        bad = compare(sub, res, [cigs[i] if cigs[i] is not None else np.zeros(0, np.uint32)
                                 for i in idx] if b.want_cigar else None, ores)
        assert bad == [], (k, bad)


def test_results_identical_alone_and_in_mix(mix):
    from paper_2607_06225_amd import aln, serving
    arrival, kinds, batches = mix
    ctx, sids = make_ctx(batches)
    reqs = serving.mixed_requests(batches, kinds, sids)
    print(f"[gpu] serving mix of {len(reqs)} requests, kinds {np.bincount(kinds)}", flush=True)

    alone_srv = aln.Server(ctx, streams=1, max_batch_pairs=1, hbm_budget=1 << 30)
    alone, alone_cig, _, _ = serving.replay(alone_srv, reqs, one_at_a_time=True)
    st_alone = alone_srv.stats()
    alone_srv.close()
    assert st_alone["batches"] == len(reqs)
    assert np.all(alone["batch_pairs"] == 1)

    srv = aln.Server(ctx, streams=4, max_batch_pairs=64, hbm_budget=1 << 30)
    mixed, mixed_cig, wall, lat = serving.replay(srv, reqs, arrival)
    st = srv.stats()
    srv.close()
    print(f"[gpu] mix: {st} wall {wall:.3f} s {serving.percentiles(lat)}", flush=True)
    assert st["completed"] == len(reqs)
    assert st["batches"] < len(reqs)          # requests were batched
    assert mixed["batch_pairs"].max() > 1
    for f in FIELDS:
        assert np.array_equal(alone[f], mixed[f]), f
    for a, b in zip(alone_cig, mixed_cig):
        assert (a is None) == (b is None)
        if a is not None:
            assert np.array_equal(a, b)
    assert np.all(mixed["error"] == 0)
    oracle_check(reqs, mixed, mixed_cig, batches)
    ctx.close()


def test_admission_waits_for_memory(mix):
    """Long-read requests only (1-10 kbp, band 256, CIGAR: up to ~5 MB of
    traceback codes each) against a 12 MiB budget with four streams for the
    class: ready micro-batches must wait for memory, the budget is never
    exceeded and the results stay exact."""
    from paper_2607_06225_amd import aln, serving
    arrival, kinds, batches = mix
    ctx, sids = make_ctx(batches)
    reqs = [rq for rq in serving.mixed_requests(batches, kinds, sids) if rq["kind"] == 2] * 3
    budget = 12 << 20
    srv = aln.Server(ctx, streams=4, max_batch_pairs=4, hbm_budget=budget, class_streams=4)
    comps, cigs, _, _ = serving.replay(srv, reqs)
    st = srv.stats()
    srv.close()
    print(f"[gpu] admission: {st}", flush=True)
    assert st["completed"] == len(reqs)
    assert st["admission_waits"] > 0
    assert st["peak_arena_bytes"] <= budget
    assert np.all(comps["error"] == 0)
    n = len(reqs) // 3
    for f in FIELDS:  # the three copies of each request agree
        assert np.array_equal(comps[f][:n], comps[f][n:2 * n]), f
        assert np.array_equal(comps[f][:n], comps[f][2 * n:]), f
    oracle_check(reqs[:n], comps[:n], cigs[:n], batches)
    ctx.close()


def test_micro_batches_overlap_on_the_device(mix):
    from paper_2607_06225_amd import aln, serving
    arrival, kinds, batches = mix
    ctx, sids = make_ctx(batches)
    reqs = serving.mixed_requests(batches, kinds, sids)
    srv = aln.Server(ctx, streams=4, max_batch_pairs=16, hbm_budget=1 << 30)
    comps, _, _, _ = serving.replay(srv, reqs)  # burst
    st = srv.stats()
    srv.close()
    assert st["peak_inflight"] >= 2
    # two micro-batches whose [launch, done] intervals intersect
    b = {}
    for c in comps:
        b[int(c["batch_id"])] = (float(c["t_launch"]), float(c["t_done"]))
    iv = sorted(b.values())
    assert any(iv[k + 1][0] < iv[k][1] for k in range(len(iv) - 1))
    ctx.close()


def test_submit_rejects_what_cannot_run(mix):
    from paper_2607_06225_amd import aln
    _, _, batches = mix
    ctx, sids = make_ctx(batches)
    srv = aln.Server(ctx, streams=2, max_batch_pairs=4, hbm_budget=1 << 20)
    rng = np.random.default_rng(1)
    big = rng.integers(0, 4, size=20000).astype(np.uint8)
    with pytest.raises(aln.AlnError, match="-4"):  # ALN_E_CAPACITY: larger than the budget
        srv.submit(sids[2], big, big, aln.GLOBAL, aln.BAND, band_w=256, want_cigar=True)
    with pytest.raises(aln.AlnError):              # unknown scoring
        srv.submit(99, big[:10], big[:10], aln.GLOBAL)
    with pytest.raises(aln.AlnError):              # XDROP needs EXTEND
        srv.submit(sids[3], big[:10], big[:10], aln.GLOBAL, aln.XDROP, xdrop=10)
    # the server still works after rejected submits
    rid = srv.submit(sids[0], big[:100], big[:90], aln.GLOBAL, want_cigar=True)
    srv.drain(60000)
    comps, cigs = srv.poll(8)
    assert len(comps) == 1 and int(comps[0]["id"]) == rid and comps[0]["error"] == 0
    assert cigs[0] is not None and len(cigs[0]) == comps[0]["cigar_len"]
    srv.close()
    ctx.close()
