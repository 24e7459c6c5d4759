"""Replay of timed single-pair requests through the alignment server.

Requests are submitted at their arrival times (seconds from the start of the
replay) while completions are polled; latency is measured on the server's
clock from the request's scheduled arrival to the moment the server saw its
micro-batch finish, so any submission lag counts against the server.
"""
import time

import numpy as np

from . import aln


def mixed_requests(batches, kinds, scoring_ids):
    """Interleave per-kind batches into one request list in arrival order.
    kinds[i] names the batch request i comes from; each batch is consumed in
    order.  Returns a list of dicts accepted by replay()."""
    cursor = [0] * len(batches)
    reqs = []
    for k in np.asarray(kinds, dtype=np.int64):
        b = batches[int(k)]
        p = cursor[int(k)]
        cursor[int(k)] += 1
        q, r = b.pair(p)
        reqs.append(dict(kind=int(k), pair=p, scoring_id=scoring_ids[int(k)], q=q, r=r,
                         mode=b.mode, prune=b.prune, band_w=b.band_w, xdrop=b.xdrop,
                         want_cigar=b.want_cigar))
    return reqs


def replay(server, requests, arrival_s=None, one_at_a_time=False, poll_max=256):
    """Submit requests at arrival_s (None: all at once) and collect every
    completion.  one_at_a_time: wait for each result before the next submit.
    Returns (completions ndarray in request order, CIGAR list, wall seconds,
    latency seconds per request)."""
    n = len(requests)
    if arrival_s is None:
        arrival_s = np.zeros(n)
    arrival_s = np.asarray(arrival_s, dtype=np.float64)
    comps = np.zeros(n, dtype=aln.COMPLETION_DTYPE)
    cigs = [None] * n
    seen = np.zeros(n, dtype=bool)
    c0 = server.clock()
    t0 = time.perf_counter()
    i = got = 0
    while got < n:
        now = time.perf_counter() - t0
        while i < n and arrival_s[i] <= now and (not one_at_a_time or i == got):
            rq = requests[i]
            server.submit(rq["scoring_id"], rq["q"], rq["r"], rq["mode"], rq["prune"],
                          rq["band_w"], rq["xdrop"], want_cigar=rq["want_cigar"], tag=i)
            i += 1
        waiting_only = i == n or one_at_a_time
        c, cg = server.poll(poll_max, wait_us=1000 if waiting_only else 0)
        for rec, cig in zip(c, cg):
            k = int(rec["tag"])
            if seen[k]:
                raise RuntimeError(f"request {k} completed twice")
            seen[k] = True
            comps[k] = rec
            cigs[k] = cig
            got += 1
        if not len(c) and i < n and not one_at_a_time:
            dt = arrival_s[i] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(min(dt, 2e-4))
    wall = time.perf_counter() - t0
    latency = comps["t_done"] - (c0 + arrival_s)
    if one_at_a_time or not np.any(arrival_s):
        latency = comps["t_done"] - comps["t_submit"]
    return comps, cigs, wall, latency


def percentiles(lat_s):
    lat = np.asarray(lat_s, dtype=np.float64) * 1e3
    return dict(p50_ms=round(float(np.percentile(lat, 50)), 3),
                p99_ms=round(float(np.percentile(lat, 99)), 3),
                mean_ms=round(float(lat.mean()), 3), max_ms=round(float(lat.max()), 3))
