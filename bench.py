#!/usr/bin/env python3
"""Benchmark: alignment throughput (GCUPS) of the batched gfx950 path on one GPU.

A step is one pass of the whole hot path over one batch already resident in
HBM: task-list upload, code validation, the fill kernels (with the int32
re-run of pairs the int16 pass flags, or the wider re-run of X-drop regions
that outgrow their window) and, when the workload asks for it, the traceback
walk to CIGAR.  GCUPS counts the cells each pair's pruning rule evaluates
(all M*N for the full matrix, the band for a static band, the surviving
cells for X-drop), exactly the `cells` field the oracle reports.

The headline workload (the JSON line's `value`) is the largest single-GPU
one, X-drop seed extension: 200,000 seeds x 2 sides, int32, score + end
cell + cells visited, every side checked against the oracle.  The other
workloads (protein Smith-Waterman, global DNA with CIGAR, banded long reads
with CIGAR, Z-drop, X-drop with CIGAR, the search schedule) are measured the
same way under "configs", and the serving mix of four of them (Poisson
arrivals through the request server) under "serving" with p50/p99 latency.
The roofline of each dominant kernel is priced by the issue rates that
aln_valu_probe measures per instruction class, at the spec clock and at the
clock measured under load; the last key, "summary", repeats each workload's
rate, roofline fraction and check in a few fields.

For each: per-kernel times from HIP events recorded on the launch stream
during the timed steps (roofline of the dominant kernel), the same kernels
launched once per pair (per-pair baseline), and the CPU oracle on a bounded
sample of the same pairs (cpu_baseline), whose results double as the
bit-exactness check of that sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GCUPS (bit-exact) at 1 GPU, batched vs per-pair; % int-VALU roofline; p50/p99"

# Algorithmic 2-input integer operations per evaluated cell, by class
# (add, max, compare-or-select):
#   H+o+e (add), E = max(E+e, .) (add, max), F = max(F+e, .) (add, max),
#   H = max(Hdiag+s, E, F) (add, 2 max)                     -> 4 add 4 max (global)
#   local adds max(., 0) and the running maximum             -> 4 add 6 max
#   extension adds the running maximum                       -> 4 add 5 max
#   X-drop adds the test against best - X                    -> 4 add 5 max 1 cmp
#   Z-drop adds |d - d_best| (absolute difference, priced as a
#   compare) and its add to H                                -> 5 add 5 max 2 cmp
# A search entry (score s, diagonal d) of unit-cost edit distance: two adds
# (mismatch, insertion), three bound tests, two max; the character compares of
# its extension depend on the data and are not counted     -> 2 add 2 max 3 cmp
# A gap-affine search entry: E (max of two sources, two bound tests), F (the
# same plus an add), H (an add, two bound tests, two max)  -> 2 add 4 max 6 cmp
OPS_BY_CLASS = {("GLOBAL", 0): dict(add=4, max=4), ("GLOBAL", 1): dict(add=4, max=4),
                ("LOCAL", 0): dict(add=4, max=6), ("LOCAL", 1): dict(add=4, max=6),
                ("EXTEND", 0): dict(add=4, max=5), ("EXTEND", 1): dict(add=4, max=5),
                ("EXTEND", 2): dict(add=4, max=5, cmp=1), ("EXTEND", 3): dict(add=5, max=5, cmp=2),
                ("GLOBAL", 4): dict(add=2, max=2, cmp=3)}
OPS_BY_CLASS_KERNEL = {"search_affine": dict(add=2, max=4, cmp=6),
                       "search_affine_wide": dict(add=2, max=4, cmp=6)}
# The minimal VALU instruction counts per cell that the roofline plan of this
# path derives for each configuration (fused 3-input ops allowed): reported
# beside the algorithmic counts above.
PLAN_INSTR_PER_CELL = {"nw_dna_1k": 16, "sw_protein": 6.0, "band_long": 16, "xdrop_ext": 15}
# Instruction class -> probe instruction whose measured issue rate prices it;
# packed 16-bit kernels issue every class as a packed op (two cells each).
PROBE_FOR_CLASS = {"add": "v_add_u32", "max": "v_max_i32", "cmp": "v_cmp_gt_i32"}
PROBE_FOR_CLASS_I16 = {"add": "v_pk_add_u16", "max": "v_pk_max_i16", "cmp": "v_pk_max_i16"}
# MI355X: 256 CUs x 4 SIMDs; spec clock 2.4 GHz; a wave64 instruction of the
# basic rate occupies its SIMD for 4 cycles (0.25 wave instructions per SIMD
# per cycle) -- the rate used when no probe measurement is at hand.
SIMDS = 1024
SPEC_CLOCK_GHZ = 2.4
BASIC_RATE = 0.25
PEAK_I32_TOPS = SIMDS * 64 * BASIC_RATE * SPEC_CLOCK_GHZ / 1e3  # 39.32
KERNEL_WIDTH = {"sw16": "i16"}
FILL_KERNELS = ("sw16", "strip_i32", "diag_band", "band_strip", "xdrop", "xdrop_lanes", "xdrop_lanes_tb",
                "zdrop", "zdrop_lanes", "xdrop_tb", "zdrop_tb",
                "search", "search_affine", "search_affine_wide")


def mix_peak_tops(by_class, rates, width, clock_ghz):
    """Peak 2-input ops per second (T) of a kernel whose cells need by_class
    ops: every SIMD issues each class at its measured rate (wave instructions
    per SIMD per cycle), a packed 16-bit instruction doing two cells' op."""
    per_lane = 2 if width == "i16" else 1
    cls = PROBE_FOR_CLASS_I16 if width == "i16" else PROBE_FOR_CLASS
    cycles = sum(n / (rates.get(cls[c], BASIC_RATE) * 64 * per_lane) for c, n in by_class.items())
    return sum(by_class.values()) / cycles * SIMDS * clock_ghz * 1e9 / 1e12


WORKLOAD_DESC = {
    "sw_protein": ("Smith-Waterman local, protein (20 letters, seeded symmetric matrix), "
                   "open -11 extend -1, 65,536 pairs, lengths lognormal median 350 clipped "
                   "50-2000 per side, 30% homologous; score + end cell"),
    "nw_dna_1k": ("Needleman-Wunsch global, DNA +2/-4 open -4 extend -2, 256 pairs of "
                  "1 kbp with 10% edits; full matrix + CIGAR"),
    "band_long": ("banded global, DNA +1/-2 open -2 extend -1, 2,048 pairs of 10-100 kbp "
                  "with 12% errors, static band half-width 256; score + CIGAR"),
    "xdrop_ext": ("X-drop extension, DNA +2/-4 open -4 extend -2, X = 100, 200,000 seeds x "
                  "2 sides of 150-5,000 bp at 5-25% divergence plus 10% random flank; "
                  "score + end cell"),
    "zdrop_ext": ("Z-drop extension (Sec. 9.3 condition), the xdrop_ext pairs with Z = 100; "
                  "score + end cell"),
    "xdrop_cigar": ("X-drop extension with CIGAR: the xdrop_ext pairs, score + end cell + "
                    "CIGAR through the pruned region (score pass, traceback pass to the end "
                    "cell, walk)"),
    "edit_search": ("unit-cost edit distance by the score-major search schedule (Sec. 6.3), "
                    "4,096 pairs of 2,000 bp at 5% divergence; score (= -edit distance)"),
    "rna_fold": ("Nussinov RNA folding (the folding recurrence of Sec. 3) with X-drop "
                 "transferred to it (Sec. 9.5): 4,096 synthetic RNAs of 76-500 nt, one point "
                 "per A-U / C-G / G-U pair, minimum loop 3, X = 2 after a warm-up of 15 spans; "
                 "the same sequences unpruned beside it"),
    "affine_search": ("gap-affine penalties (mismatch 4, open 6, extend 2) by the score-major "
                      "search schedule, the edit_search pair shape (4,096 pairs of 2,000 bp at "
                      "5% divergence, other seed); score (= -smallest penalty)"),
}
MODE_NAME = {0: "GLOBAL", 1: "LOCAL", 2: "EXTEND"}
PRUNE_NAME = {0: "full", 1: "band", 2: "xdrop", 3: "zdrop", 4: "search"}

# The paper's edit-distance table (Sec. 9.1): antidiagonal (full matrix) and
# search times on its CPU, in the table's units (the text calls them
# milliseconds, the caption seconds), keyed by (length, divergence).
PAPER_EDIT_TABLE = {(500, 0.01): (0.069, 0.0007), (2000, 0.01): (0.87, 0.0089),
                    (4000, 0.01): (4.15, 0.0138), (500, 0.05): (0.050, 0.0019),
                    (2000, 0.05): (0.71, 0.052), (4000, 0.05): (4.27, 0.19),
                    (500, 0.30): (0.051, 0.11), (2000, 0.30): (0.72, 1.58),
                    (4000, 0.30): (4.36, 6.02)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def trimmed_mean(xs):
    """The paper's protocol (Sec. 9.1): of 10 runs drop the 2 highest and the 2
    lowest and average the rest; for fewer runs, drop proportionally."""
    xs = sorted(xs)
    k = int(len(xs) * 0.2)
    core = xs[k: len(xs) - k] if len(xs) - 2 * k > 0 else xs
    return float(np.mean(core))


def host_cores():
    """Host threads this process may use: the CPU affinity set, capped by the
    cgroup CPU quota when one is set (a container's share), and the CPU model."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()[:2]
        if q != "max":
            quota = max(1, int(int(q) / int(per)))
    except (OSError, ValueError):
        pass
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return (min(n, quota) if quota else n), n, quota, model


def cpu_baseline(batch, work, target_s, runs=10):
    """The oracle on a bounded sample of the batch, timed with the paper's
    protocol (Sec. 9.1): `runs` runs, the 2 highest and 2 lowest dropped, the
    mean of the rest.  The sample (the first k pairs) is sized so that all
    runs together take about target_s on every host core; a single-thread
    run of a smaller sample gives the one-core rate.  ``work`` is a per-pair
    cost estimate used only to size the samples."""
    from tests.parity import oracle_batch
    cores, nproc, quota, model = host_cores()
    n = batch.n
    k0 = min(n, 64)
    sub0 = batch.subset(np.arange(k0))
    t0 = time.perf_counter()
    o0 = oracle_batch(sub0, nthreads=cores)
    dt0 = max(time.perf_counter() - t0, 1e-3)
    rate = max(float(o0["cells"].sum()), 1.0) / dt0
    cum = np.cumsum(work.astype(np.float64))
    k = int(np.searchsorted(cum, rate * target_s / runs)) + 1
    k = max(k0, min(n, k))
    sub = batch.subset(np.arange(k))
    times = []
    ores = None
    for _ in range(runs):
        t0 = time.perf_counter()
        ores = oracle_batch(sub, nthreads=cores)
        times.append(time.perf_counter() - t0)
    dt = trimmed_mean(times)
    cells = float(ores["cells"].sum())
    # one core: a sample of about a tenth of the all-core run's cells
    k1 = max(1, int(np.searchsorted(cum, 0.1 * cells)) + 1)
    k1 = min(k1, k)
    sub1 = batch.subset(np.arange(k1))
    t0 = time.perf_counter()
    o1 = oracle_batch(sub1, nthreads=1)
    dt1 = time.perf_counter() - t0
    cells1 = float(o1["cells"].sum())
    return dict(value=round(cells / dt / 1e9, 4), unit="GCUPS", cores=cores, kind="oracle",
                sample=f"first {k} of {n} pairs in generation order ({cells:.3e} cells); "
                       f"trimmed mean of {runs} runs (2 highest and 2 lowest dropped) "
                       f"on {cores} host threads",
                seconds=round(dt, 3), run_seconds=[round(t, 3) for t in times],
                nproc=nproc, cgroup_cpu_quota=quota, cpu_model=model,
                single_core=dict(value=round(cells1 / dt1 / 1e9, 4), unit="GCUPS",
                                 sample=f"first {k1} pairs ({cells1:.3e} cells), one run",
                                 seconds=round(dt1, 3))), ores, k


def measured_traffic(family, workload):
    """HBM bytes per launch of a kernel family on a workload, from the
    rocprofv3 FETCH_SIZE / WRITE_SIZE passes summarised in
    profiles/traffic.json (scaled by a copy of known size).  None when the
    kernel's source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    for e in table.get("kernels", []):
        if e["family"] == family and e["workload"] == workload:
            with open(os.path.join(ROOT, e["source"]), "rb") as src:
                if hashlib.sha256(src.read()).hexdigest()[:16] != e["source_sha256_16"]:
                    return None
            return int(e["hbm_bytes_per_launch"])
    return None


def bit_exact_check(batch, res, cig, work, ores, k, rate, budget_s):
    """Compare GPU results with the oracle: the first k pairs (the CPU
    baseline's sample, whose oracle results are in ores) and, when
    budget_s > 0, further pairs spread evenly over the whole batch -- every
    pair if the oracle can do them all in about budget_s at `rate` cells/s."""
    from tests.parity import compare, oracle_batch
    sub = batch.subset(np.arange(k))
    bad = compare(sub, res[:k], cig[:k] if cig is not None else None, ores)
    checked = k
    rest = np.arange(k, batch.n)
    if budget_s > 0 and rest.size and rate:
        w = work[rest].astype(np.float64)
        frac = min(1.0, rate * budget_s / max(float(w.sum()), 1.0))
        if frac < 1.0:
            step = max(1, int(np.ceil(1.0 / frac)))
            rest = rest[::step]
        t0 = time.perf_counter()
        sub = batch.subset(rest)
        o = oracle_batch(sub)
        bad += compare(sub, res[rest], [cig[i] for i in rest] if cig is not None else None, o)
        checked += rest.size
        log(f"[bench] checked {rest.size} more pairs in {time.perf_counter() - t0:.1f} s")
    if checked == batch.n:
        how = "every pair"
    elif checked == k:
        how = f"the first {k} pairs (the CPU baseline's sample) only"
    else:
        how = (f"the first {k} pairs and every {max(1, (batch.n - k) // (checked - k))}-th "
               f"pair after them")
    return dict(pairs=int(checked), of=int(batch.n), sample=how, mismatches=len(bad),
                first=bad[:3])


def run_workload(name, batch, args, cpu_seconds, pp_cap, check_seconds=0.0, machine=None):
    import torch
    from paper_2607_06225_amd import aln
    from tests.parity import compare

    mode_name = MODE_NAME[batch.mode]
    ctx = aln.Context(0)
    sid = ctx.set_scoring(batch.matrix, batch.gap_open, batch.gap_extend)
    tuning = None
    db = aln.DeviceBatch(batch)
    if not args.no_autotune:
        # tune on the batch itself, or on its first 65,536 pairs
        tb = batch if batch.n <= 65536 else batch.subset(np.arange(65536))
        tdb = db if tb is batch else aln.DeviceBatch(tb)
        t0 = time.perf_counter()
        tuning = ctx.autotune(sid, tdb, batch.mode, batch.prune, batch.band_w, batch.xdrop,
                              want_cigar=batch.want_cigar,
                              cache=None if args.no_tuning_cache else args.tuning_cache,
                              scoring=(batch.matrix, batch.gap_open, batch.gap_extend))
        tuning = dict(ms=round((time.perf_counter() - t0) * 1e3, 1), sample_pairs=tb.n,
                      **{k: v for k, v in tuning.items() if k != "valid"})
        del tdb
    t0 = time.perf_counter()
    plan = ctx.plan(sid, batch.q_len, batch.r_len, batch.mode, batch.prune, batch.band_w,
                    batch.xdrop, aln.W_AUTO, batch.want_cigar)
    plan_ms = (time.perf_counter() - t0) * 1e3
    buf = aln.Buffers(plan)
    stream = torch.cuda.current_stream()

    def step():
        ctx.execute(plan, db, buf.ws, buf.res, buf.cigar, stream=stream)

    log(f"[bench] {name}: warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.kernel_times()

    # timed steps; per-kernel HIP events ride on the same stream
    log(f"[bench] {name}: timing {args.steps} steps")
    ctx.set_profiling(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for s in range(args.steps):
        step()
        ev[s + 1].record(stream)
    torch.cuda.synchronize()
    ctx.set_profiling(False)
    ktimes = ctx.kernel_times()
    per_step = [ev[s].elapsed_time(ev[s + 1]) for s in range(args.steps)]
    ms_per_step = ev[0].elapsed_time(ev[-1]) / args.steps
    res = buf.results(batch.n)
    cig = buf.cigars(res)
    cells = int(res["cells"].sum())
    full_cells = int((batch.q_len.astype(np.int64) * batch.r_len).sum())
    gcups = cells / (ms_per_step * 1e-3) / 1e9

    kernel_ms = {k: v[0] / args.steps for k, v in ktimes.items()}
    fills = {k: v for k, v in kernel_ms.items() if k in FILL_KERNELS}
    dom = max(fills or kernel_ms, key=(fills or kernel_ms).get)
    dom_launches = ktimes[dom][1] / args.steps
    dom_launch_ms = ktimes[dom][0] / ktimes[dom][1]
    width = KERNEL_WIDTH.get(dom, "i32")
    by_class = OPS_BY_CLASS_KERNEL.get(dom, OPS_BY_CLASS[(mode_name, batch.prune)])
    ops = sum(by_class.values())
    # every evaluated cell passes through the dominant fill kernel once
    cells_per_launch = cells / dom_launches
    achieved = cells_per_launch * ops / (dom_launch_ms * 1e-3) / 1e12
    rates = (machine or {}).get("issue_rates", {})
    clk = (machine or {}).get("clock_ghz")
    peak = mix_peak_tops(by_class, rates, width, SPEC_CLOCK_GHZ)
    roof = dict(bound="alu", achieved=round(achieved, 3), peak=round(peak, 2), unit="TOP/s",
                frac=round(achieved / peak, 4), traffic=measured_traffic(dom, name),
                kernel=dom, ops_per_cell=ops, ops_by_class=by_class, op_width=width,
                peak_basis=("issue rate of each op class measured by aln_valu_probe, at the "
                            "2.4 GHz spec clock" if rates else
                            "0.25 wave instructions per SIMD per cycle, 2.4 GHz spec clock"),
                cells_per_launch=int(cells_per_launch), launches_per_step=dom_launches,
                avg_launch_ms=round(dom_launch_ms, 4))
    if clk:
        pk = mix_peak_tops(by_class, rates, width, clk)
        roof.update(clock_ghz_measured=round(clk, 3), peak_at_measured_clock=round(pk, 2),
                    frac_at_measured_clock=round(achieved / pk, 4))
    if name in PLAN_INSTR_PER_CELL:
        # the plan's formula: GCUPS x minimal instructions per cell over
        # 256 CUs x 64 lanes x clock (packed int16: instructions are per cell)
        ipc = PLAN_INSTR_PER_CELL[name]
        ach_i = cells_per_launch * ipc / (dom_launch_ms * 1e-3) / 1e12
        roof["plan_instr_per_cell"] = ipc
        roof["frac_plan_count"] = round(ach_i / (256 * 64 * SPEC_CLOCK_GHZ / 1e3), 4)
        if clk:
            roof["frac_plan_count_at_measured_clock"] = round(ach_i / (256 * 64 * clk / 1e3), 4)

    per_pair = None
    if pp_cap:
        # the first k pairs, k bounded by a pair count and a cell budget
        k = int(np.searchsorted(np.cumsum(res["cells"].astype(np.float64)),
                                args.per_pair_cells, side="right"))
        k = max(1, min(batch.n, pp_cap, k))
        if k < batch.n:
            sub = batch.subset(np.arange(k))
            splan = ctx.plan(sid, sub.q_len, sub.r_len, sub.mode, sub.prune, sub.band_w,
                             sub.xdrop, aln.W_AUTO, sub.want_cigar)
            sdb, sbuf = aln.DeviceBatch(sub), aln.Buffers(splan)
        else:
            sub, splan, sdb, sbuf = batch, plan, db, buf
        log(f"[bench] {name}: per-pair baseline over {k} pairs")
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        torch.cuda.synchronize()
        e[0].record(stream)
        ctx.execute(splan, sdb, sbuf.ws, sbuf.res, sbuf.cigar, stream=stream)
        e[1].record(stream)
        torch.cuda.synchronize()
        bat_res = sbuf.results(sub.n)
        e[2].record(stream)
        ctx.execute_per_pair(splan, sdb, sbuf.ws, sbuf.res, sbuf.cigar, stream=stream)
        e[3].record(stream)
        torch.cuda.synchronize()
        pp_ms, b_ms = e[2].elapsed_time(e[3]), e[0].elapsed_time(e[1])
        pp_res = sbuf.results(sub.n)
        sc = int(pp_res["cells"].sum())
        per_pair = dict(pairs=k, ms=round(pp_ms, 3), gcups=round(sc / (pp_ms * 1e-3) / 1e9, 4),
                        batched_ms_same_pairs=round(b_ms, 3),
                        batched_speedup=round(pp_ms / b_ms, 2),
                        identical=bool(np.array_equal(pp_res, bat_res)))
        if splan is not plan:
            splan.close()

    cpu = verified = None
    if cpu_seconds > 0:
        log(f"[bench] {name}: CPU oracle on a bounded sample")
        # the oracle's work per pair: its own cells (for a search batch, the
        # full matrix of the definition it evaluates)
        work = (batch.q_len.astype(np.int64) * batch.r_len if batch.prune == 4
                else res["cells"])
        cpu, ores, k = cpu_baseline(batch, work, cpu_seconds)
        if batch.prune == 4:
            cpu["alignments_per_s"] = round(k / cpu["seconds"], 1)
        log(f"[bench] {name}: bit-exact check against the oracle")
        verified = bit_exact_check(batch, res, cig, work, ores, k,
                                   rate=float(ores["cells"].sum()) / max(cpu["seconds"], 1e-6),
                                   budget_s=check_seconds)

    out = dict(
        workload=name, desc=WORKLOAD_DESC[name], pairs=batch.n, cells=cells,
        full_matrix_cells=full_cells, mode=mode_name.lower(), prune=PRUNE_NAME[batch.prune],
        dtype=width, ms_per_step=round(ms_per_step, 4), gcups=round(gcups, 3),
        step_ms_trimmed_mean=round(trimmed_mean(per_step), 4),
        step_ms_median=round(float(np.median(per_step)), 4),
        kernel_ms_per_step={k: round(v, 4) for k, v in kernel_ms.items()},
        roofline=roof, per_pair=per_pair, cpu_baseline=cpu, bit_exact_check=verified,
        plan_ms=round(plan_ms, 2), autotune=tuning,
        statuses={int(s): int(c) for s, c in zip(*np.unique(res["status"], return_counts=True))},
    )
    if batch.prune in (2, 3):
        out["widened_pairs"] = int(((res["flags"] & aln.F_WIDENED) != 0).sum())
        out["too_wide_pairs"] = int((res["status"] == aln.R_TOO_WIDE).sum())
        if batch.want_cigar:
            out["cigar_cap_pairs"] = int((res["status"] == aln.R_CIGAR_CAP).sum())
    if batch.mode == 1 and batch.prune == 0:
        out["int32_reruns"] = int(((res["flags"] & aln.F_I16_RERUN) != 0).sum())
    if batch.prune == 4:
        # entries are (score, diagonal) pairs; also report the full-matrix
        # equivalent rate and alignments per second
        out["equivalent_gcups"] = round(full_cells / (ms_per_step * 1e-3) / 1e9, 3)
        out["alignments_per_s"] = round(batch.n / (ms_per_step * 1e-3), 1)
        out["mean_edit_distance" if batch.gap_open == 0 and batch.gap_extend == -1
            else "mean_penalty"] = round(float(-res["score"].mean()), 2)
    plan.close()
    ctx.close()
    log(f"[bench] {name}: " + json.dumps({k: out[k] for k in (
        "gcups", "ms_per_step", "cells", "kernel_ms_per_step", "per_pair", "cpu_baseline",
        "bit_exact_check")}))
    return out


def measure_machine():
    """Issue rates of the instruction classes the roofline prices, and the
    shader clock under a VALU load, from aln_valu_probe: every SIMD busy with
    one instruction over 8 independent chains (4 waves per SIMD), and the
    latency of a dependent chain (one wave per SIMD)."""
    from paper_2607_06225_amd import aln
    ctx = aln.Context(0)
    rows, rates, by_waves = [], {}, {}
    for op in aln.PROBE_OPS:
        for wps in (2, 4, 8):
            r = aln.valu_probe(ctx, op, waves_per_simd=wps, iters=2000)
            rows.append(r)
            by_waves.setdefault(op, {})[wps] = round(r["issue_per_simd_cycle"], 4)
        # the peak is the best rate any occupancy reaches
        rates[op] = max(by_waves[op].values())
    dep = {}
    for op in ("v_add_u32", "v_max_i32", "v_max3_i32", "v_cndmask_b32"):
        r = aln.valu_probe(ctx, op, dependent=True, waves_per_simd=1, iters=2000)
        rows.append(r)
        dep[op] = round(r["cycles_per_instr_one_wave"], 2)
    ctx.close()
    clocks = sorted(r["clock_ghz"] for r in rows if r["clock_ghz"])
    return dict(clock_ghz=clocks[len(clocks) // 2] if clocks else None,
                clock_ghz_range=[round(clocks[0], 3), round(clocks[-1], 3)] if clocks else None,
                issue_rates=rates, issue_rates_by_waves_per_simd=by_waves,
                dependent_cycles_per_instr=dep,
                note="issue rates in wave64 instructions per SIMD per shader cycle, every SIMD "
                     "busy (2, 4 or 8 waves each, 8 independent chains per wave; the best of the "
                     "three is the rate used); clock from s_memtime over s_memrealtime (100 MHz) "
                     "during those loops")


def summarize(r):
    """Short record of one workload's line."""
    bx = r.get("bit_exact_check") or {}
    rf = r["roofline"]
    rec = dict(gcups=r["gcups"], ms=r["ms_per_step"], kernel=rf["kernel"], frac=rf["frac"],
               frac_at_measured_clock=rf.get("frac_at_measured_clock"),
               checked=f"{bx.get('pairs', 0)}/{r['pairs']}",
               mismatches=bx.get("mismatches"))
    if r.get("per_pair"):
        rec["batched_vs_per_pair"] = r["per_pair"]["batched_speedup"]
    if r.get("cpu_baseline"):
        rec["cpu_gcups"] = r["cpu_baseline"]["value"]
    for k in ("widened_pairs", "too_wide_pairs", "cigar_cap_pairs", "alignments_per_s"):
        if k in r:
            rec[k] = r[k]
    return rec


def run_fold(args, cpu_seconds, check_seconds, machine):
    """Nussinov folding with X-drop (and the same sequences unpruned): cells
    and bifurcation terms per second, the kernel's roofline (one add and one
    max per term), the oracle beside it, and every sequence checked."""
    import torch
    import oracle
    from paper_2607_06225_amd import aln
    from paper_2607_06225_amd import workloads as W

    ctx = aln.Context(0)
    stream = torch.cuda.current_stream()
    fbx = W.rna_fold()
    out = dict(workload="rna_fold", desc=WORKLOAD_DESC["rna_fold"], sequences=fbx.n,
               lengths=[int(fbx.length.min()), int(fbx.length.max())])
    runs = {}
    for tag, fb in (("xdrop", fbx), ("unpruned", fbx.with_params(xdrop=-1))):
        plan = aln.fold_plan(ctx, fb)
        fdb = aln.FoldDeviceBatch(fb)
        ws = torch.empty(max(plan.workspace_bytes, 1), dtype=torch.uint8, device="cuda")
        res = torch.zeros(fb.n * aln.FOLD_RESULT_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        for _ in range(args.warmup):
            aln.fold_execute(ctx, plan, fdb, ws, res, stream=stream)
        torch.cuda.synchronize()
        ctx.kernel_times()
        ctx.set_profiling(True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
        ev[0].record(stream)
        for k in range(args.steps):
            aln.fold_execute(ctx, plan, fdb, ws, res, stream=stream)
            ev[k + 1].record(stream)
        torch.cuda.synchronize()
        ctx.set_profiling(False)
        kt = ctx.kernel_times()
        per_step = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)]
        ms = ev[0].elapsed_time(ev[-1]) / args.steps
        r = np.frombuffer(res.cpu().numpy().tobytes(), dtype=aln.FOLD_RESULT_DTYPE, count=fb.n).copy()
        cells, terms = int(r["cells"].sum()), int(r["terms"].sum())
        kms, launches = kt["fold"][0] / args.steps, kt["fold"][1] / args.steps
        by_class = dict(add=1, max=1)
        rates = (machine or {}).get("issue_rates", {})
        clk = (machine or {}).get("clock_ghz")
        achieved = terms * 2 / (kms * 1e-3) / 1e12
        peak = mix_peak_tops(by_class, rates, "i32", SPEC_CLOCK_GHZ)
        roof = dict(bound="alu", achieved=round(achieved, 3), peak=round(peak, 2), unit="TOP/s",
                    frac=round(achieved / peak, 4), traffic=None, kernel="fold",
                    ops_per_term=2, ops_by_class=by_class, launches_per_step=launches,
                    avg_launch_ms=round(kms / max(launches, 1), 4),
                    note="achieved = bifurcation terms x 2 (add, max) / fold kernel time; the "
                         "kernel also spends two address adds and two LDS reads per term")
        if clk:
            pk = mix_peak_tops(by_class, rates, "i32", clk)
            roof.update(clock_ghz_measured=round(clk, 3), frac_at_measured_clock=round(achieved / pk, 4))
        runs[tag] = dict(ms_per_step=round(ms, 4), step_ms_trimmed_mean=round(trimmed_mean(per_step), 4),
                         kernel_ms_per_step=round(kms, 4), cells=cells, terms=terms,
                         gcups=round(cells / (ms * 1e-3) / 1e9, 3),
                         gterms_per_s=round(terms / (ms * 1e-3) / 1e9, 2),
                         sequences_per_s=round(fb.n / (ms * 1e-3), 1), roofline=roof,
                         results=r, batch=fb)
        plan.close()
        log(f"[bench] rna_fold {tag}: {ms:.3f} ms, {runs[tag]['gterms_per_s']} Gterms/s")
    rx, ru = runs["xdrop"]["results"], runs["unpruned"]["results"]
    out["xdrop_equals_unpruned"] = round(float(np.mean(rx["score"] == ru["score"])), 4)
    out["xdrop_cells_fraction"] = round(runs["xdrop"]["cells"] / max(runs["unpruned"]["cells"], 1), 4)
    out["xdrop_speedup"] = round(runs["unpruned"]["ms_per_step"] / runs["xdrop"]["ms_per_step"], 3)
    # the oracle: CPU baseline on a sample (paper's protocol), then every
    # sequence of both runs checked
    if cpu_seconds > 0:
        cores, nproc, quota, model = host_cores()
        fb = runs["xdrop"]["batch"]

        def ofold(b, nthreads):
            return oracle.fold_batch(b.pair, b.x, b.off, b.length, min_loop=b.min_loop,
                                     xdrop=b.xdrop, warmup=b.warmup, nthreads=nthreads)
        t0 = time.perf_counter()
        o0 = ofold(fb.subset(np.arange(64)), cores)
        rate = float(o0["terms"].sum()) / max(time.perf_counter() - t0, 1e-3)
        cum = np.cumsum(rx["terms"].astype(np.float64))
        k = max(64, min(fb.n, int(np.searchsorted(cum, rate * cpu_seconds / 10)) + 1))
        sub = fb.subset(np.arange(k))
        times = []
        for _ in range(10):
            t0 = time.perf_counter()
            o = ofold(sub, cores)
            times.append(time.perf_counter() - t0)
        dt = trimmed_mean(times)
        k1 = max(1, k // 10)
        t0 = time.perf_counter()
        o1 = ofold(fb.subset(np.arange(k1)), 1)
        dt1 = time.perf_counter() - t0
        out["cpu_baseline"] = dict(
            value=round(float(o["cells"].sum()) / dt / 1e9, 4), unit="GCUPS", cores=cores,
            kind="oracle", gterms_per_s=round(float(o["terms"].sum()) / dt / 1e9, 3),
            sample=f"first {k} of {fb.n} sequences (X-drop), trimmed mean of 10 runs on "
                   f"{cores} host threads", seconds=round(dt, 3), nproc=nproc,
            cgroup_cpu_quota=quota, cpu_model=model,
            single_core=dict(value=round(float(o1["cells"].sum()) / dt1 / 1e9, 4),
                             gterms_per_s=round(float(o1["terms"].sum()) / dt1 / 1e9, 3),
                             sample=f"first {k1} sequences, one run"))
    if check_seconds > 0:
        for tag in ("xdrop", "unpruned"):
            b, r = runs[tag]["batch"], runs[tag]["results"]
            o = oracle.fold_batch(b.pair, b.x, b.off, b.length, min_loop=b.min_loop,
                                  xdrop=b.xdrop, warmup=b.warmup, nthreads=host_cores()[0])
            mism = [p for p in range(b.n)
                    if any(int(r[f][p]) != int(o[f][p]) for f in ("score", "i", "j", "cells",
                                                                    "terms", "full"))]
            runs[tag]["bit_exact_check"] = dict(pairs=b.n, of=b.n, sample="every sequence",
                                                mismatches=len(mism), first=mism[:3])
    for tag in runs:
        runs[tag].pop("results")
        runs[tag].pop("batch")
    out.update(runs)
    # the line-level fields the summary reads: the X-drop run
    x = runs["xdrop"]
    out.update(gcups=x["gcups"], ms_per_step=x["ms_per_step"], roofline=x["roofline"],
               pairs=fbx.n, bit_exact_check=x.get("bit_exact_check"), per_pair=None)
    ctx.close()
    return out


def run_edit_table(args):
    """Unit-cost edit distance at the lengths and divergences of the paper's
    table (Sec. 9.1): the same pairs through the score-major search schedule
    and through the full-matrix path (the antidiagonal schedule), each timed
    with HIP events (median of 3 after a warm-up).  Scores must agree with
    each other on every pair and with the CPU oracle on a sample."""
    import torch
    from paper_2607_06225_amd import aln
    from paper_2607_06225_amd import workloads as W
    from tests.parity import compare, oracle_batch

    ctx = aln.Context(0)
    stream = torch.cuda.current_stream()
    rows = []
    for (length, div), (p_ad, p_search) in sorted(PAPER_EDIT_TABLE.items(),
                                                   key=lambda x: (x[0][1], x[0][0])):
        n = args.edit_table_pairs
        bs = W.edit_pairs(n, length, div, seed=700 + length + int(1000 * div))
        sid = ctx.set_scoring(bs.matrix, bs.gap_open, bs.gap_extend)
        db = aln.DeviceBatch(bs)
        times, res = {}, {}
        for prune in (W.SEARCH, W.FULL):
            plan = ctx.plan(sid, bs.q_len, bs.r_len, W.GLOBAL, prune)
            buf = aln.Buffers(plan)
            ctx.execute(plan, db, buf.ws, buf.res, None, stream=stream)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
            for k in range(3):
                ev[2 * k].record(stream)
                ctx.execute(plan, db, buf.ws, buf.res, None, stream=stream)
                ev[2 * k + 1].record(stream)
            torch.cuda.synchronize()
            times[prune] = float(np.median([ev[2 * k].elapsed_time(ev[2 * k + 1])
                                            for k in range(3)]))
            res[prune] = buf.results(n)
            plan.close()
        agree = bool(np.array_equal(res[W.SEARCH]["score"], res[W.FULL]["score"]))
        k = min(n, args.edit_table_check)
        sub = bs.subset(np.arange(k))
        bad = compare(sub, res[W.SEARCH][:k], None, oracle_batch(sub))
        rows.append(dict(
            length=length, divergence=div, pairs=n,
            mean_edit_distance=round(float(-res[W.SEARCH]["score"].mean()), 2),
            search_ms=round(times[W.SEARCH], 4), full_ms=round(times[W.FULL], 4),
            search_us_per_alignment=round(1e3 * times[W.SEARCH] / n, 3),
            full_us_per_alignment=round(1e3 * times[W.FULL] / n, 3),
            search_over_full=round(times[W.FULL] / times[W.SEARCH], 2),
            scores_agree=agree, oracle_checked=k, oracle_mismatches=len(bad),
            paper_ad_time=p_ad, paper_search_time=p_search,
            paper_search_over_ad=round(p_ad / p_search, 2)))
        log(f"[bench] edit table {length} bp {div}: {json.dumps(rows[-1])}")
        del db
    ctx.close()
    return dict(note="paper times: its CPU (Intel Core i9-285K), one alignment, in the table's "
                     "units (ms per the text of Sec. 9.1, s per the caption); context only",
                rows=rows)


def sustained_rate(comps, lo=0.1, hi=0.9):
    """Completions per second between the lo and hi fractions of a burst's
    completions (reported beside the burst's rate: short requests finish
    first, so this rate runs ahead of the mix's)."""
    t = np.sort(np.asarray(comps["t_done"], dtype=np.float64))
    n = len(t)
    a, b = int(lo * n), max(int(hi * n) - 1, int(lo * n) + 1)
    b = min(b, n - 1)
    return (b - a) / max(t[b] - t[a], 1e-9)


def run_serving(args):
    """Serving mix: requests drawn from the four workloads (40/30/10/20) at
    full size.  Saturation is the rate of a burst of every request (all
    submitted at once: tens of micro-batches at full queue, start to last
    completion); Poisson arrivals then run at 0.5x and 0.8x of it.  The
    device budget is 0.9 x the free HBM, and the burst runs again under a
    256 MB budget.  Latency is arrival to completion on the server clock."""
    import torch
    from paper_2607_06225_amd import aln, serving
    from paper_2607_06225_amd import workloads as W
    from tests.parity import compare, oracle_batch

    n = args.serving_requests
    log(f"[bench] serving: generating {n} requests")
    arrival1, kinds, batches = W.serving_requests(n, qps=1.0, seed=505)
    ctx = aln.Context(0)
    sids = [ctx.set_scoring(b.matrix, b.gap_open, b.gap_extend) for b in batches]
    reqs = serving.mixed_requests(batches, kinds, sids)
    torch.cuda.empty_cache()
    free_b, total_b = torch.cuda.mem_get_info()
    budget = int(0.9 * free_b) // (1 << 20) << 20
    cfg = dict(streams=args.serving_streams, max_batch_pairs=1024, hbm_budget=budget,
               class_streams=args.serving_class_streams)
    out = dict(requests=n, mix="40/30/10/20 of nw_dna_1k/sw_protein/band_long/xdrop_ext "
                              "(one pair or one extension side per request)",
               streams=cfg["streams"], hbm_free_bytes=int(free_b), hbm_budget_bytes=budget,
               levels=[])

    def level(name, arrival, budget_b):
        srv = aln.Server(ctx, **dict(cfg, hbm_budget=budget_b))
        comps, cigs, wall, lat = serving.replay(srv, reqs, arrival)
        st = srv.stats()
        srv.close()
        rec = dict(level=name, hbm_budget_bytes=budget_b, wall_s=round(wall, 3),
                   qps_achieved=round(n / wall, 1),
                   gcups=round(st["cells"] / wall / 1e9, 3), batches=st["batches"],
                   mean_batch_pairs=round(n / max(st["batches"], 1), 2),
                   peak_inflight=st["peak_inflight"], admission_waits=st["admission_waits"],
                   errors=int((comps["error"] != 0).sum()), **serving.percentiles(lat))
        if arrival is None:
            rec["completion_rate_mid80"] = round(sustained_rate(comps), 1)
        log(f"[bench] serving {name}: {json.dumps(rec)}")
        return rec, comps, cigs

    log("[bench] serving: burst (saturation)")
    sat, comps, cigs = level("burst", None, budget)
    out["levels"].append(sat)
    out["saturation_qps"] = sat["qps_achieved"]
    for frac in (0.5, 0.8):
        qps = frac * sat["qps_achieved"]
        rec, _, _ = level(f"{frac}x", arrival1 / qps, budget)
        rec["qps_offered"] = round(qps, 1)
        out["levels"].append(rec)
    log("[bench] serving: burst under a 256 MB budget")
    small, _, _ = level("burst_256MB", None, 256 << 20)
    out["levels"].append(small)

    # bit-exact check of the burst level against the oracle on the first k requests
    k = min(n, args.serving_check)
    bad = 0
    first = []
    for kind, b in enumerate(batches):
        idx = [i for i in range(k) if reqs[i]["kind"] == kind]
        if not idx:
            continue
        sub = b.subset([reqs[i]["pair"] for i in idx])
        ores = oracle_batch(sub)
        gc = [cigs[i] if cigs[i] is not None else np.zeros(0, np.uint32) for i in idx]
        mism = compare(sub, comps[idx], gc if b.want_cigar else None, ores)
        bad += len(mism)
        first += mism[:2]
    out["bit_exact_check"] = dict(requests=k, mismatches=bad, first=first[:3])
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="xdrop_ext",
                    choices=sorted(k for k in WORKLOAD_DESC if k != "rna_fold"),
                    help="headline workload (the JSON line's value)")
    ap.add_argument("--edit-table-pairs", type=int, default=1024,
                    help="pairs per cell of the edit-distance table (0: skip the table)")
    ap.add_argument("--edit-table-check", type=int, default=16,
                    help="pairs per cell checked against the CPU oracle")
    ap.add_argument("--configs",
                    default="sw_protein,nw_dna_1k,band_long,zdrop_ext,xdrop_cigar,edit_search,"
                            "affine_search,rna_fold",
                    help="comma list of further workloads to measure, or 'none'")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="plan with built-in tile costs instead of measured ones")
    ap.add_argument("--no-per-pair", action="store_true")
    ap.add_argument("--tuning-cache",
                    default=os.path.expanduser("~/.cache/paper_2607_06225_amd/tuning.json"),
                    help="JSON file of tile choices kept across runs (per device, library "
                         "hash, scoring, parameters and batch shape)")
    ap.add_argument("--no-tuning-cache", action="store_true",
                    help="time every candidate tile even when a cached choice exists")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="headline: oracle seconds of the CPU baseline (all 10 runs)")
    ap.add_argument("--extra-cpu-seconds", type=float, default=6.0,
                    help="other workloads: oracle seconds of the CPU baseline")
    ap.add_argument("--check-seconds", type=float, default=60.0,
                    help="headline: oracle seconds for the bit-exact check beyond the "
                         "baseline's sample (enough for every pair of the default headline)")
    ap.add_argument("--extra-check-seconds", type=float, default=5.0,
                    help="other workloads: oracle seconds for the bit-exact check")
    ap.add_argument("--per-pair-cap", type=int, default=2048,
                    help="largest number of pairs launched one by one")
    ap.add_argument("--serving-requests", type=int, default=20000,
                    help="requests per serving level (0: skip the serving mix)")
    ap.add_argument("--serving-streams", type=int, default=4)
    ap.add_argument("--serving-class-streams", type=int, default=0,
                    help="streams one request class may hold (0: the server default, streams/4)")
    ap.add_argument("--no-probe", action="store_true",
                    help="price the roofline at 0.25 wave instructions per SIMD per cycle "
                         "instead of the probe's measured issue rates")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only run the VALU issue-rate / clock probe and print its JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (calibrates HBM "
                         "byte counters against a transfer of known size)")
    ap.add_argument("--serving-only", action="store_true",
                    help="measure only the serving mix (no headline line)")
    ap.add_argument("--serving-check", type=int, default=600,
                    help="requests of the burst level checked against the oracle")
    ap.add_argument("--per-pair-cells", type=float, default=1e9,
                    help="cell budget of the one-launch-per-pair sample")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "one GPU only: pairs are independent, so a multi-GPU run "
                                   "would shard them by cells with no exchange between GPUs; "
                                   "run with --gpus 1"}))
        return 2

    import torch
    from paper_2607_06225_amd import workloads as W

    torch.cuda.set_device(0)
    extras = [] if args.configs == "none" else [c for c in args.configs.split(",") if c]
    for c in extras:
        if c not in WORKLOAD_DESC:
            ap.error(f"unknown workload {c}")
    pp_cap = 0 if args.no_per_pair else args.per_pair_cap

    if args.copy_calibration:
        n = args.copy_calibration << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n, "copies": 5}), flush=True)
        return 0
    if args.valu_probe:
        print(json.dumps({"valu_probe": measure_machine()}), flush=True)
        return 0
    machine = None if args.no_probe else measure_machine()
    if machine:
        log(f"[bench] probe: clock {machine['clock_ghz']:.3f} GHz, rates {machine['issue_rates']}")
    if args.serving_only:
        print(json.dumps({"serving": run_serving(args)}), flush=True)
        return 0
    log(f"[bench] generating {args.workload}")
    head = run_workload(args.workload, W.WORKLOADS[args.workload](), args,
                        0 if args.no_cpu_baseline else args.cpu_seconds, pp_cap,
                        args.check_seconds, machine)
    configs = {}
    for c in extras:
        if c == args.workload:
            continue
        if c == "rna_fold":
            configs[c] = run_fold(args, 0 if args.no_cpu_baseline else args.extra_cpu_seconds,
                                  args.extra_check_seconds, machine)
            continue
        log(f"[bench] generating {c}")
        t0 = time.perf_counter()
        b = W.WORKLOADS[c]()
        log(f"[bench] {c}: {b.n} pairs generated in {time.perf_counter() - t0:.1f} s")
        configs[c] = run_workload(c, b, args, 0 if args.no_cpu_baseline
                                  else args.extra_cpu_seconds, pp_cap, args.extra_check_seconds,
                                  machine)
        del b
    edit_table = run_edit_table(args) if args.edit_table_pairs > 0 else None
    serving_out = run_serving(args) if args.serving_requests > 0 else None

    out = {
        "metric": METRIC,
        "value": head["gcups"],
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOAD_DESC[args.workload]}",
                   "pairs": head["pairs"], "cells": head["cells"], "mode": head["mode"],
                   "prune": head["prune"]},
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
        "per_pair": head["per_pair"],
        "bit_exact_check": head["bit_exact_check"],
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "step_ms_trimmed_mean": head["step_ms_trimmed_mean"],
        "step_ms_median": head["step_ms_median"],
        "plan_ms": head["plan_ms"],
        "autotune": head["autotune"],
        "machine": machine,
        "configs": configs,
        "edit_table": edit_table,
        "serving": serving_out,
    }
    for k in ("int32_reruns", "statuses", "widened_pairs", "cigar_cap_pairs", "too_wide_pairs",
              "equivalent_gcups", "alignments_per_s", "mean_edit_distance", "mean_penalty"):
        if k in head:
            out[k] = head[k]
    # last key: one short record per workload, so that a truncated copy of the
    # line still holds every workload's rate, roofline fraction and check
    out["summary"] = {w: summarize(r) for w, r in [(args.workload, head)] + list(configs.items())}
    if serving_out:
        out["summary"]["serving"] = {
            lv["level"]: dict(qps=lv["qps_achieved"], gcups=lv["gcups"],
                              p50_ms=lv.get("p50_ms"), p99_ms=lv.get("p99_ms"))
            for lv in serving_out["levels"]}
        out["summary"]["serving"]["requests"] = serving_out["requests"]
        out["summary"]["serving"]["bit_exact"] = serving_out["bit_exact_check"]["mismatches"] == 0
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
