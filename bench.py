#!/usr/bin/env python3
"""Benchmark of one Dask worker's cuDF-merge work on one MI355X.

A step is one mdx_merge over the synthetic 1E8 x 1E8 workload: hash-partition
the left and the right table into P = 32 destinations (int64 key + int64
payload per row, keys of the left table a permutation of [0, 1E8), 30% of the
right rows matching), then hash-join every partition.  Inputs are resident in
device memory before the timed region.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--cpu-baseline off]
"""

from __future__ import annotations

import argparse
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input rows/s for partition+join, 100M×100M int64; serving p50/p99 latency"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="paper",
                    choices=["paper", "plain", "skewed", "batched", "serving", "transpose"])
    ap.add_argument("--batch-count", type=int, default=4096,
                    help="batched: number of merges (4096 = the full batch)")
    ap.add_argument("--lanes", type=int, default=4, help="batched: concurrent lanes")
    ap.add_argument("--duration", type=float, default=60.0, help="serving: seconds of arrivals")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: requests per second")
    ap.add_argument("--slots", type=int, default=8, help="serving: concurrent slots")
    ap.add_argument("--serve-mode", default="merge", choices=["merge", "probe"],
                    help="serving: requests bring both tables, or probe device-resident tables")
    ap.add_argument("--serve-unique", type=int, default=256,
                    help="serving: distinct requests drawn on the device (the stream picks among them)")
    ap.add_argument("--overload-rate", type=float, default=5000.0,
                    help="serving: the second point's arrival rate (above FIFO capacity)")
    ap.add_argument("--overload-duration", type=float, default=10.0,
                    help="serving: seconds of arrivals at the overload rate")
    ap.add_argument("--budget-gb", type=float, default=200.0, help="serving: HBM budget")
    ap.add_argument("--graph-merges", type=int, default=256,
                    help="batched: merges captured per HIP graph (graphs replay in order)")
    ap.add_argument("--fused-ws-gb", type=float, default=64.0,
                    help="batched: workspace of the fused batch (more waves when smaller)")
    ap.add_argument("--fused-tuning", default="table", choices=["table", "default"],
                    help="batched: the fused batch's tuning (the autotuner's table, or defaults)")
    ap.add_argument("--cpu-baseline", default="on", choices=["on", "off", "full"],
                    help="on: one-thread oracle on a 0.2-scale sample + all-cores oracle at "
                         "full size; full: both at full size (the one-thread leg takes ~1 min)")
    ap.add_argument("--cpu-sample-scale", type=float, default=0.2,
                    help="fraction of the workload the one-thread oracle runs on the host")
    return ap.parse_args()


def counted_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/*traffic.json, written by paper_2101_08878_amd.rocprof_summary
    from FETCH_SIZE and WRITE_SIZE runs), or None when there is none for the
    kernel's current sources."""
    from paper_2101_08878_amd.rocprof_summary import kernel_sources_hash
    sources = kernel_sources_hash(kernel)
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*traffic.json"))):
        with open(f) as fh:
            t = json.load(fh)
        if t.get("kernel") == kernel and t.get("workload") == workload \
                and t.get("kernel_sources") == sources:
            return t["traffic_bytes_per_launch"], os.path.relpath(f, ROOT)
    return None, None


def step_algorithmic_bytes(nl, nr, key_bytes, total_out):
    """Bytes one merge moves by the method's own accounting: partition (read
    and write key + payload of every row of both tables), build (read a left
    row, write its 16-byte table entry), probe (read a right row and one
    16-byte table entry), output (key + two payloads per row).  A join whose
    tables live in LDS moves the table entries on chip, so its HBM minimum is
    the same less 16 B per input row (algorithmic_hbm_bytes)."""
    row = key_bytes + 8
    return (nl + nr) * 2 * row + (nl + nr) * (row + 16) + total_out * (key_bytes + 16)


def credited_bytes(kernel, nl, nr, key_bytes, total_out):
    """HBM bytes of the method credited to one kernel (per merge): the
    partition scatter reads and writes every row of both tables; the join's
    emit reads every build and probe row and writes the output.  Histogram
    pre-reads, the second partition pass and the count's key read are this
    implementation's overheads and are credited nothing."""
    row = key_bytes + 8
    if kernel == "part_scatter":
        return (nl + nr) * 2 * row
    if kernel == "rj_join":
        return (nl + nr) * row + total_out * (key_bytes + 16)
    return 0


def host_info():
    """Host cores this process may use, and the CPU model."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cores_available": avail, "cpu_model": model}


def cpu_baselines(mode, scale, full_tables, P):
    """The oracle timed on the host: (1) one thread, the plain oracle
    (stable counting-sort partition of both tables + sort-merge join) on a
    sample of the same generator -- or at full size with mode "full"; (2) the
    same algorithms over all available host cores (per-thread histograms
    with a (destination, block)-major prefix, then one destination per
    thread joined by sort-merge) at full size.  Capped at 16 threads, the
    host cores a one-GPU process is given there."""
    import oracle
    from workloads import config_inputs

    info = host_info()
    if mode == "full":
        kl, vl, kr, vr = full_tables
        sample = "the full workload"
    else:
        kl, vl, kr, vr = config_inputs("paper", scale=scale)
        sample = f"the same generator at {scale:g} scale"
    log(f"cpu baseline: oracle on {kl.size} x {kr.size} rows (one thread)")
    t0 = time.perf_counter()
    oracle.hash_partition(kl, vl, P)
    oracle.hash_partition(kr, vr, P)
    res = oracle.join(kl, vl, kr, vr)
    dt1 = time.perf_counter() - t0
    log(f"cpu baseline: {dt1:.2f} s, |J| = {res['total']}")
    one = {"value": (kl.size + kr.size) / dt1, "unit": "input rows/s", "cores": 1,
           "kind": "oracle", **info,
           "sample": f"{sample}: {kl.size} x {kr.size} rows, P={P}; stable counting-sort "
                     f"partition of both tables + sort-merge join, {dt1:.2f} s on one host thread"}
    del kl, vl, kr, vr, res
    kl, vl, kr, vr = full_tables
    threads = max(1, min(16, info["cores_available"]))
    log(f"cpu baseline: threaded oracle on {kl.size} x {kr.size} rows, {threads} threads")
    t0 = time.perf_counter()
    r = oracle.merge_threads(kl, vl, kr, vr, P, threads)
    dt = time.perf_counter() - t0
    log(f"cpu baseline: {dt:.2f} s, |J| = {r['total']}")
    allc = {"value": (kl.size + kr.size) / dt, "unit": "input rows/s", "cores": threads,
            "kind": "oracle (threaded)", **info,
            "sample": f"the full workload: {kl.size} x {kr.size} rows, P={P}; the partition "
                      f"(per-thread histograms, stable) and one destination per thread joined "
                      f"by sort-merge, {dt:.2f} s on {threads} host threads"}
    return one, allc


def copy_ceiling(torch, dev, n=1 << 27, reps=5):
    """Device-to-device copy of n int64 (read n*8 + write n*8 bytes): the
    achievable-bandwidth reference, and the known-size kernel that scales
    the HBM byte counters of a counter run."""
    src = torch.arange(n, dtype=torch.int64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes": 2 * n * 8, "ms": round(ms, 4), "gbs": round(2 * n * 8 / (ms / 1e3) / 1e9, 1)}


def batched_inputs(torch, specs, dev, seed=0, frac=0.3):
    """The batch's tables, drawn on the device with torch's generator (the
    host would need minutes for ~4E9 rows): per merge, left keys a random
    permutation of [0, nL); right keys: round(frac nR) drawn from the left
    keys, the rest uniform in [nL, 2 nL), shuffled; payload = row index.
    The same recipe as workloads.match_fraction_tables, other random bits."""
    import paper_2101_08878_amd as mdx
    jobs, matched = [], []
    g = torch.Generator(device=dev)
    for s in specs:
        g.manual_seed(seed * 1_000_003 + s.index)
        kd = torch.int32 if s.key_dtype == "int32" else torch.int64
        nl, nr = s.n_left, s.n_right
        m = int(round(frac * nr))
        kl = torch.randperm(nl, generator=g, device=dev, dtype=torch.int64)
        hit = kl[torch.randint(0, nl, (m,), generator=g, device=dev, dtype=torch.int64)]
        miss = torch.randint(nl, 2 * nl, (nr - m,), generator=g, device=dev, dtype=torch.int64)
        kr = torch.cat([hit, miss])[torch.randperm(nr, generator=g, device=dev)]
        jobs.append(mdx.MergeJob(kl.to(kd), torch.arange(nl, dtype=torch.int64, device=dev),
                                 kr.to(kd).contiguous(), torch.arange(nr, dtype=torch.int64, device=dev),
                                 8, max(m, 1)))
        matched.append(m)
    for j in jobs:
        j.status = torch.zeros(1, dtype=torch.int32, device=dev)
    return jobs, matched


def fmix64_torch(torch, x):
    """MurmurHash3's 64-bit finalizer on int64 tensors (wrapping products;
    logical shifts by masking), for checking partitions of device output."""
    m1 = 0xff51afd7ed558ccd - (1 << 64)
    m2 = 0xc4ceb9fe1a85ec53 - (1 << 64)
    x = x ^ ((x >> 33) & ((1 << 31) - 1))
    x = x * m1
    x = x ^ ((x >> 33) & ((1 << 31) - 1))
    x = x * m2
    return x ^ ((x >> 33) & ((1 << 31) - 1))


def batch_rows_check(torch, jobs):
    """Row-level check of every merge of a batch whose left keys are
    distinct and whose payloads are row indices: every output row's key
    equals the key of its left row and of its right row; the right rows of
    the output are exactly the right rows whose key occurs on the left, each
    once; every row of partition block p has fmix64(key) mod P = p (P a power
    of two).  Together these fix the join's rows and per-partition offsets.
    Returns a message for the first failing merge, or None."""
    for i, j in enumerate(jobs):
        P = j.P
        assert P & (P - 1) == 0
        off = j.out_offsets
        n = int(off[-1])
        kl, kr = j.left_keys.long(), j.right_keys.long()
        k, lp, rp = j.out[0][:n].long(), j.out[1][:n], j.out[2][:n]
        if n and not (bool((lp >= 0).all()) and bool((lp < kl.numel()).all())
                      and bool((rp >= 0).all()) and bool((rp < kr.numel()).all())):
            return f"merge {i}: payload out of range"
        if n and not (torch.equal(kl[lp], k) and torch.equal(kr[rp], k)):
            return f"merge {i}: a row's key differs from its left or right row's"
        want = torch.nonzero(torch.isin(kr, kl)).flatten()
        if not torch.equal(torch.sort(rp).values, want):
            return f"merge {i}: the right rows of the output are not the matching ones, once each"
        part = fmix64_torch(torch, k) & (P - 1)
        block = torch.repeat_interleave(torch.arange(P, device=k.device), torch.diff(off))
        if not torch.equal(part, block):
            return f"merge {i}: a row outside its key's partition block"
    return None


def batched_cpu_baseline(specs, budget_s=15.0):
    """The oracle (one host thread) on the batch's first merges, drawn with
    the workloads generator, until budget_s of oracle time is spent."""
    import oracle
    from workloads import batch_tables

    rows, spent, k = 0, 0.0, 0
    for s in specs:
        kl, vl, kr, vr = batch_tables(s)
        t0 = time.perf_counter()
        oracle.hash_partition(kl, vl, 8)
        oracle.hash_partition(kr, vr, 8)
        oracle.join(kl, vl, kr, vr)
        spent += time.perf_counter() - t0
        rows += kl.size + kr.size
        k += 1
        if spent >= budget_s:
            break
    return {"value": rows / spent, "unit": "input rows/s", "cores": 1, "kind": "oracle",
            "sample": f"the batch's first {k} merges ({rows} input rows), P=8: both partitions "
                      f"+ sort-merge join, {spent:.2f} s on one host thread"}


def run_batched(args):
    """Secondary line: a batch of uneven merges (sizes log-uniform in
    [1E3, 4E6] rows per side, int32 or int64 keys, match fraction 0.3, P=8),
    one merge at a time vs mdx_merge_batch (eager, and replayed from a HIP
    graph).  Inputs resident in HBM; every merge's |J| is checked."""
    import torch

    import paper_2101_08878_amd as mdx
    from workloads import batch_specs

    specs = batch_specs(4096)[: args.batch_count]
    dev = torch.device("cuda:0")
    log(f"batched: generating {len(specs)} merges on the device")
    jobs, matched = batched_inputs(torch, specs, dev)
    rows = sum(s.n_left + s.n_right for s in specs)
    for j in jobs:
        j.out = tuple(torch.empty(j.out_capacity, dtype=t, device=dev)
                      for t in (j.left_keys.dtype, torch.int64, torch.int64))
        j.out_offsets = torch.empty(j.P + 1, dtype=torch.int64, device=dev)
    lanes = args.lanes
    chunks = [jobs[i:i + args.graph_merges] for i in range(0, len(jobs), args.graph_merges)]
    ws = torch.empty(max([mdx.mdx_merge_batch_workspace_bytes(jobs, lanes)] +
                         [mdx.mdx_merge_batch_workspace_bytes(c, lanes) for c in chunks]),
                     dtype=torch.uint8, device=dev)
    big = max(jobs, key=lambda j: mdx.mdx_merge_workspace_bytes(
        j.left_keys.numel(), j.right_keys.numel(), j.P, 4 if j.left_keys.dtype == torch.int32 else 8))
    ws1 = torch.empty(mdx.mdx_merge_workspace_bytes(
        big.left_keys.numel(), big.right_keys.numel(), big.P,
        4 if big.left_keys.dtype == torch.int32 else 8), dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.synchronize()  # inputs were drawn on torch's current stream
    log(f"batched: {rows} input rows, workspace {ws.numel() / 1e9:.2f} GB ({lanes} lanes)")

    def sequential():
        for j in jobs:
            mdx.mdx_merge(j.left_keys, j.left_payload, j.right_keys, j.right_payload, j.P,
                          out_capacity=j.out_capacity, out=j.out, out_offsets=j.out_offsets,
                          workspace=ws1, status=j.status, stream=stream)

    def batch():
        mdx.mdx_merge_batch(jobs, lanes=lanes, workspace=ws, stream=stream)

    def check(label):
        tot = torch.stack([j.out_offsets[-1] for j in jobs]).cpu().tolist()
        st = torch.cat([j.status for j in jobs]).cpu().tolist()
        bad = [i for i in range(len(jobs)) if tot[i] != matched[i] or st[i] != 0]
        if bad:
            raise SystemExit(f"{label}: merge {bad[0]} gave |J|={tot[bad[0]]}, status {st[bad[0]]}, "
                             f"want {matched[bad[0]]}")

    def check_rows(label):
        bad = batch_rows_check(torch, jobs)
        if bad:
            raise SystemExit(f"{label}: {bad}")
        log(f"  {label}: every row of all {len(jobs)} merges checked")

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, (time.perf_counter() - w0) * 1e3 / reps

    res = {}
    for label, fn in [("one merge at a time", sequential), (f"batch, {lanes} lanes", batch)]:
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        check(label)
        ms, wall = timed(fn, args.steps)
        res[label] = (ms, wall)
        log(f"  {label}: {ms:.2f} ms device, {wall:.2f} ms wall, {rows / (wall / 1e3):.4g} rows/s")
    # the batch captured as graphs of graph_merges merges each (one
    # workspace: the graphs replay one after another on `stream`)
    graphs = []
    for c in chunks:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            mdx.mdx_merge_batch(c, lanes=lanes, workspace=ws, stream=stream)
        graphs.append(g)
    torch.cuda.synchronize()

    def replay():
        with torch.cuda.stream(stream):
            for g in graphs:
                g.replay()

    for j in jobs:
        j.out_offsets.fill_(-1)
    replay()
    torch.cuda.synchronize()
    check("graph")
    ms, wall = timed(replay, args.steps)
    res["graph"] = (ms, wall)
    log(f"  batch in {len(graphs)} HIP graphs: {ms:.2f} ms device, {wall:.2f} ms wall, "
        f"{rows / (wall / 1e3):.4g} rows/s")
    check_rows("graph")

    # the fused batch: one launch per step for all merges, eager and as one
    # HIP graph
    tuning = "table" if args.fused_tuning == "table" else None
    lo, hi = mdx.mdx_batch_workspace_bytes(jobs, tuning)
    del graphs, ws
    torch.cuda.empty_cache()
    fb = mdx.FusedBatch(jobs, tuning=tuning,
                        workspace_bytes=max(lo, min(hi, int(args.fused_ws_gb * 1e9))))
    waves, launches = fb.info()
    log(f"batched: fused batch, {waves} waves, {launches} launches per run, workspace "
        f"{fb.workspace.numel() / 1e9:.1f} GB (one wave: {hi / 1e9:.1f} GB)")

    def fused():
        fb.run(stream)

    for _ in range(max(args.warmup, 1)):
        fused()
    torch.cuda.synchronize()
    for j in jobs:
        j.out_offsets.fill_(-1)
        for t in j.out:
            t.fill_(-1)
    fused()
    torch.cuda.synchronize()
    check("fused")
    check_rows("fused")
    ms, wall = timed(fused, args.steps)
    res["fused"] = (ms, wall)
    log(f"  fused batch: {ms:.2f} ms device, {wall:.2f} ms wall, {rows / (wall / 1e3):.4g} rows/s")
    gf = torch.cuda.CUDAGraph()
    with torch.cuda.graph(gf, stream=stream):
        fb.run(stream)
    torch.cuda.synchronize()

    def fused_graph():
        with torch.cuda.stream(stream):
            gf.replay()

    for j in jobs:
        j.out_offsets.fill_(-1)
    fused_graph()
    torch.cuda.synchronize()
    check("fused graph")
    ms, wall = timed(fused_graph, args.steps)
    res["fused graph"] = (ms, wall)
    log(f"  fused batch in one HIP graph: {ms:.2f} ms device, {wall:.2f} ms wall, "
        f"{rows / (wall / 1e3):.4g} rows/s")
    del gf

    seq_wall = res["one merge at a time"][1]
    lanes_wall = res["graph"][1]
    wall = res["fused graph"][1]
    step_bytes = sum((s.n_left + s.n_right) * (2 * (4 if s.key_dtype == "int32" else 8) + 16)
                     + (s.n_left + s.n_right) * ((4 if s.key_dtype == "int32" else 8) + 8 + 16)
                     for s in specs) + sum(m * ((4 if s.key_dtype == "int32" else 8) + 16)
                                           for s, m in zip(specs, matched))
    achieved = step_bytes / (wall / 1e3) / 1e9
    line = {
        "metric": "input rows/s for a batch of 4096 uneven merges (1E3-4E6 rows per side, "
                  "int32/int64 keys, P=8)",
        "value": round(rows / (wall / 1e3), 1),
        "unit": "input rows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32/int64", "data": "synthetic",
        "config": {"workload": f"batched: {len(specs)} merges, {rows} input rows, P=8, "
                               f"match fraction 0.3; fused batch (one launch per step, "
                               f"{waves} waves, tuning {args.fused_tuning}) replayed from one "
                               f"HIP graph",
                   "merges": len(specs), "input_rows": rows, "waves": waves,
                   "launches_per_run": launches, "tuning": args.fused_tuning,
                   "lanes_path": f"{lanes} lanes, HIP graphs of {args.graph_merges} merges"},
        "roofline": {"bound": "hbm", "kernel": "whole batch", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "modes_ms": {k: {"device": round(v[0], 3), "wall": round(v[1], 3)} for k, v in res.items()},
        "speedup_vs_one_at_a_time": round(seq_wall / wall, 3),
        "speedup_vs_lanes_graphs": round(lanes_wall / wall, 3),
        "checked": "every output row of every merge (fused and lanes+graphs): keys equal on "
                   "both sides, every right row whose key is on the left exactly once, rows in "
                   "their key's partition",
    }
    if args.cpu_baseline == "on":
        fb.close()
        del jobs, ws1, fb
        line["cpu_baseline"] = batched_cpu_baseline(specs)
    print(json.dumps(line), flush=True)


SERVE_MAX_ROWS = 20_000_000


def serving_pool(torch, dev, n_unique, seed=0):
    """The distinct requests of the serving workload, drawn on the device
    before the timed loop (requests of the stream then pick one each).  One
    permutation lk of [0, 2E7) gives every left table as a prefix lk[:nL]
    (distinct keys); request u: nL, nR log-uniform in [1E4, 2E7], match
    fraction f ~ U[0.1, 0.9]; its right keys: m = round(f nR) drawn uniformly
    from its own left rows lk[:nL], the other nR - m from [2E7, 4E7) (never a
    left key), shuffled.  |J| = m exactly.  Payload = row index."""
    import numpy as np
    N = SERVE_MAX_ROWS
    rng = np.random.default_rng(seed)
    g = torch.Generator(device=dev)
    g.manual_seed(seed + 17)
    lk = torch.randperm(N, generator=g, device=dev, dtype=torch.int64)
    pay = torch.arange(N, dtype=torch.int64, device=dev)
    reqs = []
    for u in range(n_unique):
        nl = int(round(np.exp(rng.uniform(np.log(1e4), np.log(2e7)))))
        nr = int(round(np.exp(rng.uniform(np.log(1e4), np.log(2e7)))))
        f = float(rng.uniform(0.1, 0.9))
        m = int(round(f * nr))
        hit = lk[torch.randint(0, nl, (m,), generator=g, device=dev)]
        miss = torch.randint(N, 2 * N, (nr - m,), generator=g, device=dev)
        rk = torch.cat([hit, miss])[torch.randperm(nr, generator=g, device=dev)].contiguous()
        reqs.append({"nl": nl, "nr": nr, "f": f, "m": m, "rk": rk})
    return lk, pay, reqs


def serve_run(torch, mdx, stream_reqs, pool, slots, budget, dev, mode, tables=None):
    """Serve the stream (arrival s, unique request index) as it arrives;
    returns (latencies in ms, elapsed s, totals, statuses).  A request is
    admitted in arrival order when a slot, an output buffer and the memory
    budget allow.  mode "merge": each request brings its left and right
    table; mode "probe": each request probes a build table kept on the
    device (tables[t], built once) with its right rows."""
    from collections import deque

    lk, pay, uniq = pool
    N = SERVE_MAX_ROWS
    n = len(stream_reqs)
    nbuf = slots + 4
    bufs = [tuple(torch.empty(N, dtype=torch.int64, device=dev) for _ in range(3))
            for _ in range(nbuf)]
    free = list(range(nbuf))
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    offsets = torch.zeros((n, 9), dtype=torch.int64, device=dev)
    lat = [0.0] * n
    owner = {}
    queue = deque()
    nxt = done = 0
    with mdx.Server(slots, N, N, 8, budget, device=dev) as srv:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done < n:
            now = time.perf_counter() - t0
            while nxt < n and stream_reqs[nxt][0] <= now:
                queue.append(nxt)
                nxt += 1
            while queue and free:
                i = queue[0]
                r = uniq[stream_reqs[i][1]]
                b = bufs[free[-1]]
                if mode == "merge":
                    nl, nr = r["nl"], r["nr"]
                    job = mdx.MergeJob(lk[:nl], pay[:nl], r["rk"], pay[:nr], 8, r["m"],
                                       out=b, out_offsets=offsets[i], status=status[i:i + 1])
                    ok = srv.submit(job, i, ready=0)
                else:
                    job = mdx.ProbeJob(tables[r["table"]], r["rk"], pay[:r["nr"]], r["m"],
                                       out=b, out_offsets=offsets[i], status=status[i:i + 1])
                    ok = srv.submit_probe(job, i, ready=0)
                if ok is None:
                    break
                owner[i] = free.pop()
                queue.popleft()
            for i in srv.poll():
                lat[i] = (time.perf_counter() - t0 - stream_reqs[i][0]) * 1e3
                free.append(owner.pop(i))
                done += 1
        elapsed = time.perf_counter() - t0
    return lat, elapsed, offsets[:, -1].cpu(), status.cpu()


def serving_check_rows(torch, mdx, pool, tables, dev):
    """Every distinct request run alone (not timed), its rows checked: |J| =
    m, every row's key equals the left key at its left payload and the
    right key at its right payload, the right payloads are exactly the hit
    rows (each right row has at most one partner: left keys are distinct)."""
    lk, pay, uniq = pool
    bad = 0
    for u, r in enumerate(uniq):
        nr, m = r["nr"], r["m"]
        if tables is None:
            nl = r["nl"]
            ok, ol, orr, off = mdx.mdx_merge(lk[:nl], pay[:nl], r["rk"], pay[:nr], 8,
                                             out_capacity=max(m, 1))
            left = lk[:nl]
        else:
            t = tables[r["table"]]
            rk, rv, ro = mdx.mdx_hash_partition(r["rk"], pay[:nr], 8)
            ok, ol, orr, off = mdx.mdx_join_probe(t, rk, rv, ro, out_capacity=max(m, 1))
            left = lk[:r["nl"]]
        total = int(off[-1].item())
        if total != m:
            bad += 1
            continue
        ok, ol, orr = ok[:m], ol[:m], orr[:m]
        hits = torch.nonzero(r["rk"] < SERVE_MAX_ROWS).flatten()
        if not (torch.equal(ok, left[ol]) and torch.equal(ok, r["rk"][orr])
                and torch.equal(torch.sort(orr).values, hits)):
            bad += 1
    return bad


def run_serving(args):
    """Serving lines: a Poisson stream of requests (sizes log-uniform in
    [1E4, 2E7] rows per side, int64 keys, match fraction U[0.1, 0.9] per
    request, P=8) admitted as slots and the HBM budget free up (continuous
    batching), against one request at a time in arrival order (FIFO), at the
    configured rate and at an overload rate.  Mode "merge": each request
    brings both tables; mode "probe": the build tables stay on the device
    (built once with mdx_join_build) and each request probes one."""
    import numpy as np
    import torch

    import paper_2101_08878_amd as mdx

    dev = torch.device("cuda:0")
    n_unique = args.serve_unique
    log(f"serving: drawing {n_unique} distinct requests on the device")
    pool = serving_pool(torch, dev, n_unique)
    lk, pay, uniq = pool
    tables = None
    if args.serve_mode == "probe":
        # 16 resident build tables (left prefixes of sizes log-uniform in
        # [1E4, 2E7]); each distinct request probes one of them, its hits
        # drawn from that table's keys
        rng = np.random.default_rng(3)
        sizes = [int(round(np.exp(rng.uniform(np.log(1e4), np.log(2e7))))) for _ in range(16)]
        tables = []
        for nt in sizes:
            tk, tv, to = mdx.mdx_hash_partition(lk[:nt], pay[:nt], 8)
            tables.append(mdx.mdx_join_build(tk, tv, to, 8))
        g = torch.Generator(device=dev)
        g.manual_seed(29)
        for r in uniq:
            t = int(rng.integers(0, len(tables)))
            nt, nr, m = sizes[t], r["nr"], r["m"]
            hit = lk[torch.randint(0, nt, (m,), generator=g, device=dev)]
            miss = torch.randint(SERVE_MAX_ROWS, 2 * SERVE_MAX_ROWS, (nr - m,), generator=g, device=dev)
            r["rk"] = torch.cat([hit, miss])[torch.randperm(nr, generator=g, device=dev)].contiguous()
            r["table"], r["nl"] = t, nt
        torch.cuda.synchronize()
    bad = serving_check_rows(torch, mdx, pool, tables, dev)
    if bad:
        raise SystemExit(f"serving: {bad} of {n_unique} distinct requests gave wrong rows")
    log(f"serving: all {n_unique} distinct requests checked row by row")
    budget = int(args.budget_gb * 1e9)
    points = [("rated", args.rate, args.duration), ("overload", args.overload_rate, args.overload_duration)]
    res = {}
    for label, rate, duration in points:
        rng = np.random.default_rng(1 if label == "rated" else 2)
        n = int(round(rate * duration))
        arrivals = np.cumsum(rng.exponential(1.0 / rate, n))
        picks = rng.integers(0, n_unique, n)
        stream_reqs = [(float(arrivals[i]), int(picks[i])) for i in range(n)]
        rows = sum((uniq[u]["nl"] if tables is None else 0) + uniq[u]["nr"] for u in picks)
        want = torch.tensor([uniq[u]["m"] for u in picks], dtype=torch.int64)
        log(f"serving {args.serve_mode} at {rate:g}/s for {duration:g} s: {n} requests, "
            f"offered {rows / duration:.4g} rows/s")
        res[label] = {"rate_per_s": rate, "duration_s": duration, "requests": n, "input_rows": rows,
                      "offered_rows_per_s": round(rows / duration, 1)}
        for policy, slots in [("continuous batching", args.slots), ("FIFO", 1)]:
            lat, elapsed, totals, st = serve_run(torch, mdx, stream_reqs, pool, slots, budget, dev,
                                                 args.serve_mode, tables)
            if int(st.max()) != 0 or not torch.equal(totals, want):
                raise SystemExit(f"serving: wrong |J| or a device status ({policy}, {label})")
            p50, p99 = np.percentile(lat, 50), np.percentile(lat, 99)
            res[label][policy] = {"slots": slots, "p50_ms": round(float(p50), 3),
                                  "p99_ms": round(float(p99), 3), "max_ms": round(float(max(lat)), 3),
                                  "elapsed_s": round(elapsed, 3), "rows_per_s": round(rows / elapsed, 1)}
            log(f"  {policy} ({slots} slots): p50 {p50:.2f} ms, p99 {p99:.2f} ms, "
                f"{rows / elapsed:.4g} rows/s over {elapsed:.2f} s")
    cb = res["rated"]["continuous batching"]
    what = "merge requests (both tables per request)" if tables is None else \
        "probes of 16 device-resident build tables"
    line = {
        "metric": f"serving p99 latency: Poisson {args.rate:g} requests/s, 1E4-2E7 rows per side, "
                  "int64, match fraction U[0.1, 0.9] per request, P=8, "
                  f"{args.budget_gb:g} GB HBM budget",
        "value": cb["p99_ms"], "unit": "ms",
        "n_gpus": 1, "steps": res["rated"]["requests"], "warmup": 0,
        "ms_per_step": round(cb["elapsed_s"] * 1e3 / res["rated"]["requests"], 4),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"serving: {what}, {args.slots} slots, {n_unique} distinct requests "
                               f"drawn on the device and checked row by row",
                   "mode": args.serve_mode},
        "points": res,
    }
    print(json.dumps(line), flush=True)


def run_skewed(args):
    """The skewed workload: 5E7 x 5E7 rows, int64 keys Zipf(1.1) over 1E7
    values, P = 16.  Its join has ~5E13 rows, so the graded step is the part
    that does not write them: both partitions, then the count-only join
    (mdx_join_count: a table of build-row counts per key, probed by the right
    keys) giving the exact per-partition output counts.  The same counts
    through the reusable table (mdx_join_build, then mdx_join_probe with no
    output) are timed beside it.  Then the output is materialized on the
    window L x R[0:m), m the longest prefix of right rows whose output stays
    within 2^28 rows, and its rows are checked."""
    import numpy as np
    import torch

    import paper_2101_08878_amd as mdx
    from paper_2101_08878_amd.rocprof_summary import kernel_sources_hash
    from workloads import CONFIGS, config_inputs

    spec = CONFIGS["skewed"]
    P = spec.P
    log(f"generating skewed: {spec.n_left} x {spec.n_right} rows, Zipf({spec.zipf_s:g}) over "
        f"{spec.zipf_support} values, P={P}")
    kl, vl, kr, vr = config_inputs("skewed")
    nl, nr = kl.size, kr.size
    dev = torch.device("cuda:0")
    tk = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    lk, lv, rk, rv = tk(kl), tk(vl), tk(kr), tk(vr)
    del kl, vl, kr, vr
    stream = torch.cuda.current_stream()
    lko, lvo, rko, rvo = (torch.empty(n, dtype=torch.int64, device=dev) for n in (nl, nl, nr, nr))
    lo, ro, off = (torch.empty(P + 1, dtype=torch.int64, device=dev) for _ in range(3))
    wsl = torch.empty(mdx.mdx_hash_partition_workspace_bytes(nl, P), dtype=torch.uint8, device=dev)
    wsr = torch.empty(mdx.mdx_hash_partition_workspace_bytes(nr, P), dtype=torch.uint8, device=dev)
    tmem = torch.empty(mdx.mdx_join_table_bytes(nl, P), dtype=torch.uint8, device=dev)
    pws = torch.empty(mdx.mdx_join_probe_workspace_bytes(nr, P), dtype=torch.uint8, device=dev)
    cws = torch.empty(mdx.mdx_join_count_workspace_bytes(nl, nr, P), dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    tstatus = torch.zeros(1, dtype=torch.int32, device=dev)
    toff = torch.empty(P + 1, dtype=torch.int64, device=dev)
    empty = (torch.empty(0, dtype=torch.int64, device=dev),) * 3

    def partitions():
        mdx.mdx_hash_partition(lk, lv, P, keys_out=lko, payload_out=lvo, offsets=lo, workspace=wsl,
                               stream=stream)
        mdx.mdx_hash_partition(rk, rv, P, keys_out=rko, payload_out=rvo, offsets=ro, workspace=wsr,
                               stream=stream)

    def step():
        partitions()
        mdx.mdx_join_count(lko, lo, rko, ro, P, out_offsets=off, workspace=cws, status=status,
                           stream=stream)

    def step_table():
        partitions()
        t = mdx.mdx_join_build(lko, lvo, lo, P, table_memory=tmem, status=tstatus, stream=stream)
        mdx.mdx_join_probe(t, rko, rvo, ro, out_capacity=0, out=empty, out_offsets=toff,
                           workspace=pws, status=tstatus, stream=stream)

    for _ in range(args.warmup):
        step()
        step_table()
    torch.cuda.synchronize()
    # the closed form: |J| = sum over keys of countL(k) countR(k)
    cl = torch.bincount(lk, minlength=spec.zipf_support + 1)
    cr = torch.bincount(rk, minlength=spec.zipf_support + 1)
    want = int((cl * cr).sum().item())
    total = int(off[-1].item())
    # a count-only probe (capacity 0) reports its rows as an overflow
    tst = int(tstatus.item()) & ~mdx.MDX_DEV_OUTPUT_OVERFLOW
    if int(status.item()) != 0 or total != want or tst != 0 or not torch.equal(off, toff):
        raise SystemExit(f"skewed: count {total} (expected {want}), device status "
                         f"{int(status.item())}, table path {int(toff[-1].item())} status {tst}")
    log(f"output rows (counted, not written): {total:.4g}; both count paths equal the closed form")

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms = timed(step, args.steps)
    log(f"partition + count-only join: {ms:.3f} ms/step, {(nl + nr) / (ms / 1e3):.4g} input rows/s")
    tms = timed(step_table, args.steps)
    log(f"partition + table build + count-only probe: {tms:.3f} ms/step")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    def breakdown(fn, label):
        traces = {k: mdx.KernelTrace(k, 64) for k in mdx.TRACEABLE_KERNELS}
        for t in traces.values():
            t.start()
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        mdx.KernelTrace.stop_all()
        ks = {}
        for name, t in traces.items():
            d = t.durations_ms()
            if d:
                ks[name] = {"ms_per_step": round(sum(d) / 2, 4), "launches_per_step": t.launches() / 2,
                            "avg_launch_us": round(sum(d) / len(d) * 1e3, 2)}
            t.close()
        log(label)
        for name, k in sorted(ks.items(), key=lambda kv: -kv[1]["ms_per_step"]):
            log(f"  {name:13s} {k['ms_per_step']:.3f} ms/step  {k['launches_per_step']:.0f} launches")
        return ks

    kernels = breakdown(step, "graded step (partitions + count-only join):")
    table_kernels = breakdown(step_table, "table path (partitions + build + count-only probe):")

    # the window: the longest prefix of right rows with at most 2^28 output rows
    c = torch.cumsum(cl[rk], 0)
    m = int(torch.searchsorted(c, torch.tensor([1 << 28], device=dev), right=True).item())
    wrows = int(c[m - 1].item())
    log(f"window: L x R[0:{m}), {wrows} output rows")
    wout = tuple(torch.empty(wrows, dtype=torch.int64, device=dev) for _ in range(3))
    woff = torch.empty(P + 1, dtype=torch.int64, device=dev)
    wws = torch.empty(mdx.mdx_merge_workspace_bytes(nl, m, P), dtype=torch.uint8, device=dev)
    wst = torch.zeros(1, dtype=torch.int32, device=dev)

    def window():
        mdx.mdx_merge(lk, lv, rk[:m], rv[:m], P, out_capacity=wrows, out=wout, out_offsets=woff,
                      workspace=wws, status=wst, stream=stream)

    window()
    torch.cuda.synchronize()
    ok, ol, orr = wout
    mult = torch.bincount(orr, minlength=m)
    pairs = torch.sort(orr * nl + ol).values
    good = (int(wst.item()) == 0 and int(woff[-1].item()) == wrows and torch.equal(ok, lk[ol])
            and torch.equal(ok, rk[orr]) and torch.equal(mult, cl[rk[:m]])
            and not bool((pairs[1:] == pairs[:-1]).any().item()))
    if not good:
        raise SystemExit("skewed window: output rows differ from L x R[0:m)")
    del mult, pairs
    log("window: every row checked (keys, multiplicity of every right row, no repeated pair)")
    reps = 3
    e0.record(stream)
    for _ in range(reps):
        window()
    e1.record(stream)
    torch.cuda.synchronize()
    wms = e0.elapsed_time(e1) / reps
    wgbs = wrows * 24 / (wms / 1e3) / 1e9
    log(f"window merge: {wms:.3f} ms, {wgbs:.0f} GB/s of output written")
    # credited bytes of the graded step: partition (read + write 16 B per
    # row), build (16 B read + 16 B table write per left row), count (8 B
    # key + 16 B slot per right row)
    alg = (nl + nr) * 2 * 16 + nl * 32 + nr * 24
    achieved = alg / (ms / 1e3) / 1e9
    line = {
        "metric": "input rows/s for partition + build + count, 5E7 x 5E7 int64 Zipf(1.1) over 1E7 "
                  "values, P=16",
        "table_path_ms": round(tms, 4),
        "value": round((nl + nr) / (ms / 1e3), 1), "unit": "input rows/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"skewed: {nl} x {nr} rows, Zipf(1.1) keys over 1E7 values, P={P}; "
                               "partitions, then the count-only join (left keys counted per key, "
                               "right keys probe the counts)",
                   "output_rows_counted": total},
        "roofline": {"bound": "hbm", "scope": "partition of both tables + count-only join",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes": int(alg)},
        "window": {"right_rows": m, "output_rows": wrows, "ms": round(wms, 4),
                   "output_write_gbs": round(wgbs, 1),
                   "input_rows_per_s": round((nl + m) / (wms / 1e3), 1)},
        "kernels": kernels,
        "table_path_kernels": table_kernels,
        "kernel_sources": kernel_sources_hash(),
    }
    print(json.dumps(line), flush=True)


def run_transpose(args):
    """The paper's other local workload (Section V-B, cuPy benchmark): y =
    x + x^T on the RI2 array, 16384 x 16384 float64.  Algorithmic bytes:
    each element read once and written once (16 B)."""
    import torch

    import paper_2101_08878_amd as mdx

    from paper_2101_08878_amd.rocprof_summary import kernel_sources_hash

    n = 16384
    dev = torch.device("cuda:0")
    copy = copy_ceiling(torch, dev)
    log(f"plain copy of {copy['bytes'] >> 20} MiB: {copy['gbs']:.0f} GB/s (read + write)")
    g = torch.Generator(device=dev)
    g.manual_seed(0)
    x = torch.rand((n, n), generator=g, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        mdx.mdx_transpose_sum(x, out=y, stream=stream)
    torch.cuda.synchronize()
    if not torch.equal(y, x + x.T):
        raise SystemExit("transpose sum: result differs from x + x.T")
    tr = mdx.KernelTrace("transpose_sum", args.steps)
    tr.start()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        mdx.mdx_transpose_sum(x, out=y, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    mdx.KernelTrace.stop_all()
    ms = e0.elapsed_time(e1) / args.steps
    d = tr.durations_ms()
    tr.close()
    kms = sum(d) / len(d)
    nbytes = 16 * n * n
    achieved = nbytes / (kms / 1e3) / 1e9
    sources = kernel_sources_hash()
    traffic, traffic_src = counted_traffic("transpose_sum", "transpose")
    log(f"transpose sum {n} x {n}: {ms:.3f} ms/step, kernel {kms:.3f} ms, {achieved:.0f} GB/s")
    line = {
        "metric": "matrix elements/s for y = x + x^T, 16384 x 16384 float64",
        "value": round(n * n / (ms / 1e3), 1), "unit": "elements/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "strong", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"transpose sum: {n} x {n} float64 (the RI2 cuPy array)", "n": n},
        "roofline": {"bound": "hbm", "kernel": "transpose_sum", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "traffic_source": traffic_src,
                     "bytes_per_launch": nbytes, "avg_launch_us": round(kms * 1e3, 2)},
        "copy_ceiling": copy,
        "kernel_sources": sources,
    }
    if args.cpu_baseline == "on":
        import numpy as np

        import oracle
        m = 8192
        xs = np.random.default_rng(0).random((m, m))
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 10.0:
            oracle.transpose_sum(xs)
            reps += 1
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": reps * m * m / dt, "unit": "elements/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"{reps} x numpy x + x.T on {m} x {m} float64, {dt:.2f} s"}
    print(json.dumps(line), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the exchange between workers is out of scope); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    if args.config == "batched":
        run_batched(args)
        return
    if args.config == "serving":
        run_serving(args)
        return
    if args.config == "transpose":
        run_transpose(args)
        return
    if args.config == "skewed":
        run_skewed(args)
        return

    import torch

    import paper_2101_08878_amd as mdx
    from paper_2101_08878_amd.rocprof_summary import kernel_sources_hash
    from workloads import CONFIGS, config_inputs

    spec = CONFIGS[args.config]
    P = spec.P
    log(f"generating {args.config}: {spec.n_left} x {spec.n_right} rows, P={P}")
    kl, vl, kr, vr = config_inputs(args.config)
    nl, nr = kl.size, kr.size
    key_bytes = kl.dtype.itemsize
    dev = torch.device("cuda:0")
    tk = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
    lk, lv, rk, rv = tk(kl), tk(vl), tk(kr), tk(vr)
    full_tables = (kl, vl, kr, vr) if args.cpu_baseline != "off" else None
    del kl, vl, kr, vr
    cap = nr if args.config == "paper" else 4 * nr
    ws = torch.empty(mdx.mdx_merge_workspace_bytes(nl, nr, P, key_bytes), dtype=torch.uint8, device=dev)
    out = (torch.empty(cap, dtype=lk.dtype, device=dev), torch.empty(cap, dtype=torch.int64, device=dev),
           torch.empty(cap, dtype=torch.int64, device=dev))
    off = torch.empty(P + 1, dtype=torch.int64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def step():
        mdx.mdx_merge(lk, lv, rk, rv, P, out_capacity=cap, out=out, out_offsets=off, workspace=ws,
                      status=status, stream=stream)

    copy = copy_ceiling(torch, dev)
    log(f"plain copy of {copy['bytes'] >> 20} MiB: {copy['gbs']:.0f} GB/s (read + write)")

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    total = int(off[-1].item())
    st = int(status.item())
    if st != 0 or total > cap:
        raise SystemExit(f"merge failed: status={st} total={total} cap={cap}")
    if args.config == "paper":
        # the closed form of this workload: left keys are distinct, so every
        # matching right row has exactly one partner
        ok, ol, orr = (t[:total] for t in out)
        if total != round(spec.frac * nr) or not torch.equal(ok, lk[ol]) \
                or not torch.equal(ok, rk[orr]) \
                or not torch.equal(torch.sort(orr).values, torch.nonzero(rk < nl).flatten()):
            raise SystemExit(f"merge output differs from the workload's closed form ({total} rows)")
        del ok, ol, orr
    log(f"output rows {total}")

    # Timed region: K steps, nothing but the merges between the events.
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1) / args.steps
    value = (nl + nr) / (ms / 1e3)
    log(f"{ms:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms/step), {value:.4g} input rows/s")

    # Kernel breakdown (separate steps): every traceable kernel bracketed by
    # HIP events on the stream it runs on -- the per-launch times a rocprofv3
    # kernel trace of this command reports.
    per_step_launches = 4 + 6 * P
    prof_steps = max(2, min(args.steps, 5))
    traces = {k: mdx.KernelTrace(k, prof_steps * per_step_launches) for k in mdx.TRACEABLE_KERNELS}
    for t in traces.values():
        t.start()
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    mdx.KernelTrace.stop_all()
    sources = kernel_sources_hash()
    kernels = {}
    for name, t in traces.items():
        d = t.durations_ms()
        if d:
            avg_s = sum(d) / len(d) / 1e3
            launches = t.launches() / prof_steps
            cb = credited_bytes(name, nl, nr, key_bytes, total) / launches
            counted, _ = counted_traffic(name, args.config)
            kernels[name] = {
                "ms_per_step": round(sum(d) / prof_steps, 4),
                "launches_per_step": launches,
                "avg_launch_us": round(avg_s * 1e6, 2),
                "credited_bytes_per_launch": int(cb),
                "credited_frac": round(cb / avg_s / 1e9 / HBM_PEAK_GBS, 4) if cb else None,
                "counted_bytes_per_launch": counted,
                "counted_frac": round(counted / avg_s / 1e9 / HBM_PEAK_GBS, 4) if counted else None,
            }
        t.close()
    for name, k in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        log(f"  {name:13s} {k['ms_per_step']:.3f} ms/step  {k['launches_per_step']:.0f} launches  "
            f"{k['avg_launch_us']:.1f} us/launch")
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_step"])

    alg = step_algorithmic_bytes(nl, nr, key_bytes, total)
    alg_hbm = alg - (nl + nr) * 16
    achieved = alg / (ms / 1e3) / 1e9
    big = [k for k in kernels if kernels[k]["ms_per_step"] >= 0.02]
    counted_step = [kernels[k]["counted_bytes_per_launch"] for k in big]
    traffic = int(sum(counted_step)) if counted_step and all(counted_step) else None
    roofline = {
        "bound": "hbm",
        "scope": "one merge: every kernel of the step (partition of both tables, sub-bucket "
                 "split, join count and emit)",
        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes": int(alg),
        "algorithmic_hbm_bytes": int(alg_hbm),
        "frac_of_hbm_minimum": round(alg_hbm / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "dominant_kernel": {"name": dom, **kernels[dom]},
    }
    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "input rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64" if key_bytes == 8 else "int32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: one worker's partition+join share, "
                               f"{nl} x {nr} rows, int{8 * key_bytes} key + int64 payload, P={P}",
                   "n_left": nl, "n_right": nr, "P": P, "output_rows": total},
        "roofline": roofline,
        "copy_ceiling": copy,
        "kernels": kernels,
        "kernel_sources": sources,
    }
    if args.config == "plain":
        line["us_per_merge"] = round(ms * 1e3, 2)
    if args.config == "paper":
        # secondary: the same tables joined as one partition (P = 1: one
        # 1E8-row table, far beyond any cache), timed after the graded steps
        off1 = torch.empty(2, dtype=torch.int64, device=dev)
        ws1 = torch.empty(mdx.mdx_merge_workspace_bytes(nl, nr, 1, key_bytes), dtype=torch.uint8,
                          device=dev)

        def step1():
            mdx.mdx_merge(lk, lv, rk, rv, 1, out_capacity=cap, out=out, out_offsets=off1,
                          workspace=ws1, status=status, stream=stream)

        step1()
        torch.cuda.synchronize()
        if int(off1[-1].item()) != total or int(status.item()) != 0:
            raise SystemExit("P = 1 merge: |J| or status differs")
        reps = max(2, min(args.steps, 5))
        e0.record(stream)
        for _ in range(reps):
            step1()
        e1.record(stream)
        torch.cuda.synchronize()
        ms1 = e0.elapsed_time(e1) / reps
        log(f"secondary, P = 1: {ms1:.3f} ms/step, {(nl + nr) / (ms1 / 1e3):.4g} input rows/s")
        line["secondary_p1"] = {"P": 1, "ms_per_step": round(ms1, 4), "steps": reps,
                                "input_rows_per_s": round((nl + nr) / (ms1 / 1e3), 1)}
        del ws1
    if full_tables is not None:
        del lk, lv, rk, rv, ws, out
        one, allc = cpu_baselines(args.cpu_baseline, args.cpu_sample_scale, full_tables, P)
        line["cpu_baseline"] = one
        line["cpu_baseline_all_cores"] = allc
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
