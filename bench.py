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
    ap.add_argument("--config", default="paper", choices=["paper", "plain"])
    ap.add_argument("--cpu-baseline", default="on", choices=["on", "off"])
    ap.add_argument("--cpu-sample-scale", type=float, default=0.2,
                    help="fraction of the workload the oracle runs on the host")
    return ap.parse_args()


def counted_traffic(kernel, workload, sources):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/*traffic.json, written by paper_2101_08878_amd.rocprof_summary
    from FETCH_SIZE and WRITE_SIZE runs), or None when there is none for the
    current kernel sources."""
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*traffic.json"))):
        with open(f) as fh:
            t = json.load(fh)
        if t.get("kernel") == kernel and t.get("workload") == workload \
                and t.get("kernel_sources") == sources:
            return t["traffic_bytes_per_launch"], os.path.relpath(f, ROOT)
    return None, None


def algorithmic_bytes_per_step(kernel, nl, nr, key_bytes, total_out):
    """Bytes the method itself moves in the given kernel per step (overheads
    such as the histogram pre-read, table clearing and extra probes are not
    credited).  Partition: read and write key + payload of every row.  Build:
    read a left row, write its 16-byte slot.  Probe: read a right row and
    one 16-byte slot, write 3 x 8 bytes per output row."""
    row = key_bytes + 8
    if kernel == "part_scatter":
        return (nl + nr) * 2 * row
    if kernel == "rj_join":
        # build: read a left row, write it to the table; probe: read a right
        # row and one table entry; output rows
        return nl * (row + 16) + nr * (row + 16) + total_out * (key_bytes + 16)
    if kernel == "tbl_insert":
        return nl * (row + 16)
    if kernel == "probe_chain":
        return nr * (row + 16) + total_out * (key_bytes + 16)
    return 0


def cpu_baseline(scale):
    import numpy as np  # noqa: F401

    import oracle
    from workloads import config_inputs

    kl, vl, kr, vr = config_inputs("paper", scale=scale)
    n = kl.size + kr.size
    log(f"cpu baseline: oracle on {kl.size} x {kr.size} rows (single thread)")
    t0 = time.perf_counter()
    oracle.hash_partition(kl, vl, 32)
    oracle.hash_partition(kr, vr, 32)
    res = oracle.join(kl, vl, kr, vr)
    dt = time.perf_counter() - t0
    log(f"cpu baseline: {dt:.2f} s, |J| = {res['total']}")
    return {
        "value": n / dt,
        "unit": "input rows/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"same generator at {scale:g} scale: {kl.size} x {kr.size} rows, P=32; "
                  f"stable counting-sort partition of both tables + sort-merge join, "
                  f"{dt:.2f} s on one host thread",
    }


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


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the exchange between workers is out of scope); run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

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
    del kl, vl
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
    if args.config == "paper" and total != round(spec.frac * nr):
        raise SystemExit(f"unexpected output size {total}")
    log(f"output rows {total}")

    # Breakdown pass (not the timed region): every traceable kernel bracketed
    # by events, to find the dominant one.
    per_step_launches = 4 + 6 * P
    prof_steps = 2
    traces = {k: mdx.KernelTrace(k, prof_steps * per_step_launches) for k in mdx.TRACEABLE_KERNELS}
    for t in traces.values():
        t.start()
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    mdx.KernelTrace.stop_all()
    kernels = {}
    for name, t in traces.items():
        d = t.durations_ms()
        if d:
            kernels[name] = {"ms_per_step": sum(d) / prof_steps,
                             "launches_per_step": t.launches() / prof_steps,
                             "avg_launch_ms": sum(d) / len(d)}
        t.close()
    for name, k in sorted(kernels.items(), key=lambda kv: -kv[1]["ms_per_step"]):
        log(f"  {name:13s} {k['ms_per_step']:.3f} ms/step  {k['launches_per_step']:.0f} launches  "
            f"{k['avg_launch_ms'] * 1e3:.1f} us/launch")
    credited = {k: v for k, v in kernels.items()
                if algorithmic_bytes_per_step(k, nl, nr, key_bytes, total) > 0}
    dom = max(credited, key=lambda k: credited[k]["ms_per_step"])

    # Timed region: K steps; only the dominant kernel is bracketed by events.
    dtrace = mdx.KernelTrace(dom, args.steps * per_step_launches)
    dtrace.start()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps (dominant kernel {dom})")
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    mdx.KernelTrace.stop_all()
    ms = e0.elapsed_time(e1) / args.steps
    value = (nl + nr) / (ms / 1e3)
    log(f"{ms:.3f} ms/step (wall {wall / args.steps * 1e3:.3f} ms/step), {value:.4g} input rows/s")
    d = dtrace.durations_ms()
    kd = {"launches_per_step": dtrace.launches() / args.steps, "avg_launch_ms": sum(d) / len(d)}
    dtrace.close()
    bytes_per_launch = algorithmic_bytes_per_step(dom, nl, nr, key_bytes, total) / kd["launches_per_step"]
    achieved = bytes_per_launch / (kd["avg_launch_ms"] / 1e3) / 1e9
    sources = kernel_sources_hash()
    traffic, traffic_src = counted_traffic(dom, args.config, sources)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_source": traffic_src, "bytes_per_launch": int(bytes_per_launch),
                "avg_launch_us": round(kd["avg_launch_ms"] * 1e3, 2)}
    step_bytes = (nl + nr) * 2 * (key_bytes + 8) + (nl + nr) * (key_bytes + 8 + 16) \
        + total * (key_bytes + 16)
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
        "step_hbm_fraction": round(step_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
        "copy_ceiling": copy,
        "kernels": {k: {kk: round(vv, 4) for kk, vv in v.items()} for k, v in kernels.items()},
        "kernel_sources": sources,
    }
    if args.cpu_baseline == "on":
        del lk, lv, rk, rv, ws, out
        line["cpu_baseline"] = cpu_baseline(args.cpu_sample_scale)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
