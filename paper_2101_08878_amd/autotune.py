"""Autotuner of the fused batch (mdx_batch_*).

For every key width and size bucket it times candidate tunings of a
synthetic batch on the device and keeps the fastest in a JSON table
(tuning.json beside this file), which ``FusedBatch(jobs, tuning="table")``
reads merge by merge:

    python -m paper_2101_08878_amd.autotune [--out PATH] [--reps 3]

Knobs (mdx_batch_tuning; they change speed, never results):
  fill       average build rows per sub-bucket as a fraction of an LDS table:
             fuller sub-buckets mean fewer of them (less fixed latency per
             sub-bucket), emptier ones more parallel work for small merges;
  fanout     destinations of the first partition pass: the split between the
             first pass (long coalesced runs) and the segmented second pass;
  part_rows  rows per thread of the first pass's tiles (8: 4096-row tiles,
             2: 1024-row tiles, which suit merges of a few thousand rows).

A batch of a cell draws both sides' sizes log-uniform in the bucket, keys of
the cell's width: left keys a random permutation of [0, nL), right keys 30%
drawn from the left keys and the rest from [nL, 2 nL), payload = row index,
P = 8.  Every timed run's |J| is checked against the number of right rows
drawn from the left.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tuning.json")

# buckets of max(n_left, n_right), rows
BUCKETS = [(1_000, 4_000), (4_000, 16_000), (16_000, 64_000), (64_000, 256_000),
           (256_000, 1_000_000), (1_000_000, 4_000_001)]
FILLS = (0.5, 0.65, 0.8, 0.9)
FANOUTS = (32, 64, 128, 256)
PART_ROWS = (2, 8)
DEFAULT = {"fill": 0.9, "fanout": 128, "part_rows": 8}

_cache: dict = {}


def load(path: str = TABLE) -> dict | None:
    """The tuning table, or None when there is none."""
    if path not in _cache:
        _cache[path] = None
        if os.path.exists(path):
            with open(path) as f:
                _cache[path] = json.load(f)
    return _cache[path]


def lookup(key_bytes: int, rows: int, path: str = TABLE) -> dict:
    """Tuning of a merge with `rows` rows on its larger side: the table's
    cell, or {} (the library's defaults) outside the table."""
    t = load(path)
    if not t:
        return {}
    for c in t["cells"]:
        if c["key_bytes"] == key_bytes and c["lo"] <= rows < c["hi"]:
            return dict(c["tuning"])
    return {}


def _cell_batch(torch, mdx, key_bytes, lo, hi, dev, seed, budget_rows=6e7, max_merges=1024):
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    mean = (hi - lo) / math.log(hi / lo)
    count = int(max(4, min(max_merges, budget_rows / (2 * mean))))
    u = torch.rand((count, 2), generator=g, dtype=torch.float64)
    sizes = torch.exp(math.log(lo) + u * (math.log(hi - 1) - math.log(lo))).round().long().tolist()
    kd = torch.int32 if key_bytes == 4 else torch.int64
    gd = torch.Generator(device=dev)
    gd.manual_seed(seed)
    jobs, matched = [], []
    for nl, nr in sizes:
        m = int(round(0.3 * nr))
        kl = torch.randperm(nl, generator=gd, device=dev, dtype=torch.int64)
        hit = kl[torch.randint(0, nl, (m,), generator=gd, device=dev, dtype=torch.int64)]
        miss = torch.randint(nl, 2 * nl, (nr - m,), generator=gd, device=dev, dtype=torch.int64)
        kr = torch.cat([hit, miss])[torch.randperm(nr, generator=gd, device=dev)]
        j = mdx.MergeJob(kl.to(kd), torch.arange(nl, dtype=torch.int64, device=dev),
                         kr.to(kd).contiguous(), torch.arange(nr, dtype=torch.int64, device=dev),
                         8, max(m, 1))
        j.out = tuple(torch.empty(j.out_capacity, dtype=t, device=dev) for t in (kd, torch.int64,
                                                                                  torch.int64))
        j.out_offsets = torch.empty(9, dtype=torch.int64, device=dev)
        j.status = torch.zeros(1, dtype=torch.int32, device=dev)
        jobs.append(j)
        matched.append(m)
    return jobs, matched, sum(a + b for a, b in sizes)


def _time(torch, mdx, jobs, matched, tuning, reps, stream):
    fb = mdx.FusedBatch(jobs, tuning=tuning)
    try:
        for j in jobs:
            j.out_offsets.fill_(-1)
        fb.run(stream)
        torch.cuda.synchronize()
        got = torch.stack([j.out_offsets[-1] for j in jobs]).cpu().tolist()
        st = torch.cat([j.status for j in jobs]).cpu().tolist()
        if got != matched or any(st):
            raise SystemExit(f"tuning {tuning}: wrong |J| or status")
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fb.run(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    finally:
        fb.close()


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args(argv)

    import torch

    import paper_2101_08878_amd as mdx

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    cands = [{"fill": f, "fanout": o, "part_rows": r} for f in FILLS for o in FANOUTS for r in PART_ROWS]
    cells = []
    t0 = time.perf_counter()
    for kb in (4, 8):
        for lo, hi in BUCKETS:
            jobs, matched, rows = _cell_batch(torch, mdx, kb, lo, hi, dev, args.seed * 7919 + lo + kb)
            torch.cuda.synchronize()
            times = []
            for c in cands:
                times.append(_time(torch, mdx, jobs, matched, c, args.reps, stream))
            best = min(range(len(cands)), key=lambda i: times[i])
            dflt = times[cands.index(DEFAULT)]
            cells.append({"key_bytes": kb, "lo": lo, "hi": hi, "merges": len(jobs), "rows": rows,
                          "tuning": cands[best], "ms": round(times[best], 4),
                          "default_ms": round(dflt, 4), "worst_ms": round(max(times), 4)})
            print(f"key {kb} B, rows [{lo}, {hi}): {len(jobs)} merges, {rows} rows: best "
                  f"{cands[best]} {times[best]:.3f} ms, default {dflt:.3f} ms, worst "
                  f"{max(times):.3f} ms ({time.perf_counter() - t0:.0f} s)", flush=True)
            del jobs
    props = torch.cuda.get_device_properties(dev)
    table = {"device": props.name, "compute_units": props.multi_processor_count,
             "candidates": {"fill": FILLS, "fanout": FANOUTS, "part_rows": PART_ROWS},
             "reps": args.reps, "seed": args.seed,
             "command": "python -m paper_2101_08878_amd.autotune", "cells": cells}
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
        f.write("\n")
    print(f"wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
