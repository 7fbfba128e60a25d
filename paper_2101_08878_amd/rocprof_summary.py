"""Summaries of rocprofv3 output, as committed under profiles/.

Kernel time per kernel (from ``rocprofv3 --kernel-trace --stats``, csv or
rocpd output):

    python -m paper_2101_08878_amd.rocprof_summary trace DIR --title T --cmd C [--note N]

HBM bytes per launch of one kernel from two counter runs (``--pmc
FETCH_SIZE``, then ``--pmc WRITE_SIZE``, csv output), each counter scaled
by what it reads for the plain device-to-device copy that bench.py runs
(``copy_ceiling``: a copy of known size, read = write = COPY_BYTES / 2):

    python -m paper_2101_08878_amd.rocprof_summary traffic FETCH_DIR WRITE_DIR \\
        --kernel part_scatter --workload paper --copy-bytes 2147483648 \\
        --cmd-fetch C1 --cmd-write C2

The traffic summary is JSON; bench.py reports its bytes as the roofline's
``traffic`` while the kernel sources still hash to the recorded value.
"""

from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL = "__amd_rocclr_copyBuffer"


# The source file that defines each traced kernel.
KERNEL_FILES = {
    "part_hist": "partition.hip", "part_scatter": "partition.hip", "seg_hist": "partition.hip",
    "seg_scatter": "partition.hip", "rj_join": "rjoin.hip", "transpose_sum": "transpose.hip",
    "transpose_sum_tiles": "transpose.hip",
}
SHARED_FILES = ("mdx_device.hpp", "mdx_internal.hpp")


_CODE_TOKENS = re.compile(r'"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'|//[^\n]*|/\*.*?\*/|\s+', re.S)


def code_of(text: str) -> str:
    """C/C++ source without its comments, whitespace runs collapsed to one
    space (string and character literals kept as they are)."""
    def keep(m):
        t = m.group(0)
        if t.startswith("//") or t.startswith("/*"):
            return " "
        return " " if t.isspace() else t
    return re.sub(r"\s+", " ", _CODE_TOKENS.sub(keep, text)).strip()


def kernel_sources_hash(kernel: str | None = None) -> str:
    """Hash of the code a kernel is built from (its own file and the shared
    device headers; every HIP/C++ source when the kernel is not known),
    comments and layout aside: counter figures taken on other code no longer
    describe it."""
    csrc = os.path.join(HERE, "csrc")
    own = KERNEL_FILES.get(kernel or "")
    files = sorted((own,) + SHARED_FILES) if own else sorted(os.listdir(csrc))
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update((f + "\n" + code_of(fh.read())).encode())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    name = name.replace("void ", "").replace("mdx::(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", name).strip()


def _trace_rows(d):
    """(name, calls, total_ns, average_ns, percent) per kernel."""
    stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
    if stats:
        rows = []
        with open(stats[0]) as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]),
                             float(r["AverageNs"]), float(r["Percentage"])))
        return rows
    dbs = glob.glob(os.path.join(d, "**", "*_results.db"), recursive=True)
    if not dbs:
        raise SystemExit(f"no kernel stats under {d}")
    cur = sqlite3.connect(dbs[0]).cursor()
    q = "select name, total_calls, total_duration, average, percentage from top_kernels"
    return [(n, int(c), float(t) * 1e3, float(a) * 1e3, float(p)) for n, c, t, a, p in cur.execute(q)]


def trace(args):
    rows = sorted(_trace_rows(args.dir), key=lambda r: -r[2])
    if args.include:
        rows = [r for r in rows if re.search(args.include, r[0])]
    out = [f"# {args.title}", "", "Command (run from the repository root on one MI355X):", "",
           "```", args.cmd, "```", ""]
    if args.note:
        out += [args.note, ""]
    out += ["| kernel | calls | total (us) | average (us) | % |", "|---|---:|---:|---:|---:|"]
    for n, c, t, a, p in rows:
        out.append(f"| `{short_name(n)}` | {c} | {t / 1e3:.1f} | {a / 1e3:.2f} | {p:.2f} |")
    print("\n".join(out))


def _counter(d, counter):
    """{short kernel name: [value per dispatch]} for one counter (KiB)."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    per = {}
    with open(files[0]) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                per.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return per


def _kernel_values(per, kernel):
    vals = [v for name, vs in per.items() if name.split("<")[0] == kernel for v in vs]
    if not vals:
        raise SystemExit(f"kernel {kernel} not in the counter output")
    return vals


def traffic(args):
    fetch, write = _counter(args.fetch_dir, "FETCH_SIZE"), _counter(args.write_dir, "WRITE_SIZE")
    half = args.copy_bytes / 2
    # the copy's dispatches of the full size: the largest readings
    cf = sorted(fetch[COPY_KERNEL])[-3:]
    cw = sorted(write[COPY_KERNEL])[-3:]
    fetch_scale = half / (sum(cf) / len(cf) * 1024)
    write_scale = half / (sum(cw) / len(cw) * 1024)
    kf, kw = _kernel_values(fetch, args.kernel), _kernel_values(write, args.kernel)
    f_kib, w_kib = sum(kf) / len(kf), sum(kw) / len(kw)
    res = {
        "kernel": args.report_as or args.kernel,
        "device_kernel": args.kernel,
        "workload": args.workload,
        "kernel_sources": kernel_sources_hash(args.report_as or args.kernel),
        "fetch_kib_per_launch": round(f_kib, 1),
        "write_kib_per_launch": round(w_kib, 1),
        "launches": [len(kf), len(kw)],
        "copy_bytes": args.copy_bytes,
        "copy_fetch_kib": round(sum(cf) / len(cf), 1),
        "copy_write_kib": round(sum(cw) / len(cw), 1),
        "fetch_scale": round(fetch_scale, 4),
        "write_scale": round(write_scale, 4),
        "read_bytes_per_launch": int(f_kib * 1024 * fetch_scale),
        "write_bytes_per_launch": int(w_kib * 1024 * write_scale),
        "traffic_bytes_per_launch": int(f_kib * 1024 * fetch_scale + w_kib * 1024 * write_scale),
        "commands": [args.cmd_fetch, args.cmd_write],
    }
    json.dump(res, sys.stdout, indent=1)
    print()


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    t.add_argument("--note", default="")
    t.add_argument("--include", default="", help="only kernels whose name matches this regex")
    c = sub.add_parser("traffic")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--kernel", required=True, help="device kernel name (before template args)")
    c.add_argument("--report-as", default="", help="name bench.py traces the kernel by")
    c.add_argument("--workload", required=True)
    c.add_argument("--copy-bytes", type=int, required=True)
    c.add_argument("--cmd-fetch", required=True)
    c.add_argument("--cmd-write", required=True)
    args = ap.parse_args(argv)
    trace(args) if args.what == "trace" else traffic(args)


if __name__ == "__main__":
    main()
