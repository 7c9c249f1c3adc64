"""Formats rocprofv3 output as a short text summary.

    python -m paper_2211_10979_amd.profile_summary <rocprofv3 output dir> [--kernel NAME]

Reads whatever the directory holds:
  * `*_kernel_stats.csv` (from --kernel-trace --stats --output-format csv):
    calls, total, average, min and max duration per kernel;
  * `*_results.db` (rocprofv3's SQLite output): the same per-kernel figures
    from its dispatch table;
  * `*_counter_collection.csv` (from --pmc): per-kernel average of each
    counter over the dispatches of that kernel (optionally only those whose
    value reaches --min-value, e.g. to leave out launches that returned at
    once);
  * with --by-grid, `*_kernel_trace.csv` (from --kernel-trace): the same
    duration figures per kernel and grid size, which tells apart launches of
    one kernel over different extents.
Durations are in microseconds.
"""

from __future__ import annotations

import argparse
import csv
import glob
import os
import sqlite3
import statistics
from collections import defaultdict


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0].strip()


def kernel_stats_csv(path):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            calls = int(r["Calls"])
            rows.append(dict(kernel=_short(r["Name"]), calls=calls, total_us=float(r["TotalDurationNs"]) / 1e3,
                             avg_us=float(r["AverageNs"]) / 1e3, min_us=float(r["MinNs"]) / 1e3,
                             max_us=float(r["MaxNs"]) / 1e3))
    return rows


def kernel_stats_db(path):
    db = sqlite3.connect(path)
    cur = db.cursor()
    durs = defaultdict(list)
    for name, start, end in cur.execute("select name, start, end from kernels"):
        durs[_short(name)].append((end - start) / 1e3)
    rows = []
    for k, v in durs.items():
        rows.append(dict(kernel=k, calls=len(v), total_us=sum(v), avg_us=statistics.fmean(v), min_us=min(v),
                         max_us=max(v)))
    rows.sort(key=lambda r: -r["total_us"])
    return rows


def counters_csv(path, min_value=0.0):
    """Per kernel and counter: (dispatches, mean) over the dispatches whose
    value is at least `min_value` (0: all of them)."""
    acc = defaultdict(lambda: defaultdict(list))
    with open(path) as f:
        for r in csv.DictReader(f):
            acc[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = {}
    for k, cs in acc.items():
        out[k] = {}
        for c, v in cs.items():
            sel = [x for x in v if x >= min_value] or [0.0]
            out[k][c] = (len(sel) if min_value > 0 else len(v), statistics.fmean(sel))
    return out


def kernel_trace_by_grid(path):
    """Per (kernel, grid size in threads): dispatch durations in us."""
    durs = defaultdict(list)
    with open(path) as f:
        for r in csv.DictReader(f):
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            durs[(_short(r["Kernel_Name"]), grid)].append(
                (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return durs


def summarize(directory, kernel=None, min_value=0.0, by_grid=False):
    out = []
    stats = []
    for p in sorted(glob.glob(os.path.join(directory, "**", "*_kernel_stats.csv"), recursive=True)):
        stats = kernel_stats_csv(p)
        out.append(f"source: {os.path.relpath(p, directory)}")
    if not stats:
        for p in sorted(glob.glob(os.path.join(directory, "**", "*_results.db"), recursive=True)):
            stats = kernel_stats_db(p)
            out.append(f"source: {os.path.relpath(p, directory)}")
    if stats:
        out.append("")
        out.append("| kernel | calls | total us | avg us | min us | max us |")
        out.append("|---|---|---|---|---|---|")
        for r in stats:
            if kernel and kernel not in r["kernel"]:
                continue
            out.append(f"| {r['kernel']} | {r['calls']} | {r['total_us']:.1f} | {r['avg_us']:.2f} | "
                       f"{r['min_us']:.2f} | {r['max_us']:.2f} |")
    if by_grid:
        for p in sorted(glob.glob(os.path.join(directory, "**", "*_kernel_trace.csv"), recursive=True)):
            out.append("")
            out.append(f"by grid: {os.path.relpath(p, directory)}")
            out.append("")
            out.append("| kernel | grid threads | calls | avg us | min us | max us |")
            out.append("|---|---|---|---|---|---|")
            for (k, grid), v in sorted(kernel_trace_by_grid(p).items(), key=lambda kv: -sum(kv[1])):
                if kernel and kernel not in k:
                    continue
                out.append(f"| {k} | {grid} | {len(v)} | {statistics.fmean(v):.2f} | {min(v):.2f} | {max(v):.2f} |")
    for p in sorted(glob.glob(os.path.join(directory, "**", "*_counter_collection.csv"), recursive=True)):
        cs = counters_csv(p, min_value)
        out.append("")
        sel = f", dispatches with value >= {min_value:g}" if min_value > 0 else ""
        out.append(f"counters: {os.path.relpath(p, directory)} (average per dispatch{sel})")
        out.append("")
        out.append("| kernel | counter | dispatches | value |")
        out.append("|---|---|---|---|")
        for k, vals in sorted(cs.items()):
            if kernel and kernel not in k:
                continue
            for c, (nd, v) in sorted(vals.items()):
                out.append(f"| {k} | {c} | {nd} | {v:.1f} |")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("directory")
    ap.add_argument("--kernel", default=None)
    ap.add_argument("--min-value", type=float, default=0.0,
                    help="counters: average only dispatches whose value is at least this")
    ap.add_argument("--by-grid", action="store_true",
                    help="also durations per kernel and grid size, from the kernel trace")
    a = ap.parse_args()
    print(summarize(a.directory, a.kernel, a.min_value, a.by_grid))


if __name__ == "__main__":
    main()
