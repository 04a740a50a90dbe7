"""Summarise rocprofv3 CSV output (kernel stats + kernel trace) as short text.

    python -m paper_2210_08494_amd.profsum <dir-with-csv> <prefix> [--kernel SUBSTR] [--grid X,Y]
        [--top N] [--cmd "the command that produced the CSV"]

Prints the top kernels by total time, and, for --kernel, the dispatch count,
average and total duration of that kernel restricted to dispatches whose grid
matches --grid (e.g. the grouped launches of one shape).
"""
from __future__ import annotations

import argparse
import csv
import os
import re


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("prefix")
    ap.add_argument("--kernel", action="append", default=[])
    ap.add_argument("--grid", action="append", default=[])
    ap.add_argument("--top", type=int, default=12)
    ap.add_argument("--cmd", default="")
    a = ap.parse_args()
    stats = list(csv.DictReader(open(os.path.join(a.dir, f"{a.prefix}_kernel_stats.csv"))))
    trace = list(csv.DictReader(open(os.path.join(a.dir, f"{a.prefix}_kernel_trace.csv"))))
    if a.cmd:
        print(f"command: {a.cmd}")
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    print(f"total kernel time {tot / 1e6:.2f} ms in {sum(int(r['Calls']) for r in stats)} dispatches")
    print(f"{'total_ms':>10} {'pct':>6} {'calls':>7} {'avg_us':>10}  kernel")
    for r in stats[:a.top]:
        name = re.sub(r"\(.*", "", r["Name"])[:100]
        print(f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['Percentage']):6.2f} {int(r['Calls']):7d} "
              f"{float(r['AverageNs']) / 1e3:10.2f}  {name}")
    for i, k in enumerate(a.kernel):
        grid = a.grid[i] if i < len(a.grid) else ""
        sel = [r for r in trace if k in r["Kernel_Name"]]
        if grid:
            gx, gy = grid.split(",")
            sel = [r for r in sel if r["Grid_Size_X"] == gx and r["Grid_Size_Y"] == gy]
        durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in sel]
        if durs:
            print(f"kernel '{k}' grid ({grid or 'any'}): {len(durs)} dispatches, avg {sum(durs) / len(durs):.2f} us, "
                  f"total {sum(durs) / 1e3:.3f} ms, min {min(durs):.2f} us, max {max(durs):.2f} us")


if __name__ == "__main__":
    main()
