"""Summarise rocprofv3 CSV output (kernel stats + kernel trace) as short text.

    python -m paper_2210_08494_amd.profsum <dir-with-csv> <prefix> [--kernel SUBSTR] [--grid X,Y]
        [--top N] [--cmd "the command that produced the CSV"]
    python -m paper_2210_08494_amd.profsum --pmc <dir> <prefix> [--trace-dir D --trace-prefix P]
        [--cmd ...]

Prints the top kernels by total time, and, for --kernel, the dispatch count,
average and total duration of that kernel restricted to dispatches whose grid
matches --grid (e.g. the grouped launches of one shape).

With --pmc: per (kernel, grid) the average of each collected counter per
dispatch (FETCH_SIZE / WRITE_SIZE are in KiB), with the run's last dispatch
(a plain device copy of known size) as the calibration reference, and, when a
kernel trace of the same command is given, the average duration of the same
(kernel, grid) and the bytes per second it implies.
"""
from __future__ import annotations

import argparse
import csv
import os
import re


def _col(row, *names):
    for n in names:
        if n in row:
            return row[n]
    raise KeyError(names)


def _grid(row):
    try:
        return ",".join(_col(row, f"Grid_Size_{a}") for a in "XYZ")
    except KeyError:
        return _col(row, "Grid_Size")


def pmc_main(argv):
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("prefix")
    ap.add_argument("--trace-dir", default="")
    ap.add_argument("--trace-prefix", default="")
    ap.add_argument("--cmd", action="append", default=[])
    ap.add_argument("--top", type=int, default=20)
    a = ap.parse_args(argv)
    rows = list(csv.DictReader(open(os.path.join(a.dir, f"{a.prefix}_counter_collection.csv"))))
    disp = {}
    for r in rows:
        did = int(_col(r, "Dispatch_Id", "Correlation_Id"))
        d = disp.setdefault(did, {"name": re.sub(r"\(.*", "", _col(r, "Kernel_Name")), "grid": _grid(r), "c": {}})
        cn = _col(r, "Counter_Name")
        d["c"][cn] = d["c"].get(cn, 0.0) + float(_col(r, "Counter_Value"))
    order = sorted(disp)
    last = disp[order[-1]]
    for c in a.cmd:
        print(f"command: {c}")
    print(f"dispatches: {len(order)}; calibration (last dispatch): {last['name'][:60]} grid {last['grid']} "
          + " ".join(f"{k}={v:.0f}" for k, v in last["c"].items()))
    durs = {}
    if a.trace_dir:
        for r in csv.DictReader(open(os.path.join(a.trace_dir, f"{a.trace_prefix}_kernel_trace.csv"))):
            key = (re.sub(r"\(.*", "", r["Kernel_Name"]), _grid(r))
            durs.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    agg = {}
    for did in order[:-1]:
        d = disp[did]
        g = agg.setdefault((d["name"], d["grid"]), {"n": 0, "c": {}})
        g["n"] += 1
        for k, v in d["c"].items():
            g["c"][k] = g["c"].get(k, 0.0) + v
    names = sorted({k for g in agg.values() for k in g["c"]})
    key0 = names[0] if names else ""
    items = sorted(agg.items(), key=lambda kv: -kv[1]["c"].get(key0, 0.0))
    print(f"{'n':>6} " + " ".join(f"{n + '/disp':>18}" for n in names) + f" {'avg_us':>9}  kernel  grid")
    for (name, grid), g in items[:a.top]:
        avg = {k: v / g["n"] for k, v in g["c"].items()}
        ds = durs.get((name, grid))
        us = sum(ds) / len(ds) if ds else float("nan")
        print(f"{g['n']:6d} " + " ".join(f"{avg.get(n, 0.0):18.1f}" for n in names) + f" {us:9.2f}  {name[:90]}  {grid}")


def main():
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "--pmc":
        return pmc_main(sys.argv[2:])
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
