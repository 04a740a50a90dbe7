"""Summarise rocprofv3 CSV output (kernel stats + kernel trace) as short text.

    python -m paper_2210_08494_amd.profsum <dir-with-csv> <prefix> [--kernel SUBSTR] [--grid X,Y]
        [--top N] [--cmd "the command that produced the CSV"]
    python -m paper_2210_08494_amd.profsum --pmc --fetch F.csv --write W.csv [--trace T.csv] [--cmd ...]
    python -m paper_2210_08494_amd.profsum --pmc --fetch F.csv --write W.csv --mops M.csv --trace T.csv

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


def _counters(path):
    """{dispatch id: (kernel name, total grid, {counter: value})} of a counter-collection CSV."""
    disp = {}
    for r in csv.DictReader(open(path)):
        did = int(_col(r, "Dispatch_Id", "Correlation_Id"))
        d = disp.setdefault(did, (re.sub(r"\(.*", "", _col(r, "Kernel_Name")), r.get("Grid_Size", ""), {}))
        cn = _col(r, "Counter_Name")
        d[2][cn] = d[2].get(cn, 0.0) + float(_col(r, "Counter_Value"))
    return disp


def pmc_main(argv):
    """HBM bytes per dispatch from a FETCH_SIZE run and a WRITE_SIZE run of the same
    command, each scaled by what its counter reads for the command's last dispatch
    (a plain device copy of --calib-mib MiB), with durations from a kernel trace of
    the same command (the k-th dispatch of each kernel and grid matched with its
    k-th in the trace)."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True, help="counter_collection.csv of the FETCH_SIZE run")
    ap.add_argument("--write", required=True, help="counter_collection.csv of the WRITE_SIZE run")
    ap.add_argument("--trace", default="", help="kernel_trace.csv of the same command")
    ap.add_argument("--calib-mib", type=float, default=256.0)
    ap.add_argument("--cmd", action="append", default=[])
    ap.add_argument("--top", type=int, default=24)
    ap.add_argument("--mops", default="",
                    help="counter_collection.csv of a run with SQ_INSTS_VALU_MFMA_MOPS_{BF16,F64,F32} "
                         "(same command as --trace): executed MFMA flops per dispatch and rate")
    a = ap.parse_args(argv)
    if a.mops:
        return mops_table(a)
    fe, wr = _counters(a.fetch), _counters(a.write)
    last = max(fe)
    kib = a.calib_mib * 1024.0
    sf = kib / fe[last][2]["FETCH_SIZE"]
    sw = kib / wr[max(wr)][2]["WRITE_SIZE"]
    # the k-th dispatch of a (kernel, grid) in the counter run is matched with the
    # k-th dispatch of the same (kernel, grid) in the trace: robust to commands whose
    # streams interleave their launches differently from run to run
    dur = {}
    if a.trace:
        seen = {}
        for r in sorted(csv.DictReader(open(a.trace)), key=lambda r: int(r["Dispatch_Id"])):
            key = (re.sub(r"\(.*", "", r["Kernel_Name"]),
                   str(int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])))
            k = seen.get(key, 0)
            seen[key] = k + 1
            dur[key + (k,)] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    for c in a.cmd:
        print(f"command: {c}")
    print(f"dispatches: {len(fe)}; reference copy of {a.calib_mib:.0f} MiB (last dispatch): FETCH_SIZE "
          f"{fe[last][2]['FETCH_SIZE']:.0f} KiB, WRITE_SIZE {wr[max(wr)][2]['WRITE_SIZE']:.0f} KiB -> "
          f"scale fetch x{sf:.3f}, write x{sw:.3f}")
    agg = {}
    for did, (name, grid, c) in sorted(fe.items()):
        if did == last or did not in wr:
            continue
        g = agg.setdefault((name, grid), {"n": 0, "f": 0.0, "w": 0.0, "t": 0.0, "nt": 0})
        key = (name, grid, g["n"])
        g["n"] += 1
        g["f"] += c.get("FETCH_SIZE", 0.0) * 1024.0 * sf
        g["w"] += wr[did][2].get("WRITE_SIZE", 0.0) * 1024.0 * sw
        if key in dur:
            g["t"] += dur[key]
            g["nt"] += 1
    items = sorted(agg.items(), key=lambda kv: -(kv[1]["f"] + kv[1]["w"]))
    print(f"{'n':>6} {'fetch_MB/disp':>14} {'write_MB/disp':>14} {'avg_us':>9} {'GB/s':>8}  kernel  (grid threads)")
    for (name, grid), g in items[:a.top]:
        f, w = g["f"] / g["n"], g["w"] / g["n"]
        t = g["t"] / g["nt"] if g["nt"] else float("nan")
        gbs = (f + w) / t / 1e9 if g["nt"] else float("nan")
        print(f"{g['n']:6d} {f / 1e6:14.2f} {w / 1e6:14.2f} {t * 1e6:9.1f} {gbs:8.0f}  {name[:95]}  ({grid})")


def _trace_by_ordinal(path):
    """{(kernel, total grid, k): duration s} of a kernel trace, k-th dispatch of each kernel and grid."""
    dur, seen = {}, {}
    for r in sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"])):
        key = (re.sub(r"\(.*", "", r["Kernel_Name"]),
               str(int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])))
        k = seen.get(key, 0)
        seen[key] = k + 1
        dur[key + (k,)] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
    return dur


PEAK_TF = {"BF16": 2500.0, "F64": 78.6, "F32": 157.3}


def mops_table(a):
    """Executed MFMA flops per (kernel, grid): 512 flops per MOPS count (the counters
    count 512-flop units), over the traced duration of the same dispatches, and the
    fraction of the dense peak of the dtype that dominates the kernel's count."""
    mo = _counters(a.mops)
    dur = _trace_by_ordinal(a.trace) if a.trace else {}
    for c in a.cmd:
        print(f"command: {c}")
    agg = {}
    for did, (name, grid, c) in sorted(mo.items()):
        g = agg.setdefault((name, grid), {"n": 0, "t": 0.0, "nt": 0, "BF16": 0.0, "F64": 0.0, "F32": 0.0})
        key = (name, grid, g["n"])
        g["n"] += 1
        for dt in ("BF16", "F64", "F32"):
            g[dt] += 512.0 * c.get(f"SQ_INSTS_VALU_MFMA_MOPS_{dt}", 0.0)
        if key in dur:
            g["t"] += dur[key]
            g["nt"] += 1
    items = sorted(agg.items(), key=lambda kv: -kv[1]["t"])
    print(f"{'n':>6} {'avg_us':>9} {'GFLOP/disp':>11} {'TFLOP/s':>8} {'dtype':>5} {'of_peak':>7}  kernel  (grid threads)")
    for (name, grid), g in items[:a.top]:
        fl = {dt: g[dt] / g["n"] for dt in ("BF16", "F64", "F32")}
        dt = max(fl, key=fl.get)
        tot = sum(fl.values())
        if tot == 0 or not g["nt"]:
            continue
        t = g["t"] / g["nt"]
        tf = tot / t / 1e12
        print(f"{g['n']:6d} {t * 1e6:9.1f} {tot / 1e9:11.3f} {tf:8.1f} {dt:>5} {tf / PEAK_TF[dt]:7.1%}  {name[:90]}  ({grid})")


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
    ap.add_argument("--last", type=int, default=0,
                    help="also report the last N dispatches of the --kernel selections together")
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
    chosen = []
    for i, k in enumerate(a.kernel):
        grid = a.grid[i] if i < len(a.grid) else ""
        sel = [r for r in trace if k in r["Kernel_Name"]]
        if grid:
            gx, gy = grid.split(",")
            sel = [r for r in sel if r["Grid_Size_X"] == gx and r["Grid_Size_Y"] == gy]
        chosen += sel
        durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in sel]
        if durs:
            print(f"kernel '{k}' grid ({grid or 'any'}): {len(durs)} dispatches, avg {sum(durs) / len(durs):.2f} us, "
                  f"total {sum(durs) / 1e3:.3f} ms, min {min(durs):.2f} us, max {max(durs):.2f} us")
    if a.last and chosen:
        chosen.sort(key=lambda r: int(r["Dispatch_Id"]))
        durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in chosen[-a.last:]]
        print(f"last {len(durs)} dispatches of the selections above: avg {sum(durs) / len(durs):.2f} us, "
              f"total {sum(durs) / 1e3:.3f} ms")


if __name__ == "__main__":
    main()
