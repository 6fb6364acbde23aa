"""Summarise rocprofv3 CSV output per kernel and launch size.

    python3 -m paper_2408_03452_amd.tracesum trace DIR    # --kernel-trace --output-format csv
    python3 -m paper_2408_03452_amd.tracesum pmc DIR      # --pmc ... --output-format csv

``trace`` groups the dispatches of ``*kernel_trace.csv`` by (kernel, grid
size) and prints calls, total, mean and median duration. A group whose
durations form two clusters (a two-means split of the log durations) with
medians more than 2x apart, each holding at least 1 % of the calls, holds
launches of different workloads that happen to share a launch size; it is
split into the rows "fast" and "slow". ``pmc`` groups the
rows of ``*counter_collection.csv`` by (kernel, grid size, counter) and prints
the mean counter value per dispatch; dispatches whose value is below 1 % of
the group's largest (launches that returned at once, e.g. after convergence)
are counted separately and left out of the mean.
"""
from __future__ import annotations

import collections
import csv
import glob
import math
import os
import statistics
import sys


def _short(name: str) -> str:
    name = name.replace("mffv::(anonymous namespace)::", "").replace("mffv::", "")
    return name.split("(")[0] if "(" in name else name


def _grid(row: dict) -> str:
    """Launch size in work-items, from whichever grid columns the CSV has."""
    if row.get("Grid_Size"):
        return row["Grid_Size"]
    dims = [row.get(f"Grid_Size_{a}") for a in "XYZ"]
    if any(dims):
        n = 1
        for d in dims:
            n *= int(d or 1)
        return str(n)
    return "?"


def _files(d: str, suffix: str) -> list:
    return sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))


def _split(v: list) -> list:
    """[(label, durations)]: one cluster, or two when a two-means split of the
    log durations gives clusters whose medians differ by more than 2x, each
    with at least 1 % of the calls."""
    s = sorted(v)
    n = len(s)
    lo = max(1, n // 100)
    if n < 2 * lo or s[0] <= 0:
        return [("", v)]
    x = [math.log(d) for d in s]
    pre, pre2 = [0.0], [0.0]
    for t in x:
        pre.append(pre[-1] + t)
        pre2.append(pre2[-1] + t * t)

    def sse(a, b):  # sum of squared deviations of x[a:b]
        m = b - a
        sm = pre[b] - pre[a]
        return (pre2[b] - pre2[a]) - sm * sm / m

    best, at = None, None
    for i in range(lo, n - lo + 1):
        c = sse(0, i) + sse(i, n)
        if best is None or c < best:
            best, at = c, i
    if at is None or statistics.median(s[at:]) <= 2.0 * statistics.median(s[:at]):
        return [("", v)]
    return [(" (fast)", s[:at]), (" (slow)", s[at:])]


def trace(d: str, top: int = 30) -> None:
    raw = collections.defaultdict(list)
    for f in _files(d, "kernel_trace.csv"):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                dur = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3
                key = (_short(row["Kernel_Name"]), _grid(row))
                raw[key].append(dur)
    groups = {}
    for (name, grid), v in raw.items():
        for label, part in _split(v):
            groups[(name + label, grid)] = part
    tot_all = sum(sum(v) for v in groups.values())
    print("| kernel | grid (work-items) | calls | total ms | mean us | median us | % of GPU time |")
    print("|---|---:|---:|---:|---:|---:|---:|")
    for (name, grid), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
        print(f"| `{name}` | {grid} | {len(v)} | {sum(v) / 1e3:.2f} | {statistics.fmean(v):.2f} | "
              f"{statistics.median(v):.2f} | {100 * sum(v) / tot_all:.2f} |")


def pmc(d: str, top: int = 30) -> None:
    groups = collections.defaultdict(list)
    for f in _files(d, "counter_collection.csv"):
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                key = (_short(row["Kernel_Name"]), _grid(row), row["Counter_Name"])
                groups[key].append(float(row["Counter_Value"]))
    print("| kernel | grid (work-items) | counter | dispatches | mean per dispatch | skipped (< 1 % of max) |")
    print("|---|---:|---|---:|---:|---:|")
    for (name, grid, ctr), v in sorted(groups.items(), key=lambda kv: -max(kv[1]))[:top]:
        hi = max(v)
        keep = [x for x in v if x >= 0.01 * hi] or v
        print(f"| `{name}` | {grid} | {ctr} | {len(keep)} | {statistics.fmean(keep):.1f} | {len(v) - len(keep)} |")


if __name__ == "__main__":
    if len(sys.argv) != 3 or sys.argv[1] not in ("trace", "pmc"):
        print(__doc__)
        sys.exit(2)
    (trace if sys.argv[1] == "trace" else pmc)(sys.argv[2])
