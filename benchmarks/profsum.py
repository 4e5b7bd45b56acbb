"""Summarise a rocprofv3 kernel trace (CSV) per kernel and grid size.

    python -m benchmarks.profsum <run_kernel_trace.csv> [top]
    python -m benchmarks.profsum --pmc <run_counter_collection.csv> [top]

Prints launches, average and total duration per kernel, then per (kernel, grid size); the
grid size separates the levels of the multigrid hierarchy and the number of live problems.
"""
from __future__ import annotations

import collections
import csv
import sys


def summarize(path: str, top: int = 25) -> str:
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(lambda: [0, 0.0])
    byname = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        name = r["Kernel_Name"].split("(")[0]
        us = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        key = (name, int(r["Grid_Size_X"]))
        agg[key][0] += 1
        agg[key][1] += us
        byname[name][0] += 1
        byname[name][1] += us
    total = sum(v[1] for v in agg.values())
    out = ["per kernel (all grid sizes):",
           f"{'kernel':60s} {'launches':>8s} {'avg_us':>10s} {'total_ms':>10s} {'share':>6s}"]
    for name, (cnt, us) in sorted(byname.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"{name[:60]:60s} {cnt:8d} {us / cnt:10.1f} {us / 1e3:10.2f} {us / total:6.3f}")
    out += ["", "per kernel and grid size (the grid separates levels and batch sizes):",
            f"{'kernel':60s} {'grid_x':>10s} {'launches':>8s} {'avg_us':>10s} {'total_ms':>10s} {'share':>6s}"]
    for (name, grid), (cnt, us) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"{name[:60]:60s} {grid:10d} {cnt:8d} {us / cnt:10.1f} {us / 1e3:10.2f} {us / total:6.3f}")
    out.append(f"total kernel time {total / 1e3:.2f} ms over {sum(v[0] for v in agg.values())} launches")
    return "\n".join(out)


def summarize_pmc(path: str, top: int = 25) -> str:
    """Mean counter value per dispatch for every (kernel, grid size, counter)."""
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        name = r.get("Kernel_Name", "?").split("(")[0]
        grid = r.get("Grid_Size", r.get("Grid_Size_X", "0"))
        key = (name, int(float(grid)), r.get("Counter_Name", "?"))
        agg[key][0] += 1
        agg[key][1] += float(r.get("Counter_Value", "nan"))
    out = [f"{'kernel':60s} {'grid':>10s} {'counter':>12s} {'dispatches':>10s} {'mean per dispatch':>18s}"]
    for (name, grid, ctr), (cnt, tot) in sorted(agg.items(), key=lambda kv: -kv[1][1] / kv[1][0])[:top]:
        out.append(f"{name[:60]:60s} {grid:10d} {ctr:>12s} {cnt:10d} {tot / cnt:18.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--pmc":
        print(summarize_pmc(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25))
        sys.exit(0)
    print(summarize(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 25))
