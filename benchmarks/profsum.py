"""Summarise a rocprofv3 kernel trace (CSV) per kernel and grid size.

    python -m benchmarks.profsum <run_kernel_trace.csv> [top]
    python -m benchmarks.profsum --pmc <run_counter_collection.csv> [top]
    python -m benchmarks.profsum --sq <run_counter_collection.csv> [<run_counter_collection.csv> ...]

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


SQ_COUNTERS = ("SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_BUSY_CU_CYCLES", "SQ_VALU_MFMA_BUSY_CYCLES",
               "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_ANY", "SQ_LDS_BANK_CONFLICT",
               "SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_LDS", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR",
               "SQ_WAIT_ANY", "SQ_ACTIVE_INST_ANY")


def summarize_sq(paths, top: int = 12, cus: int = 256) -> str:
    """Derived per-dispatch ratios of the SQ counters (means over the dispatches of each kernel and
    grid size, counters from several --pmc runs merged):
      mfma_busy  = SQ_VALU_MFMA_BUSY_CYCLES / (4 SIMDs x SQ_BUSY_CU_CYCLES)
      valu_busy  = SQ_ACTIVE_INST_VALU / (4 x SQ_BUSY_CU_CYCLES)
      lds_conf   = SQ_LDS_BANK_CONFLICT / SQ_BUSY_CU_CYCLES (bank-conflict cycles per busy CU cycle)
      waves/CU   = 4 x SQ_WAVE_CYCLES / SQ_BUSY_CU_CYCLES (wave cycles are counted per 4 cycles)
      wait       = SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES (share of wave time waiting on issued memory)
    and instruction counts per wave."""
    agg = collections.defaultdict(lambda: [0, 0.0])
    for path in paths:
        for r in csv.DictReader(open(path)):
            name = r.get("Kernel_Name", "?").split("(")[0]
            grid = int(float(r.get("Grid_Size", r.get("Grid_Size_X", "0"))))
            agg[(name, grid, r.get("Counter_Name", "?"))][0] += 1
            agg[(name, grid, r.get("Counter_Name", "?"))][1] += float(r.get("Counter_Value", "nan"))
    mean = {k: v[1] / v[0] for k, v in agg.items()}
    kern = {}
    for (name, grid, ctr), v in mean.items():
        kern.setdefault((name, grid), {})[ctr] = v
    rows = sorted(kern.items(), key=lambda kv: -kv[1].get("SQ_BUSY_CU_CYCLES", 0.0))[:top]
    out = [f"{'kernel':48s} {'grid':>9s} {'busy_us':>8s} {'mfma':>5s} {'valu':>5s} {'ldsconf':>7s} "
           f"{'waves/CU':>8s} {'wait':>5s} {'valu/w':>7s} {'mfma/w':>7s} {'lds/w':>6s} {'vmrd/w':>6s}"]
    for (name, grid), c in rows:
        busy = c.get("SQ_BUSY_CU_CYCLES", float("nan"))
        waves = c.get("SQ_WAVES", float("nan"))
        f = lambda k: c.get(k, float("nan"))
        out.append(f"{name[:48]:48s} {grid:9d} {busy / cus / 2400.0:8.1f} "
                   f"{f('SQ_VALU_MFMA_BUSY_CYCLES') / (4 * busy):5.2f} {f('SQ_ACTIVE_INST_VALU') / (4 * busy):5.2f} "
                   f"{f('SQ_LDS_BANK_CONFLICT') / busy:7.3f} {4 * f('SQ_WAVE_CYCLES') / busy:8.1f} "
                   f"{f('SQ_WAIT_INST_ANY') / f('SQ_WAVE_CYCLES'):5.2f} {f('SQ_INSTS_VALU') / waves:7.1f} "
                   f"{f('SQ_INSTS_MFMA') / waves:7.1f} {f('SQ_INSTS_LDS') / waves:6.1f} {f('SQ_INSTS_VMEM_RD') / waves:6.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--sq":
        print(summarize_sq(sys.argv[2:]))
        sys.exit(0)
    if len(sys.argv) > 1 and sys.argv[1] == "--pmc":
        print(summarize_pmc(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25))
        sys.exit(0)
    print(summarize(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 25))
