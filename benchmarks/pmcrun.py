"""Short workload for hardware-counter runs (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE).

Runs, in one process on one GPU:
  1. a plain streaming kernel over COPY_MIB MiB (torch: dst = 2 * src), whose compulsory HBM
     traffic is known (COPY_MIB MiB read + COPY_MIB MiB written): it calibrates what the
     counters read per byte;
  2. `iters` stationary iterations (residual + V-cycle + update) of the benchmark's batch:
     64 problems at 1023 x 1023, random 16 x 16 blocks, f32 state, f64 u, hand-set weights, the
     benchmark's autotuned tile table.

    rocprofv3 --pmc FETCH_SIZE -d <dir> -o run -f csv -- python3 -m benchmarks.pmcrun
    rocprofv3 --pmc WRITE_SIZE -d <dir> -o run -f csv -- python3 -m benchmarks.pmcrun
    python -m benchmarks.profsum --pmc <dir>/run_counter_collection.csv
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_MIB = 1024


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--iters", type=int, default=2)
    args = ap.parse_args()
    import torch

    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd import autotune
    from paper_2312_11093_amd.handbuilt import vcycle_weights

    autotune.load()                                   # the benchmark's tile table

    src = torch.ones(COPY_MIB * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    print(f"stream: {COPY_MIB} MiB read + {COPY_MIB} MiB written", flush=True)
    n, B = args.n, args.batch
    a, b, f = datagen.make_batch("blocks1023", n, B, seed=0)
    S = Solver(vcycle_weights(), state="f32", u="f64", f32_split=2)   # the benchmark's setting
    S.setup(torch.from_numpy(a).cuda(), b)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    S.forward(torch.from_numpy(f).cuda(), u, args.iters)
    torch.cuda.synchronize()
    print(f"{args.iters} stationary iterations of {B} x {n}^2 done", flush=True)
    S.close()


if __name__ == "__main__":
    main()
