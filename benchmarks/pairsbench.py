"""The paper's problem batched: 64 problems at 1023 x 1023 (white-noise coefficients, mesh
Reynolds number up to 10^3, the non-divergence operator, f = 1), the 8-channel network trained
by the paper's protocol, the stationary iteration to relative residual 1e-8 with the paper's
level count (coarsest grid 3 x 3), hipGraph-captured iterations; one state slot per problem or
packed pairs (two problems per 16-channel slot), in f32 or bf16 state, f64 u.

Prints one JSON line per configuration: setup + solve wall time of the batch (best of `reps`
after one untimed warm-up), solves/s, mean and largest iteration count.  The rocprofv3 kernel
trace of this program is the evidence behind the packed-pair figures of the benchmark's
`legs.paper_1023_batch64` entry.

    python -m benchmarks.pairsbench [--state bf16] [--pairs 1] [--reps 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(ROOT, "paper_2312_11093_amd", "trained", "t5_c8.npy")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--state", default="bf16", choices=["f32", "bf16"])
    ap.add_argument("--pairs", type=int, default=1, choices=[0, 1])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-8)
    args = ap.parse_args()
    import numpy as np
    import torch

    import datagen
    from paper_2312_11093_amd import Solver, autotune
    from paper_2312_11093_amd.weights import embed_channels

    autotune.load()
    w = embed_channels(np.load(WEIGHTS, allow_pickle=False))
    n, B = args.n, args.batch
    a, b, f = datagen.make_batch("paper_re1e3", n, B, seed=0)
    da, df = torch.from_numpy(a).cuda(), torch.from_numpy(f).cuda()
    S = Solver(w, state=args.state, u="f64", form="nondiv", levels=-1, use_graph=True, check_every=1,
               pack_pairs=bool(args.pairs), f32_split=2 if args.state == "f32" else True)
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
    times = []
    for rep in range(args.reps + 1):
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.setup(da, b)
        st, it, rr, ps = S.solve(df, u, args.tol, 400)
        torch.cuda.synchronize()
        if rep > 0:
            times.append(time.perf_counter() - t0)
    S.close()
    best = min(times)
    print(json.dumps({"workload": f"paper_re1e3: {B} problems at {n}x{n}, stationary, tol {args.tol:g}",
                      "state": args.state, "packed_pairs": bool(args.pairs),
                      "solves_per_s": round(B / best, 2) if (np.asarray(ps) == 0).all() else 0.0,
                      "ms_per_batch": round(1e3 * best, 2), "iters_mean": float(np.mean(it)),
                      "iters_max": int(np.max(it))}), flush=True)


if __name__ == "__main__":
    main()
