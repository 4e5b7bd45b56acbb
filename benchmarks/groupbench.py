"""Uneven-size batch on one GPU: `count` problems whose sides are drawn uniformly from
63, 127, ..., 2047 (the training-mixture coefficients: lognormal GRF, 8 x 8 checkerboard,
inclusions; random b; f ~ N(0, 1)), solved together through mgcnn_group_* (one batched
problem set per size, the sizes on concurrent streams) to relative residual `tol`.

Prints one JSON line: wall time of setup + solve for the whole set (after one untimed
warm-up of the same call), solves/s, per-size problem counts and mean iterations, the 50th
and 99th percentiles of the iteration counts, and the largest final relative residual (the
library's f64 residual of every returned solution).

    python -m benchmarks.groupbench [--count 256] [--precond network|gmg]
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=6000)
    ap.add_argument("--restart", type=int, default=63)
    ap.add_argument("--deflate", type=int, default=8)
    ap.add_argument("--precond", default="network", choices=["network", "gmg"])
    args = ap.parse_args()
    import numpy as np
    import torch

    import datagen
    from paper_2312_11093_amd import GroupSolver
    from paper_2312_11093_amd.handbuilt import vcycle_weights

    sizes = datagen.var_sizes(args.count, args.seed)
    probs = [datagen.make_problem("mixture_var", n, i, args.seed) for i, n in enumerate(sizes)]
    a = [torch.from_numpy(p.a).cuda() for p in probs]
    f = [torch.from_numpy(p.f).cuda() for p in probs]
    b = np.stack([p.b for p in probs])
    u = [torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda") for p in probs]
    w = vcycle_weights() if args.precond == "network" else None
    G = GroupSolver(w, state="f32", u="f64", method="fgmres", restart=args.restart, gs_passes=1,
                    deflate=args.deflate, precond=args.precond)

    def run():
        for x in u:
            x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        G.setup(a, b)
        res = G.solve(f, u, args.tol, args.maxit)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, res

    run()
    print("[groupbench] warm-up done", file=sys.stderr, flush=True)
    t, (st, it, rr, stat) = run()
    G.close()
    it = np.asarray(it)
    per_size = {}
    for n in sorted(set(sizes)):
        sel = [i for i, m in enumerate(sizes) if m == n]
        per_size[str(n)] = {"problems": len(sel), "mean_iters": round(float(it[sel].mean()), 1),
                            "max_iters": int(it[sel].max())}
    print(json.dumps({
        "what": f"{args.count} problems, sides uniform over {sorted(set(datagen.VAR_SIZES))}, "
                f"mixture coefficients, FGMRES({args.restart}) deflate {args.deflate}, "
                f"{args.precond} preconditioner, tol {args.tol:g}, f32 state, f64 u",
        "seconds": round(t, 3), "solves_per_s": round(args.count / t, 3),
        "converged": bool((np.asarray(stat) == 0).all()),
        "iters_p50": float(np.percentile(it, 50)), "iters_p99": float(np.percentile(it, 99)),
        "iters_max": int(it.max()), "per_size": per_size,
        "relres_max": float(np.max(rr)),
        "fine_nodes": int(sum(n * n for n in sizes)),
    }))


if __name__ == "__main__":
    main()
