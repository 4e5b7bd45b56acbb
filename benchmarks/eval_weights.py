"""Iteration counts and solve times of a weight set on a seeded workload, per outer method.

For each grid size, `batch` problems of the workload are solved to `tol` (f32 state, f64 u)
with the stationary iteration of Eq. (1) and/or FGMRES(restart) with deflated restarts, the
network as preconditioner.  Prints one JSON line per (size, method): status counts, mean / max
iterations, the asymptotic contraction per iteration estimated from the iteration counts,
setup and solve times.

    python -m benchmarks.eval_weights --weights W.npy [--workload blocks1023] [--sizes 255,1023]
                                      [--batch 8] [--methods stationary,fgmres] [--levels 0]
                                      [--form div] [--tol 1e-8] [--maxit 2000]

W.npy is a flat float32 vector of a C-channel network (C <= 16; read with allow_pickle=False),
or "handbuilt" for the hand-set V(1,1) cycle.
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
    ap.add_argument("--weights", required=True)
    ap.add_argument("--workload", default="blocks1023")
    ap.add_argument("--sizes", default="255,1023")
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--methods", default="stationary,fgmres")
    ap.add_argument("--levels", type=int, default=0)
    ap.add_argument("--form", default=None, choices=[None, "div", "nondiv"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=2000)
    ap.add_argument("--restart", type=int, default=63)
    ap.add_argument("--deflate", type=int, default=8)
    ap.add_argument("--state", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    import numpy as np
    import torch

    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd.handbuilt import vcycle_weights
    from paper_2312_11093_amd.weights import embed_channels

    if args.weights == "handbuilt":
        w = vcycle_weights()
    else:
        w = embed_channels(np.load(args.weights, allow_pickle=False))
    form = args.form or datagen.WORKLOADS[args.workload].form
    for n in [int(x) for x in args.sizes.split(",")]:
        a, b, f = datagen.make_batch(args.workload, n, args.batch, seed=args.seed)
        ad, fd = torch.from_numpy(a).cuda(), torch.from_numpy(f).cuda()
        for method in args.methods.split(","):
            kw = dict(method=method, restart=args.restart, gs_passes=1,
                      deflate=args.deflate if method == "fgmres" else 0)
            S = Solver(w, state=args.state, u="f64", form=form, levels=args.levels,
                       f32_split=2 if args.state == "f32" else True, **kw)
            u = torch.zeros((args.batch, n, n), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.setup(ad, b)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, it, rr, ps = S.solve(fd, u, args.tol, args.maxit)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            S.close()
            ok = ps == 0
            its = it[ok]
            rate = float(np.exp(np.log(args.tol) / its.mean())) if ok.any() else None
            print(json.dumps({
                "n": n, "batch": args.batch, "workload": args.workload, "form": form,
                "levels": args.levels, "method": method, "state": args.state,
                "converged": int(ok.sum()), "diverged": int((ps == -6).sum()),
                "not_converged": int((ps == 1).sum()),
                "iters_mean": float(its.mean()) if ok.any() else None,
                "iters_max": int(its.max()) if ok.any() else None,
                "rate_per_iter": rate, "relres_max": float(np.max(rr)),
                "setup_ms": round(1e3 * (t1 - t0), 2), "solve_ms": round(1e3 * (t2 - t1), 1),
                "solves_per_s": round(args.batch / (t2 - t0), 3)}), flush=True)


if __name__ == "__main__":
    main()
