"""Symmetric problems on one GPU: a batch of n x n block-coefficient problems with b = 0 (A
symmetric positive definite), solved to relative residual `tol` with the GMG V-cycle as
preconditioner, once by preconditioned conjugate gradients and once by FGMRES(63) with
deflated restarts (k = 8), the method the benchmark uses for nonsymmetric problems.

Prints one JSON line per method: wall time of the solve of the whole batch (the second of two
identical solves), solves/s, mean and largest step counts, and the largest relative residual
(the library's f64 residual of each returned solution).

    python -m benchmarks.pcgbench [--n 1023] [--batch 64] [--tol 1e-8]
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
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=4000)
    args = ap.parse_args()
    import numpy as np
    import torch

    import datagen
    from paper_2312_11093_amd import Solver

    n, B = args.n, args.batch
    a, b, f = datagen.make_batch("blocks1023", n, B, seed=0)
    b = np.zeros_like(b)
    da = torch.from_numpy(a).cuda()
    df = torch.from_numpy(f).cuda()
    print("[pcgbench] inputs resident", file=sys.stderr, flush=True)
    for name, kw in (("pcg", dict(method="pcg")),
                     ("fgmres63_deflate8", dict(method="fgmres", restart=63, gs_passes=1, deflate=8))):
        S = Solver(None, precond="gmg", state="f32", u="f64", **kw)
        S.setup(da, b)
        for rep in range(2):
            u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, it, rr, ps = S.solve(df, u, args.tol, args.maxit)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
        S.close()
        print(json.dumps({"method": name, "preconditioner": "gmg", "n": n, "batch": B, "tol": args.tol,
                          "converged": bool((np.asarray(ps) == 0).all()), "seconds": round(t, 3),
                          "solves_per_s": round(B / t, 2), "iters_mean": float(np.mean(it)),
                          "iters_max": int(np.max(it)), "relres_max": float(np.max(rr))}), flush=True)


if __name__ == "__main__":
    main()
