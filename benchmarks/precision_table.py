"""Precision of the solve on one large grid: a single n x n problem (lognormal Gaussian random
field coefficients, length 0.05, variance 2, b = (1, 1), f ~ U(-1, 1)) solved to relative
residual `tol` by FGMRES with the network preconditioner in three precisions:

  * f32 state, f64 u and residual (the library's default);
  * plain FP32: f32 state, f32 u and f32 residual arithmetic;
  * bf16 state (bf16 matrix products with f32 accumulation), f64 u and residual.

Prints one JSON line per variant: status, iterations, the relative residual the solver reports
and the one recomputed in f64 by the library for the returned u (the floor a variant stalls at
when it cannot reach `tol`), the solve time, and the relative difference of its u from the
f32-state / f64-u solution.

    python -m benchmarks.precision_table [--n 4095] [--tol 1e-10] [--maxit 400]
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
    ap.add_argument("--n", type=int, default=4095)
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--maxit", type=int, default=400)
    ap.add_argument("--restart", type=int, default=30)
    args = ap.parse_args()
    import torch

    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd import mgcnn as M
    from paper_2312_11093_amd.handbuilt import vcycle_weights

    n = args.n
    p = datagen.make_problem("grf4095", n, 0, 0)
    a = torch.from_numpy(p.a).cuda().view(1, n, n)
    f = torch.from_numpy(p.f).cuda().view(1, n, n)
    ref = None
    check = Solver(vcycle_weights(), state="f32", u="f64")      # f64 residual of any returned u
    check.setup(a, p.b.reshape(1, 2))
    for name, state, udt in (("f32 state, f64 u", "f32", "f64"), ("plain FP32", "f32", "f32"),
                             ("bf16 state, f64 u", "bf16", "f64")):
        S = Solver(vcycle_weights(), state=state, u=udt, method="fgmres", restart=args.restart)
        u = torch.zeros((1, n, n), dtype=S.u_dtype, device="cuda")
        S.setup(a, p.b.reshape(1, 2))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            st, it, rr, ps = S.solve(f, u, args.tol, args.maxit)
            status, iters, reported = int(ps[0]), int(it[0]), float(rr[0])
        except M.MGCNNError as e:
            status, iters, reported = e.status, -1, float("nan")
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        S.close()
        ud = u.double()
        true_rr = float(check.residual_norms(f, ud)[0])
        if ref is None:
            ref = ud.clone()
        diff = float(torch.linalg.vector_norm(ud - ref) / torch.linalg.vector_norm(ref))
        print(json.dumps({"variant": name, "n": n, "tol": args.tol, "status": status,
                          "iterations": iters, "relres_reported": reported, "relres_f64": true_rr,
                          "seconds": round(t, 3), "u_rel_diff_vs_f32_f64": diff}), flush=True)
    check.close()


if __name__ == "__main__":
    main()
