"""The paper's own test problems on this library (Sec. 4.1 problem and iterative-method settings):
the non-divergence operator, white-noise coefficients with mesh Reynolds number in [1, Re],
v = (sin 0.5, cos 0.5), right-hand side 1, one problem per solve, the stationary iteration to
relative residual 1e-8.  For every grid size it reports, averaged over `draws` coefficient
draws, the iteration count, setup time and solve time of

  * GMG: the geometric multigrid baseline with the paper's settings (levels log2(n+1) - 3,
    three sweeps of weight 0.67, exact coarsest solve);
  * network: the MGCNN solve network, f32 state, f64 u; by default with the hand-set
    coefficient-aware V(1,1) weights as the preconditioner of FGMRES(30) (as a stationary
    iteration these weights diverge on white-noise coefficients); with --weights FILE (a .npy
    flat vector of a C-channel network, C <= 16, read with allow_pickle=False) a trained network,
    by default in the stationary iteration of Sec. 4.1 (--method stationary|fgmres);

next to the GMG iteration counts the paper prints (Sec. 4.2, double precision table).
--data mldata takes the coefficients from the multi-level generator of Alg. 4 instead of white
noise (Sec. 4.3, Re = 1000); --net-levels sets the network's level count (0: log2(n+1), coarsest
grid 1 x 1; -1: the count of Sec. 4.1, coarsest grid 3 x 3).

    python -m benchmarks.paper_table [--re 1000] [--data white|mldata] [--net-levels 0]
                                     [--sizes 31,63,...] [--draws 3] [--weights W.npy]
                                     [--method stationary|fgmres] [--no-gmg]
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

# GMG iterations printed in the paper for Re = 1000 (Sec. 4.2, double precision, tolerance 1e-8)
PAPER_GMG = {31: 16.7, 63: 19.2, 127: 21, 255: 25.9, 511: 33.7, 1023: 45, 2047: 61, 4095: 84}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--re", type=float, default=1000.0, choices=[10.0, 1000.0, 1e5])
    ap.add_argument("--sizes", default="31,63,127,255,511,1023,2047,4095")
    ap.add_argument("--draws", type=int, default=3)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=2000)
    ap.add_argument("--data", default="white", choices=["white", "mldata"])
    ap.add_argument("--net-levels", type=int, default=0)
    ap.add_argument("--weights", default=None)
    ap.add_argument("--method", default=None, choices=["stationary", "fgmres"])
    ap.add_argument("--no-gmg", action="store_true")
    args = ap.parse_args()
    import numpy as np
    import torch

    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd.handbuilt import vcycle_weights
    from paper_2312_11093_amd.weights import embed_channels

    if args.weights:
        net_w = embed_channels(np.load(args.weights, allow_pickle=False))
        method = args.method or "stationary"
    else:
        net_w = vcycle_weights()
        method = args.method or "fgmres"

    if args.data == "mldata":
        if args.re != 1000.0:
            ap.error("--data mldata is posed with Re = 1000")
        wl = "paper_mldata"
    else:
        wl = {10.0: "paper_re10", 1000.0: "paper_re1e3", 1e5: "paper_re1e5"}[args.re]
    sizes = [int(x) for x in args.sizes.split(",")]
    rows = []
    for n in sizes:
        row = {"n": n, "paper_gmg_iters": PAPER_GMG.get(n) if wl == "paper_re1e3" else None}
        for name in (("network",) if args.no_gmg else ("gmg", "network")):
            if name == "gmg":
                S = Solver(None, precond="gmg", u="f64", form="nondiv", use_graph=True)
            else:
                S = Solver(net_w, state="f32", u="f64", form="nondiv", method=method,
                           restart=30, levels=args.net_levels)
            its, tset, tsol, ok = [], [], [], True
            for d in range(args.draws + 1):          # draw 0 warms up
                p = datagen.make_problem(wl, n, d, 0)
                a = torch.from_numpy(p.a).cuda().view(1, n, n)
                f = torch.from_numpy(p.f).cuda().view(1, n, n)
                u = torch.zeros((1, n, n), dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                S.setup(a, p.b.reshape(1, 2))
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                st, it, rr, ps = S.solve(f, u, args.tol, args.maxit)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                if d == 0:
                    continue
                its.append(int(it[0]))
                ok &= int(ps[0]) == 0
                tset.append(1e3 * (t1 - t0))
                tsol.append(1e3 * (t2 - t1))
            S.close()
            row[name] = {"iters": float(np.mean(its)), "converged": ok,
                         "setup_ms": round(float(np.mean(tset)), 3),
                         "solve_ms": round(float(np.mean(tsol)), 3)}
        rows.append(row)
        print(json.dumps(row), flush=True)
    if args.no_gmg:
        return
    print(f"{'n':>6} {'paper GMG it':>12} {'GMG it':>7} {'GMG setup':>10} {'GMG solve':>10} "
          f"{'net it':>7} {'net setup':>10} {'net solve':>10}  (ms; network: {method})")
    for r in rows:
        g, w = r["gmg"], r["network"]
        pg = f"{r['paper_gmg_iters']:.1f}" if r["paper_gmg_iters"] is not None else "-"
        print(f"{r['n']:>6} {pg:>12} {g['iters']:>7.1f} {g['setup_ms']:>10.2f} {g['solve_ms']:>10.2f} "
              f"{w['iters']:>7.1f} {w['setup_ms']:>10.2f} {w['solve_ms']:>10.2f}"
              + ("" if g["converged"] and w["converged"] else "  (not all converged)"))


if __name__ == "__main__":
    main()
