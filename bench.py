"""Benchmark: batched MGCNN solves to relative residual 1e-8 on one MI355X.

One step = the whole hot path over one batch: setup phase for every problem, then the
stationary iteration (residual, stopping test, V-cycle, update) until every problem of the
batch reaches ||f - A u|| / ||f|| <= 1e-8 (or maxit).  Inputs (coefficients, velocities,
right-hand sides) are synthetic, seeded, resident in HBM before the timed region.

Default workload: 64 problems at 1023 x 1023, 16 x 16 random block coefficients with
log10 a ~ U(-2, 2), b = |b|(cos t, sin t) with |b| ~ U(0, 10), f ~ N(0, 1); 16 channels,
10 levels; bf16 state on MFMA with f32 accumulation, f64 u / residual / norm.

Prints one JSON line (rank 0): metric, value (solves/s, whole batch), roofline of the
dominant kernel (HIP events around its launches in a profiled pass), the plain-FP32
unbatched form on the same GPU, and the FP64 oracle timed on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s to rel-residual 1e-8 (1023², batch 64) vs plain FP32; HBM GB/s"
HBM_PEAK_GBS = 8000.0
TRAINED = os.path.join(ROOT, "paper_2312_11093_amd", "weights", "mgcnn_c16.npy")


def load_weights(path):
    import datagen
    if path and os.path.exists(path):
        return np.load(path, allow_pickle=False).astype(np.float32), os.path.relpath(path, ROOT)
    return datagen.xavier_weights(16, 0), "xavier-seed0 (untrained)"


def cpu_baseline(weights, a, b, f, iters_per_solve, sample_iters=2):
    """Time the FP64 oracle on the host: setup + `sample_iters` V-cycle iterations of one
    problem; extrapolate one solve to the GPU's mean iteration count."""
    from oracle import solve as osv
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    S = osv.Solver(weights, a, b)
    t1 = time.perf_counter()
    u = np.zeros(f.shape)
    for _ in range(sample_iters):
        u = S.step(f, u)
    t2 = time.perf_counter()
    per_iter = (t2 - t1) / sample_iters
    solve_s = (t1 - t0) + per_iter * max(iters_per_solve, 1.0)
    return {
        "value": 1.0 / solve_s, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"one {f.shape[0]}x{f.shape[1]} problem: oracle setup ({t1 - t0:.2f} s) + "
                   f"{sample_iters} V-cycle iterations ({per_iter:.2f} s each), extrapolated to "
                   f"{iters_per_solve:.1f} iterations per solve"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--workload", default="blocks1023")
    ap.add_argument("--state", default="bf16", choices=["bf16", "f32"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=100)
    ap.add_argument("--check-every", type=int, default=4)
    ap.add_argument("--weights", default=TRAINED)
    ap.add_argument("--plain-sample", type=int, default=4, help="problems solved one by one in the plain-FP32 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd import mgcnn as M

    n, B = args.n, args.batch
    weights, wsrc = load_weights(args.weights)
    a, b, f = datagen.make_batch(args.workload, n, B, seed=0)
    da = torch.from_numpy(a).cuda()
    df = torch.from_numpy(f).cuda()
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")

    S = Solver(weights, state=args.state, u="f64", check_every=args.check_every,
               use_graph=not args.no_graph)

    def step():
        u.zero_()
        S.setup(da, b)
        return S.solve(df, u, args.tol, args.maxit)

    for _ in range(args.warmup):
        res = step()
    torch.cuda.synchronize()
    times = []
    its = []
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, rr, ps = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        its.append(it.copy())
    ms = 1000.0 * float(np.mean(times))
    converged = bool((ps == 0).all())
    mean_iters = float(np.mean(its[-1]))
    value = B / (ms / 1000.0) if converged else 0.0

    # time of one batched V-cycle iteration (residual + network + update), weight independent
    KI = 10
    u.zero_()
    S.forward(df, u, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.forward(df, u, KI)
    torch.cuda.synchronize()
    iter_ms = 1000.0 * (time.perf_counter() - t0) / KI

    # independent check of the returned solutions (sampled problems, host FP64 residual)
    from oracle import solve as osv
    u.zero_()
    step()
    check = [osv.relres(a[p], b[p], f[p], u[p].cpu().numpy()) for p in (0, B - 1)]

    # profiled pass: HIP events around every launch of one solve
    u.zero_()
    S.setup(da, b)
    S.profile_begin()
    S.solve(df, u, args.tol, args.maxit)
    stats = S.profile_end()
    by_kind = {}
    for s_ in stats:
        by_kind.setdefault(s_["kind"], 0.0)
        by_kind[s_["kind"]] += s_["ms_total"]
    dom = max(by_kind, key=by_kind.get)
    fine = [s_ for s_ in stats if s_["kind"] == dom and s_["level"] == 0][0]
    avg_ms = fine["ms_total"] / fine["launches"]
    achieved = fine["bytes_per_launch"] / (avg_ms / 1000.0) / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "kernel": f"{dom} (finest level, {fine['launches']} launches, {avg_ms:.3f} ms avg)",
            "bytes_per_launch": fine["bytes_per_launch"]}
    kernel_share = {k: round(v / sum(by_kind.values()), 4) for k, v in sorted(by_kind.items(), key=lambda kv: -kv[1])}
    S.close()

    # plain FP32 unbatched form on the same GPU: f32 state, one problem at a time
    plain = None
    if not args.no_plain:
        P = min(args.plain_sample, B)
        Sp = Solver(weights, state="f32", u="f64", check_every=1)
        up = torch.zeros((1, n, n), dtype=torch.float64, device="cuda")
        # warm the single-problem path once
        Sp.setup(da[0:1].contiguous(), b[0:1]); Sp.solve(df[0:1].contiguous(), up, args.tol, args.maxit)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pit = []
        for p in range(P):
            up.zero_()
            Sp.setup(da[p:p + 1].contiguous(), b[p:p + 1])
            stp, itp, _, psp = Sp.solve(df[p:p + 1].contiguous(), up, args.tol, args.maxit)
            pit.append(int(itp[0]))
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) / P
        plain = {"value": 1.0 / tp, "unit": "solves/s", "problems_timed": P, "mean_iters": float(np.mean(pit))}
        Sp.close()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(weights, a[0], b[0], f[0], mean_iters)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f64" if args.state == "bf16" else "f32+f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {B} problems at {n}x{n}, 16 channels, "
                               f"{datagen.levels_for(n)} levels, tol {args.tol:g}",
                   "global_batch": B, "n": n, "state": args.state, "u": "f64", "weights": wsrc,
                   "parallelism": "single GPU"},
        "converged": converged, "mean_iters": mean_iters, "max_iters": int(np.max(its[-1])),
        "ms_per_iteration": round(iter_ms, 3),
        "oracle_relres_sampled": [float(x) for x in check],
        "roofline": roof, "kernel_time_share": kernel_share,
        "plain_fp32_unbatched": plain,
        "speedup_vs_plain_fp32": (round(value / plain["value"], 3) if plain and plain["value"] > 0 and converged else None),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
