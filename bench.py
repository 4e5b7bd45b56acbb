"""Benchmark: batched MGCNN solves to relative residual 1e-8 on one MI355X.

One step = the whole hot path over one batch: the setup phase for every problem, then the
solve until every problem of the batch reaches ||f - A u|| / ||f|| <= 1e-8.  The solve is the
restarted FGMRES wrapper (the network as right preconditioner) by default, or the plain
stationary iteration.  Inputs (coefficients, velocities, right-hand sides) are synthetic,
seeded and resident in HBM before the timed region.

Default workload: 64 problems at 1023 x 1023, a piecewise constant on a random 16 x 16 block
partition with log10 a ~ U(-2, 2), b = |b|(cos t, sin t) with |b| ~ U(0, 10), f ~ N(0, 1);
16 channels, 10 levels; float32 state on MFMA, f64 u / residual / norm.  Weights: the hand-set
coefficient-aware V(1,1) cycle (no trained weights ship with the library).

Prints one JSON line: metric, value (solves/s, whole batch, setup + solve; the setup time and
the solve-only rate beside it), roofline of the dominant kernel
(HIP events around its launches in a profiled pass), the same solver run one problem at a time
in FP32 ("plain FP32 unbatched") on the same GPU, and the FP64 oracle timed on the host cores.
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
FP32_PEAK_TFS = 157.3
BF16_PEAK_TFS = 2500.0


def load_weights(spec):
    """'handbuilt' (the hand-set V(1,1) cycle), 'xavier' (seed 0, untrained) or a .npy path."""
    import datagen
    from paper_2312_11093_amd.handbuilt import vcycle_weights
    if spec == "handbuilt":
        import inspect
        om = inspect.signature(vcycle_weights).parameters["omega"].default
        return vcycle_weights(), f"hand-set coefficient-aware V(1,1) cycle (omega {om})"
    if spec == "xavier":
        return datagen.xavier_weights(16, 0), "xavier-seed0 (untrained)"
    return np.load(spec, allow_pickle=False).astype(np.float32), os.path.relpath(os.path.abspath(spec), ROOT)


def cpu_baseline(weights, a, b, f, iters_per_solve, sample_iters=2):
    """Time the FP64 oracle on the host: setup + `sample_iters` network iterations of one
    problem; one solve is extrapolated to the GPU's mean iteration count."""
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
                   f"{sample_iters} iterations of residual + network ({per_iter:.2f} s each), "
                   f"extrapolated to {iters_per_solve:.1f} iterations per solve (the GPU mean; "
                   f"the Krylov vector work of those iterations is not included)"),
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_finest_level_64x1023_f32.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2312_11093_amd", "csrc", f)
                  for f in ("kernels_conv16.hip", "kernels_stencil.hip")]


def measured_traffic_ratio(kind):
    """HBM traffic / algorithmic bytes of a finest-level kernel from the committed rocprofv3
    --pmc summary, or None if the summary is missing or the kernel sources changed since."""
    import hashlib
    try:
        line = [ln for ln in open(TRAFFIC_FILE) if ln.startswith("traffic_json:")][0]
        rec = json.loads(line.split(":", 1)[1])
        h = hashlib.sha1()
        for f in KERNEL_SOURCES:
            h.update(open(f, "rb").read())
        if h.hexdigest() != rec["source_sha1"]:
            return None
        return rec["ratio"].get(kind)
    except (OSError, IndexError, ValueError, KeyError):
        return None


def matrix_peak(kind, level, split):
    """(peak in algorithmic TFLOP/s, arithmetic) of a kernel's matrix instructions.  With f32
    state: the 16 -> 16 same-size convs run on bf16 MFMA over a k-way bf16 split of both operands
    (k(k+1)/2 bf16 products per algorithmic product: 6 for the three-way split, 3 for the two-way
    split of the finest down smoother when split = 2), so their algorithmic peak is the dense bf16
    peak / that count; the restriction, the prolongation and the finest down smoother at split
    = 1 use f32 MFMA.  split < 0: bf16 state, every conv on plain bf16 MFMA."""
    if split < 0:
        return BF16_PEAK_TFS, "bf16 MFMA"
    if split == 0:
        return FP32_PEAK_TFS, "f32 MFMA"
    if kind == "smooth_in":
        return (BF16_PEAK_TFS / 3, "bf16 MFMA, two-way split (3 products)") if split == 2 else (
            FP32_PEAK_TFS, "f32 MFMA")
    if kind in ("smooth_down", "smooth_up"):
        return BF16_PEAK_TFS / 6, "bf16 MFMA, three-way split (6 products)"
    return FP32_PEAK_TFS, "f32 MFMA"


def roofline_of(stats, split=1):
    """Per-kind time shares and the roofline of the (kind, level) entry with the most time.
    A kernel whose algorithmic intensity (flops / HBM bytes) is above the ridge point of its
    matrix arithmetic (``matrix_peak``) / 8 TB/s is judged against that matrix peak, otherwise
    against HBM."""
    by_kind = {}
    for s_ in stats:
        by_kind[s_["kind"]] = by_kind.get(s_["kind"], 0.0) + s_["ms_total"]
    top = max(stats, key=lambda s_: s_["ms_total"])
    avg_ms = top["ms_total"] / top["launches"]
    gbs = top["bytes_per_launch"] / (avg_ms / 1000.0) / 1e9
    tfs = top["flops_per_launch"] / (avg_ms / 1000.0) / 1e12
    intensity = top["flops_per_launch"] / max(top["bytes_per_launch"], 1.0)
    mpeak, arith = matrix_peak(top["kind"], top["level"], split)
    ridge = mpeak * 1e12 / (HBM_PEAK_GBS * 1e9)
    what = f"{top['kind']} (level {top['level']}, {top['launches']} launches, {avg_ms:.3f} ms avg)"
    ratio = measured_traffic_ratio(top["kind"]) if top["level"] == 0 else None
    traffic = round(ratio * top["bytes_per_launch"]) if ratio is not None else None
    traffic_note = ("HBM bytes per launch: rocprofv3 FETCH_SIZE + WRITE_SIZE of the full-size launch, "
                    "calibrated on a 1 GiB streaming kernel, as a ratio to the algorithmic bytes "
                    "(profiles/pmc_finest_level_64x1023_f32.md)") if traffic is not None else None
    if intensity > ridge:
        roof = {"bound": "mfma", "achieved": round(tfs, 2), "peak": round(mpeak, 1), "unit": "TFLOP/s",
                "frac": round(tfs / mpeak, 4), "traffic": traffic, "kernel": what, "arithmetic": arith,
                "flops_per_launch": top["flops_per_launch"], "bytes_per_launch": top["bytes_per_launch"],
                "traffic_note": traffic_note,
                "intensity_flop_per_byte": round(intensity, 2), "hbm_gbs": round(gbs, 1)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": what, "arithmetic": arith,
                "matrix_peak_tflops": round(mpeak, 1), "achieved_tflops": round(tfs, 2),
                "bytes_per_launch": top["bytes_per_launch"], "traffic_note": traffic_note,
                "intensity_flop_per_byte": round(intensity, 2)}
    total = sum(by_kind.values())
    share = {k: round(v / total, 4) for k, v in sorted(by_kind.items(), key=lambda kv: -kv[1])}
    per_level0 = {s_["kind"]: {"ms": round(s_["ms_total"] / s_["launches"], 4),
                               "GB/s": round(s_["bytes_per_launch"] / (s_["ms_total"] / s_["launches"]) / 1e6, 1)}
                  for s_ in stats if s_["level"] == 0 and s_["kind"] in
                  ("smooth_in", "smooth_up", "prolong", "restrict", "out_update", "residual")}
    return roof, share, total, per_level0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--workload", default="blocks1023")
    ap.add_argument("--method", default="fgmres", choices=["fgmres", "stationary"])
    ap.add_argument("--restart", type=int, default=63)
    ap.add_argument("--gs-passes", type=int, default=1, choices=[1, 2],
                    help="classical Gram-Schmidt passes per Arnoldi step")
    ap.add_argument("--state", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--f32-split", type=int, default=2, choices=[0, 1, 2],
                    help="f32 state: 0 = f32 MFMA, 1 = three-way bf16 split of the 16->16 convs, "
                         "2 = as 1 with a two-way split in the finest down smoother")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=10000)
    ap.add_argument("--check-every", type=int, default=4)
    ap.add_argument("--weights", default="handbuilt")
    ap.add_argument("--plain-sample", type=int, default=2,
                    help="problems solved one by one in the plain-FP32 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--deflate", type=int, default=8,
                    help="FGMRES deflated restarts: directions kept across a restart (0 = plain)")
    ap.add_argument("--no-gmg", action="store_true",
                    help="skip the geometric multigrid baseline (same outer method, same batch)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    from paper_2312_11093_amd import Solver

    n, B = args.n, args.batch
    weights, wsrc = load_weights(args.weights)
    a, b, f = datagen.make_batch(args.workload, n, B, seed=0)
    da = torch.from_numpy(a).cuda()
    df = torch.from_numpy(f).cuda()
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")

    def make(state, use_graph):
        return Solver(weights, state=state, u="f64", check_every=args.check_every,
                      use_graph=use_graph and args.method == "stationary", method=args.method,
                      restart=args.restart, gs_passes=args.gs_passes, deflate=dfl,
                      f32_split=args.f32_split)

    dfl = args.deflate if args.method == "fgmres" else 0
    S = make(args.state, not args.no_graph)

    setup_times = []

    def step():
        u.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.setup(da, b)
        torch.cuda.synchronize()
        setup_times.append(time.perf_counter() - t0)
        return S.solve(df, u, args.tol, args.maxit)

    for _ in range(args.warmup):
        step()
        print(f"[bench] warmup step done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, its = [], []
    del setup_times[:]
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, it, rr, ps = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        its.append(it.copy())
        print(f"[bench] step {k}: {times[-1]:.3f} s, iterations mean {it.mean():.1f} max {it.max()}",
              file=sys.stderr, flush=True)
    ms = 1000.0 * float(np.mean(times))
    converged = bool((ps == 0).all())
    mean_iters = float(np.mean(its[-1]))
    value = B / (ms / 1000.0) if converged else 0.0

    # the returned solutions of two sampled problems, for the host FP64 check of the CPU leg
    sampled = {p: u[p].cpu().numpy() for p in (0, B - 1)}

    # time of one batched stationary iteration (residual + network + update), weight independent
    KI = 10
    S2 = Solver(weights, state=args.state, u="f64", f32_split=args.f32_split)
    S2.setup(da, b)
    u.zero_()
    S2.forward(df, u, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S2.forward(df, u, KI)
    torch.cuda.synchronize()
    iter_ms = 1000.0 * (time.perf_counter() - t0) / KI
    S2.close()

    # profiled pass: HIP events around every launch of one more whole solve (bytes are counted
    # for the problems still live at each launch)
    u.zero_()
    S.setup(da, b)
    S.profile_begin()
    S.solve(df, u, args.tol, args.maxit)
    stats = S.profile_end()
    roof, kernel_share, prof_ms, level0 = roofline_of(stats, args.f32_split if args.state == "f32" else -1)
    S.close()
    print("[bench] profiled pass done", file=sys.stderr, flush=True)

    # the same solver, one problem at a time, FP32 state, no graphs
    plain = None
    if not args.no_plain:
        P = min(args.plain_sample, B)
        # plain FP32: float32 matrix instructions, one problem per call, no graphs
        Sp = Solver(weights, state="f32", u="f64", check_every=1, method=args.method, restart=args.restart,
                    gs_passes=args.gs_passes, f32_split=False, deflate=dfl)
        up = torch.zeros((1, n, n), dtype=torch.float64, device="cuda")
        Sp.setup(da[0:1].contiguous(), b[0:1])
        Sp.solve(df[0:1].contiguous(), up, args.tol, min(args.maxit, 2 * args.restart))   # warm-up
        torch.cuda.synchronize()
        pit, pst, tset, tsol = [], [], [], []
        for p in range(P):
            up.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Sp.setup(da[p:p + 1].contiguous(), b[p:p + 1])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, itp, _, psp = Sp.solve(df[p:p + 1].contiguous(), up, args.tol, args.maxit)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            tset.append(t1 - t0)
            tsol.append(t2 - t1)
            pit.append(int(itp[0]))
            pst.append(int(psp[0]))
        per_iter = sum(tsol) / max(sum(pit), 1)
        # iteration counts differ widely between problems: extrapolate the measured single-problem
        # setup time and time per iteration to the batch's own iteration counts
        t_batch_seq = B * float(np.mean(tset)) + per_iter * float(np.sum(its[-1]))
        plain = {"value": B / t_batch_seq, "unit": "solves/s",
                 "how": (f"problems 0..{P - 1} solved one at a time (FP32 state on f32 MFMA, f64 u, no graphs); "
                         f"their setup time and time per iteration, applied to the iteration counts "
                         f"of all {B} problems"),
                 "problems_timed": P, "iters": pit, "batched_iters_same_problems": [int(its[-1][p]) for p in range(P)],
                 "setup_ms": round(1000 * float(np.mean(tset)), 3), "ms_per_iteration": round(1000 * per_iter, 4),
                 "measured_solves_per_s_sample": round(P / (sum(tset) + sum(tsol)), 4),
                 "converged": all(x == 0 for x in pst)}
        Sp.close()
        print("[bench] plain FP32 unbatched done", file=sys.stderr, flush=True)

    # the paper's comparison solver on the same GPU: geometric multigrid (rediscretised coarse
    # operators, bilinear transfers, 3 + 3 weighted-Jacobi sweeps with weight 0.67, exact
    # coarsest solve) as the preconditioner of the same outer method, same batch and tolerance
    gmg = None
    if not args.no_gmg:
        Sg = Solver(None, precond="gmg", u="f64", check_every=args.check_every, method=args.method,
                    restart=args.restart, gs_passes=args.gs_passes, deflate=dfl)

        def gstep():
            u.zero_()
            Sg.setup(da, b)
            return Sg.solve(df, u, args.tol, args.maxit)

        gstep()
        gt, git = [], None
        for k in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, git, _, gps = gstep()
            torch.cuda.synchronize()
            gt.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Sg.setup(da, b)
        torch.cuda.synchronize()
        gsetup = time.perf_counter() - t0
        gms = 1000.0 * float(np.mean(gt))
        gconv = bool((gps == 0).all())
        gsampled = {p: u[p].cpu().numpy() for p in (0, B - 1)}
        gmg = {"value": round(B / (gms / 1000.0), 3) if gconv else 0.0, "unit": "solves/s",
               "ms_per_step": round(gms, 3), "setup_ms": round(1000 * gsetup, 3),
               "converged": gconv, "mean_iters": float(np.mean(git)), "max_iters": int(np.max(git)),
               "oracle_relres_sampled": None,
               "settings": {"levels": Sg.gmg_levels, "sweeps": 3, "omega": 0.67,
                            "coarsest": "exact solve", "coarse_coefficient": "injection"},
               "what": "geometric multigrid V-cycle (Sec. 2.3 / Sec. 4.1 settings) as the "
                       "preconditioner of the same outer method, same batch and tolerance"}
        Sg.close()
        print("[bench] GMG baseline done", file=sys.stderr, flush=True)

    # CPU leg: the FP64 oracle timed on the host, and the oracle's residual of the sampled
    # solutions (main solve and GMG baseline)
    cpu, check = None, None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(weights, a[0], b[0], f[0], mean_iters)
        from oracle import solve as osv
        check = [float(osv.relres(a[p], b[p], f[p], x)) for p, x in sampled.items()]
        if gmg is not None:
            gmg["oracle_relres_sampled"] = [float(osv.relres(a[p], b[p], f[p], x))
                                            for p, x in gsampled.items()]
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{args.state}+f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {B} problems at {n}x{n}, 16 channels, "
                               f"{datagen.levels_for(n)} levels, tol {args.tol:g}",
                   "global_batch": B, "n": n, "method": args.method,
                   "restart": args.restart if args.method == "fgmres" else None,
                   "gs_passes": args.gs_passes if args.method == "fgmres" else None,
                   "deflate": dfl if args.method == "fgmres" else None,
                   "state": args.state, "f32_split": args.f32_split if args.state == "f32" else None,
                   "u": "f64", "weights": wsrc, "parallelism": "single GPU"},
        "converged": converged, "mean_iters": mean_iters, "max_iters": int(np.max(its[-1])),
        "ms_per_stationary_iteration": round(iter_ms, 3),
        "oracle_relres_sampled": check,
        "roofline": roof, "kernel_time_share": kernel_share, "finest_level_kernels": level0,
        "profiled_pass": {"what": "one whole solve of the batch", "kernel_ms": round(prof_ms, 2)},
        "plain_fp32_unbatched": plain,
        "setup_ms": round(1000.0 * float(np.mean(setup_times)), 3),
        "solves_per_s_solve_only": (round(B / ((ms - 1000.0 * float(np.mean(setup_times))) / 1000.0), 3)
                                    if converged else 0.0),
        "speedup_vs_plain_fp32": (round(value / plain["value"], 3)
                                  if plain and plain["value"] > 0 and converged else None),
        "gmg_baseline": gmg,
        "mgcnn_over_gmg": (round(value / gmg["value"], 3)
                           if gmg and gmg["value"] > 0 and converged else None),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
