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


def cpu_baseline(weights, a, b, f, iters_per_solve, sample_iters=2, basis=0, gs_passes=1):
    """Time the FP64 oracle on the host: setup + `sample_iters` network iterations of one
    problem; one solve is extrapolated to the GPU's mean iteration count.  With `basis` > 0 (an
    FGMRES solve) the Krylov vector work of an Arnoldi step at that basis size is timed too
    (w = A z with the oracle's operator, `gs_passes` classical Gram-Schmidt passes against the
    basis, normalisation; numpy f64) and added to every iteration."""
    from oracle import operator as oop
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
    kry = 0.0
    if basis > 0:
        rng = np.random.default_rng(0)
        V = rng.standard_normal((basis, f.size))
        z = rng.standard_normal(f.shape)
        t3 = time.perf_counter()
        for _ in range(sample_iters):
            w = oop.apply_A(a, b, z).ravel()
            for _ in range(gs_passes):
                w -= V.T @ (V @ w)
            w /= np.linalg.norm(w)
        kry = (time.perf_counter() - t3) / sample_iters
    solve_s = (t1 - t0) + (per_iter + kry) * max(iters_per_solve, 1.0)
    krylov = (f"; plus the Krylov vector work of an Arnoldi step at basis size {basis} "
              f"({kry:.3f} s: A z, {gs_passes} Gram-Schmidt pass(es), normalisation)") if basis > 0 else ""
    return {
        "value": 1.0 / solve_s, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
        "sample": (f"one {f.shape[0]}x{f.shape[1]} problem: oracle setup ({t1 - t0:.2f} s) + "
                   f"{sample_iters} iterations of residual + network ({per_iter:.2f} s each){krylov}, "
                   f"extrapolated to {iters_per_solve:.1f} iterations per solve (the GPU mean)"),
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


def _solve_timed(S, f, u, tol, maxit):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, it, rr, ps = S.solve(f, u, tol, maxit)
    torch.cuda.synchronize()
    return st, it, rr, ps, time.perf_counter() - t0


def leg_latency31(weights, levels):
    """One 31 x 31 problem (lognormal GRF, l = 0.1, sigma^2 = 1, b = (1, 1), f ~ U(-1, 1)),
    stationary iteration to 1e-8 or 200 iterations, f32 state, f64 u, hipGraph-captured blocks
    of 8 iterations: with untrained Xavier weights (seed 0) and with the benchmark's weights.
    Small grids are launch-bound: time per iteration and kernel launches per iteration."""
    import torch
    import datagen
    from paper_2312_11093_amd import Solver
    a, b, f = datagen.make_batch("grf31", 31, 1)
    da, df = torch.from_numpy(a).cuda(), torch.from_numpy(f).cuda()
    out = {"workload": "grf31: one 31x31 problem, 5 levels, tol 1e-8, maxit 200"}
    for name, w in (("xavier", datagen.xavier_weights(16, 0)), ("bench_weights", weights)):
        S = Solver(w, state="f32", u="f64", use_graph=True, check_every=8, levels=levels)
        S.setup(da, b)
        u = torch.zeros((1, 31, 31), dtype=torch.float64, device="cuda")
        _solve_timed(S, df, u, 1e-8, 200)                                   # warm-up, graph capture
        u.zero_()
        st, it, rr, ps, sec = _solve_timed(S, df, u, 1e-8, 200)
        # launches per iteration and eager time per iteration from a fixed-K forward
        u2 = torch.zeros_like(u)
        S.profile_begin()
        S.forward(df, u2, 4)
        stats = S.profile_end()
        K = 50
        u2.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.forward(df, u2, K)
        torch.cuda.synchronize()
        eager_us = 1e6 * (time.perf_counter() - t0) / K
        S.close()
        out[name] = {"status": int(ps[0]), "iters": int(it[0]), "relres": float(rr[0]),
                     "us_per_iteration_graph_solve": round(1e6 * sec / max(int(it[0]), 1), 1),
                     "us_per_iteration_eager_forward": round(eager_us, 1),
                     "launches_per_iteration": sum(s_["launches"] for s_ in stats) / 4.0}
    return out


def leg_precision4095(weights, levels):
    """One 4095 x 4095 problem to relative residual 1e-10 in three precisions: plain FP32
    (f32 state, f32 u and residual), f32 state with f64 u / residual / norm, and bf16 state
    (bf16 storage, MFMA with f32 accumulation) with f64 u / residual / norm.
      - lognormal GRF (l = 0.05, sigma^2 = 2, b = (1, 1), f ~ U(-1, 1)), divergence form, the
        benchmark's weights as the preconditioner of FGMRES(30) (as a stationary iteration they
        do not converge on this problem);
      - the paper's problem (white-noise coefficients, Re = 1000, f = 1, non-divergence form) with
        the network trained by the paper's protocol, stationary iteration of Eq. (1)."""
    import torch
    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd.weights import embed_channels
    n = 4095
    res, checks = {}, {}
    cases = (("grf4095", weights, dict(method="fgmres", restart=30, gs_passes=1, levels=levels), "div"),
             ("paper_re1e3", embed_channels(np.load(PAPER_WEIGHTS, allow_pickle=False)),
              dict(method="stationary", use_graph=True, levels=-1), "nondiv"))
    for wl, w, kw, form in cases:
        a, b, f = datagen.make_batch(wl, n, 1)
        da, df = torch.from_numpy(a).cuda(), torch.from_numpy(f).cuda()
        sub, sols = {"workload": f"{wl}: one {n}x{n} problem, tol 1e-10, maxit 400, {kw['method']}"}, {}
        for name, state, udt, split in (("plain_fp32", "f32", "f32", 0), ("f32_state_f64_u", "f32", "f64", 1),
                                        ("bf16_state_f64_u", "bf16", "f64", 1)):
            S = Solver(w, state=state, u=udt, f32_split=split, check_every=4, form=form, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.setup(da, b)
            torch.cuda.synchronize()
            tset = time.perf_counter() - t0
            u = torch.zeros((1, n, n), dtype=S.u_dtype, device="cuda")
            st, it, rr, ps, sec = _solve_timed(S, df, u, 1e-10, 400)
            S.close()
            sols[name] = u[0].to(torch.float64).cpu().numpy()
            sub[name] = {"status": int(ps[0]), "iters": int(it[0]), "relres_library": float(rr[0]),
                         "setup_ms": round(1e3 * tset, 2), "solve_ms": round(1e3 * sec, 2)}
            del u
        ref = sols["f32_state_f64_u"]
        nr = float(np.linalg.norm(ref))
        for name in ("plain_fp32", "bf16_state_f64_u"):
            sub[name]["rel_diff_vs_f32_state_f64_u"] = float(np.linalg.norm(sols[name] - ref) / nr)
        res[wl] = sub
        checks[wl] = (a[0], b[0], f[0], form, sols)
    return res, checks


def leg_training127(weights, steps=5):
    """One training step of the unrolled network: 32 problems at 127 x 127 (mixture of lognormal
    GRF, 8 x 8 checkerboards with contrast 1e3 and 20 inclusions with contrast 1e2), random
    velocities, f ~ N(0, 1), K = 8 recorded iterations, loss = mean squared relative residual;
    setup + recorded forward + loss + reverse pass through the iterations and the setup network.
    Device memory: what the library holds beyond the inputs (hipMemGetInfo before / after)."""
    import torch
    import datagen
    from paper_2312_11093_amd import Solver
    n, B, K = 127, 32, 8
    a, b, f = datagen.make_batch("mixture127", n, B, seed=0)
    da, df = torch.from_numpy(a).cuda(), torch.from_numpy(f).cuda()
    wd = torch.from_numpy(np.ascontiguousarray(weights, dtype=np.float32)).cuda()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    S = Solver(weights, state="f32", u="f32")
    u = torch.zeros((B, n, n), dtype=torch.float32, device="cuda")
    du = torch.empty_like(u)
    times, losses = [], []
    for k in range(steps + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.set_weights_device(wd)
        S.setup(da, b)
        u.zero_()
        S.forward(df, u, K, record=True)
        losses.append(S.loss(df, u, du))
        g = S.backward(du)
        torch.cuda.synchronize()
        if k >= 2:
            times.append(time.perf_counter() - t0)
    used = free0 - torch.cuda.mem_get_info()[0]
    finite = bool(torch.isfinite(g).all())
    S.close()
    return {"workload": f"mixture127: {B} problems at {n}x{n}, K = {K}, loss mean relres^2",
            "ms_per_step": round(1e3 * float(np.mean(times)), 2), "steps_timed": steps,
            "loss": float(losses[-1]), "gradient_finite": finite,
            "device_memory_gb": round(used / 1e9, 3)}


def _uneven_run(G, ps, tol, maxit):
    import torch
    a = [torch.from_numpy(p.a).cuda() for p in ps]
    f = [torch.from_numpy(p.f).cuda() for p in ps]
    b = np.stack([p.b for p in ps])
    u = [torch.zeros((p.n, p.n), dtype=torch.float64, device="cuda") for p in ps]
    G.setup(a, b)
    G.solve(f, u, tol, maxit)                                   # warm-up (graph capture)
    for x in u:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G.setup(a, b)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, it, rr, stat = G.solve(f, u, tol, maxit)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ok = stat == 0
    out = {"aligned_levels": G.aligned, "converged": int(ok.sum()), "count": len(ps),
           "solves_per_s": round(len(ps) / (t2 - t0), 2) if ok.all() else 0.0,
           "setup_ms": round(1e3 * (t1 - t0), 1), "solve_ms": round(1e3 * (t2 - t1), 1),
           "iters_p50": float(np.percentile(it, 50)), "iters_p99": float(np.percentile(it, 99)),
           "iters_max": int(np.max(it))}
    if G.aligned:
        ct = G.completion_times()
        out.update({"completion_ms_p50": round(1e3 * float(np.percentile(ct, 50)), 2),
                    "completion_ms_p99": round(1e3 * float(np.percentile(ct, 99)), 2),
                    "completion_note": "device wall clock at each problem's stopping test, from the "
                                       "start of the iterations (after ||f|| and the solver state)"})
    return out, u


def leg_uneven256(weights, levels, count=256):
    """Uneven-size batches: `count` problems with sides drawn uniformly from {63, ..., 2047}.
      - the paper's problem family (white-noise coefficients, Re = 1000, v = (sin 0.5, cos 0.5),
        f = 1, non-divergence form) with the network trained by the paper's protocol, stationary
        iteration to 1e-8 on the aligned levels (one stream, one launch per operation and level
        size, one hipGraph-captured iteration per host check), f32 and bf16 state (bf16 also in
        packed pairs), f64 u; per-problem completion times from device timestamps;
      - the mixture (lognormal GRF, 8 x 8 checkerboards with contrast 1e3, 20 inclusions with
        contrast 1e2; random velocities; f ~ N(0, 1); divergence form) with the benchmark's
        weights as preconditioner of FGMRES(63) with deflated restarts (k = 8), per-size buckets
        on concurrent streams (no trained network converges there as a stationary iteration)."""
    import concurrent.futures as cf
    import datagen
    from paper_2312_11093_amd import GroupSolver
    from paper_2312_11093_amd.weights import embed_channels
    sizes = datagen.var_sizes(count, seed=0)
    res, checks = {"sizes": "uniform in {63, 127, 255, 511, 1023, 2047}", "count": count}, {}
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        pp = list(ex.map(lambda i: datagen.make_problem("paper_re1e3", sizes[i], i, 0), range(count)))
    nodes = float(sum(p.n * p.n for p in pp))
    wt = embed_channels(np.load(PAPER_WEIGHTS, allow_pickle=False))
    for state, pack in (("f32", False), ("bf16", False), ("bf16", True)):
        G = GroupSolver(wt, state=state, u="f64", method="stationary", check_every=1, levels=-1,
                        use_graph=True, form="nondiv", pack_pairs=pack)
        out, u = _uneven_run(G, pp, 1e-8, 400)
        G.close()
        out["workload"] = f"paper_re1e3 family, {nodes / 1e6:.1f} M nodes, stationary, tol 1e-8"
        key = f"paper_family_{state}_" + ("pairs" if pack else "state")
        res[key] = out
        if state == "f32" or pack:
            checks[key] = (pp, u, "nondiv")
        else:
            del u
        print(f"[bench]   uneven paper family {state}{' pairs' if pack else ''} done", file=sys.stderr, flush=True)
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        pm = list(ex.map(lambda i: datagen.make_problem("mixture_var", sizes[i], i, 0), range(count)))
    G = GroupSolver(weights, state="f32", u="f64", method="fgmres", restart=63, gs_passes=1, deflate=8,
                    check_every=4, levels=levels, f32_split=2)
    out, u = _uneven_run(G, pm, 1e-8, 5000)
    G.close()
    out["workload"] = f"mixture_var, {float(sum(p.n * p.n for p in pm)) / 1e6:.1f} M nodes, FGMRES(63) k = 8, tol 1e-8"
    res["mixture_fgmres"] = out
    checks["mixture_fgmres"] = (pm, u, "div")
    return res, checks


PAPER_WEIGHTS = os.path.join(ROOT, "paper_2312_11093_amd", "trained", "t5_c8.npy")


def leg_paper1023(B=64, steps=3):
    """The paper's own problem, batched: B problems at 1023 x 1023 (non-divergence operator,
    white-noise coefficients with Re = 1000, v = (sin 0.5, cos 0.5), f = 1; Sec. 4.1), solved to
    1e-8 by the stationary iteration of Eq. (1) with the network trained by the paper's protocol
    (8 channels, Table 5; log2(n+1) - 1 levels), hipGraph-captured blocks of 4 iterations:
    f32 state and bf16 state (both with f64 u, residual and norm), each also with packed pairs
    (two problems per 16-channel state slot, which the 8-channel network allows), against the
    plain FP32 form (f32 state on f32 MFMA, one problem per call, no graphs) and against the
    paper's GMG (stationary, Sec. 4.1 settings) on the same batch."""
    import torch
    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd.weights import embed_channels
    n = 1023
    w = embed_channels(np.load(PAPER_WEIGHTS, allow_pickle=False))
    a, b, f = datagen.make_batch("paper_re1e3", n, B, seed=0)
    da, df = torch.from_numpy(a).cuda(), torch.from_numpy(f).cuda()
    u = torch.zeros((B, n, n), dtype=torch.float64, device="cuda")

    def timed(S, dA, bb, dF, uu, reps):
        out = []
        for r in range(reps + 1):
            uu.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S.setup(dA, bb)
            st, it, rr, ps = S.solve(dF, uu, 1e-8, 400)
            torch.cuda.synchronize()
            if r > 0:
                out.append(time.perf_counter() - t0)
        return float(np.mean(out)), it, ps

    res = {"workload": f"paper_re1e3: {B} problems at {n}x{n}, stationary, tol 1e-8",
           "weights": os.path.relpath(PAPER_WEIGHTS, ROOT)}
    nets = (("network_f32_state", "f32", False), ("network_bf16_state", "bf16", False),
            ("network_f32_pairs", "f32", True), ("network_bf16_pairs", "bf16", True))
    sampled = {}                                   # the oracle re-checks problems 0 and B - 1 (CPU leg)
    for name, state, pack in nets:
        S = Solver(w, state=state, u="f64", form="nondiv", levels=-1, use_graph=True, check_every=1,
                   f32_split=2, pack_pairs=pack)
        sec, it, ps = timed(S, da, b, df, u, steps)
        S.close()
        sampled[name] = {p: u[p].cpu().numpy() for p in (0, B - 1)}
        res[name] = {"solves_per_s": round(B / sec, 2) if (ps == 0).all() else 0.0,
                     "ms_per_batch": round(1e3 * sec, 2), "iters_mean": float(np.mean(it)),
                     "iters_max": int(np.max(it)), "converged": int((ps == 0).sum())}
    # plain FP32, one problem per call: every problem of the batch timed (setup + solve), after
    # one untimed warm-up solve
    Sp = Solver(w, state="f32", u="f64", form="nondiv", levels=-1, f32_split=0, check_every=1)
    up = torch.zeros((1, n, n), dtype=torch.float64, device="cuda")
    timed(Sp, da[0:1].contiguous(), b[0:1], df[0:1].contiguous(), up, 1)
    tp, pconv = 0.0, 0
    for p in range(B):
        up.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Sp.setup(da[p:p + 1].contiguous(), b[p:p + 1])
        _, _, _, ps = Sp.solve(df[p:p + 1].contiguous(), up, 1e-8, 400)
        torch.cuda.synchronize()
        tp += time.perf_counter() - t0
        pconv += int((ps == 0).all())
    Sp.close()
    res["plain_fp32_unbatched"] = {"solves_per_s": round(B / tp, 2) if pconv == B else 0.0,
                                   "how": f"all {B} problems one at a time (f32 MFMA, no graphs)"}
    Sg = Solver(None, precond="gmg", u="f64", form="nondiv", use_graph=True, check_every=1)
    sec, it, ps = timed(Sg, da, b, df, u, steps)
    Sg.close()
    res["gmg_stationary"] = {"solves_per_s": round(B / sec, 2) if (ps == 0).all() else 0.0,
                             "ms_per_batch": round(1e3 * sec, 2), "iters_mean": float(np.mean(it)),
                             "converged": int((ps == 0).sum())}
    pl = res["plain_fp32_unbatched"]["solves_per_s"]
    for name, _, _ in nets:
        res[name]["over_plain_fp32_unbatched"] = round(res[name]["solves_per_s"] / pl, 3)
        if res["gmg_stationary"]["solves_per_s"] > 0:
            res[name]["over_gmg"] = round(res[name]["solves_per_s"] / res["gmg_stationary"]["solves_per_s"], 3)
    check = {p: (a[p], b[p], f[p]) for p in (0, B - 1)}
    return res, (check, sampled)


def run_legs(weights, args):
    legs = {}
    legs["paper_1023_batch64"], paper = leg_paper1023()
    print("[bench] leg paper problem 1023^2 x 64 done", file=sys.stderr, flush=True)
    legs["latency_31"] = leg_latency31(weights, args.levels)
    print("[bench] leg 31^2 done", file=sys.stderr, flush=True)
    legs["precision_4095"], check = leg_precision4095(weights, args.levels)
    print("[bench] leg 4095^2 done", file=sys.stderr, flush=True)
    legs["training_step_127"] = leg_training127(weights)
    print("[bench] leg training step done", file=sys.stderr, flush=True)
    legs["uneven_batch"], uneven = leg_uneven256(weights, args.levels)
    print("[bench] leg uneven batch done", file=sys.stderr, flush=True)
    return legs, (check, uneven, paper)


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
    ap.add_argument("--plain-sample", type=int, default=64,
                    help="problems solved one by one in the plain-FP32 comparison (all of the batch by "
                         "default: the rate is then measured, not extrapolated)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--deflate", type=int, default=8,
                    help="FGMRES deflated restarts: directions kept across a restart (0 = plain)")
    ap.add_argument("--no-gmg", action="store_true",
                    help="skip the geometric multigrid baseline (FGMRES(63), same batch)")
    ap.add_argument("--no-tuning", action="store_true",
                    help="keep the default tile of every convolution (no autotuned table)")
    ap.add_argument("--levels", type=int, default=0,
                    help="network levels: 0 = log2(n+1), -1 = the count of Sec. 4.1, ...")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the compact legs of the other workloads (31^2 latency, 4095^2 "
                         "precision, training step, uneven sizes)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import datagen
    from paper_2312_11093_amd import Solver

    from paper_2312_11093_amd import autotune
    tuned = 0 if args.no_tuning else autotune.load()

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
                      f32_split=args.f32_split, levels=args.levels)

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
    S2 = Solver(weights, state=args.state, u="f64", f32_split=args.f32_split, levels=args.levels)
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
                    gs_passes=args.gs_passes, f32_split=False, deflate=dfl, levels=args.levels)
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
        # with a sample of the batch, iteration counts differ widely between problems: the measured
        # single-problem setup time and time per iteration are applied to the batch's own counts
        t_batch_seq = B * float(np.mean(tset)) + per_iter * float(np.sum(its[-1]))
        measured = P / (sum(tset) + sum(tsol))
        whole = P == B
        plain = {"value": measured if whole else B / t_batch_seq, "unit": "solves/s",
                 "how": (f"all {B} problems solved one at a time (FP32 state on f32 MFMA, f64 u, no graphs), "
                         f"setup + solve timed per problem" if whole else
                         f"problems 0..{P - 1} solved one at a time (FP32 state on f32 MFMA, f64 u, no graphs); "
                         f"their setup time and time per iteration, applied to the iteration counts "
                         f"of all {B} problems"),
                 "problems_timed": P, "iters_mean": float(np.mean(pit)), "iters_max": int(np.max(pit)),
                 "iters_differ_from_batched": int(sum(int(pit[p] != its[-1][p]) for p in range(P))),
                 "setup_ms": round(1000 * float(np.mean(tset)), 3), "ms_per_iteration": round(1000 * per_iter, 4),
                 "measured_solves_per_s": round(measured, 4),
                 "extrapolated_from_batched_iterations": round(B / t_batch_seq, 4),
                 "converged": all(x == 0 for x in pst)}
        Sp.close()
        print("[bench] plain FP32 unbatched done", file=sys.stderr, flush=True)

    # the paper's comparison solver on the same GPU: geometric multigrid (rediscretised coarse
    # operators, bilinear transfers, 3 + 3 weighted-Jacobi sweeps with weight 0.67, exact
    # coarsest solve), same batch and tolerance, as the preconditioner of FGMRES(63) with
    # deflated restarts (k = 8): as a stationary iteration it diverges on the block workload
    # (injected coarse coefficients misrepresent the 1e4 jumps)
    gmg = None
    if not args.no_gmg:
        Sg = Solver(None, precond="gmg", u="f64", check_every=args.check_every, method="fgmres",
                    restart=63, gs_passes=1, deflate=8)

        def gstep():
            u.zero_()
            Sg.setup(da, b)
            return Sg.solve(df, u, args.tol, args.maxit)

        gstep()
        gt, git = [], None
        for k in range(min(args.steps, 5)):
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
                       "preconditioner of FGMRES(63) with deflated restarts (k = 8), same batch "
                       "and tolerance"}
        Sg.close()
        print("[bench] GMG baseline done", file=sys.stderr, flush=True)

    # CPU leg: the FP64 oracle timed on the host, and the oracle's residual of the sampled
    # solutions (main solve and GMG baseline)
    cpu, check = None, None
    if not args.no_cpu_baseline:
        # FGMRES with deflated restarts runs its Arnoldi steps at basis sizes deflate .. restart - 1
        basis = (args.deflate + args.restart) // 2 if args.method == "fgmres" else 0
        cpu = cpu_baseline(weights, a[0], b[0], f[0], mean_iters, basis=basis, gs_passes=args.gs_passes)
        from oracle import solve as osv
        check = [float(osv.relres(a[p], b[p], f[p], x)) for p, x in sampled.items()]
        if gmg is not None:
            gmg["oracle_relres_sampled"] = [float(osv.relres(a[p], b[p], f[p], x))
                                            for p, x in gsampled.items()]
        print("[bench] cpu baseline done", file=sys.stderr, flush=True)

    full = datagen.levels_for(n)
    net_levels = full + args.levels if args.levels < 0 else (args.levels or full)
    legs, legs_check = (None, None) if args.no_legs else run_legs(weights, args)
    if legs_check is not None and cpu is not None:
        # the oracle's f64 residual of every 4095^2 solution and of one problem of each size of
        # the uneven batch (CPU leg)
        from oracle import solve as osv
        checks4, uneven_checks, (paper_probs, paper_sols) = legs_check
        for name, sols in paper_sols.items():
            legs["paper_1023_batch64"][name]["oracle_relres_sampled"] = [
                float(osv.relres(*paper_probs[p], x, "nondiv")) for p, x in sorted(sols.items())]
        for wl, (a4, b4, f4, form4, sols) in checks4.items():
            for name, x in sols.items():
                legs["precision_4095"][wl][name]["relres_oracle"] = float(osv.relres(a4, b4, f4, x, form4))
        for key, (ups, uu, form_u) in uneven_checks.items():
            seen = {}
            for p, x in zip(ups, uu):
                if p.n not in seen:
                    seen[p.n] = float(osv.relres(p.a, p.b, p.f, x.cpu().numpy(), form_u))
            legs["uneven_batch"][key]["oracle_relres_one_per_size"] = {str(k): v for k, v in sorted(seen.items())}
        print("[bench] oracle residuals of the legs done", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": round(value, 3), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": f"{args.state}+f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {B} problems at {n}x{n}, 16 channels, "
                               f"{net_levels} levels, tol {args.tol:g}",
                   "global_batch": B, "n": n, "method": args.method,
                   "restart": args.restart if args.method == "fgmres" else None,
                   "gs_passes": args.gs_passes if args.method == "fgmres" else None,
                   "deflate": dfl if args.method == "fgmres" else None,
                   "state": args.state, "f32_split": args.f32_split if args.state == "f32" else None,
                   "u": "f64", "weights": wsrc, "parallelism": "single GPU",
                   "tile_variants": (f"{tuned} autotuned entries "
                                     f"({os.path.relpath(autotune.DEFAULT_FILE, ROOT)})" if tuned else "defaults")},
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
        "legs": legs,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
