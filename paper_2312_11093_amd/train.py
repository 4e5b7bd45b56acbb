"""Offline training of the MGCNN weights on the GPU (Sec. 3.4; schedule after Appendix A.1,
Table 5): unsupervised residual loss with white-noise right-hand sides, setup and solve
networks trained jointly through K unrolled iterations, progressively growing grid sizes
with shrinking batches, Adam with a step learning-rate decay.

Coefficients come from the seeded generators (random 16 x 16 blocks with log10 a in
[-2, 2], lognormal Gaussian random fields, 8 x 8 checkerboards with contrast 1e3, circular
inclusions with contrast 1e2) with random velocities |b| <= 10.  Every step draws a batch of
coefficient fields from a pre-generated pool and fresh N(0, 1) right-hand sides on the GPU.

    python -m paper_2312_11093_amd.train --out weights.npy [--resume ckpt.pt] [--minutes 15]

Checkpoints (weights + Adam state + progress) make long schedules resumable across runs.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# (n, batch, K, steps, slow_fraction, max_pre_iterations) -- grid sizes double while the
# batch halves (Table 5 pattern).  A fraction of the steps trains on "slow" right-hand sides:
# the residual left after a few unrecorded iterations of the current network, so the loss
# (relative residual after K more iterations) measures the contraction of the slowest modes.
DEFAULT_SCHEDULE = [(31, 16, 2, 4000, 0.5, 12), (63, 8, 2, 4000, 0.5, 16),
                    (127, 4, 2, 4000, 0.6, 20), (255, 2, 2, 3000, 0.6, 24)]


FAMILIES = ("blocks", "grf", "checker", "inclusions")


def coefficient_pool(n: int, count: int, seed: int, mix=(1, 1, 1, 1)):
    """Float32 coefficient fields (count, n, n) from the four families (blocks, GRF,
    checkerboard, inclusions) in the proportions `mix`."""
    import datagen
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 9001, n])))
    out = np.empty((count, n, n), np.float32)
    kinds = np.repeat(np.arange(4), np.asarray(mix, dtype=int))
    for i in range(count):
        kind = int(kinds[i % len(kinds)])
        if kind == 0:
            a = datagen.blocks_lognormal(n, rng)
        elif kind == 1:
            a = np.exp(datagen.grf(n, rng, rng.uniform(0.05, 0.2), rng.uniform(0.5, 2.0)))
        elif kind == 2:
            a = datagen.checkerboard(n, rng)
        else:
            a = datagen.inclusions(n, rng)
        out[i] = a
    return out


def random_velocity(rng, B):
    th = rng.uniform(0, 2 * math.pi, B)
    mag = rng.uniform(0, 10, B)
    return np.stack([mag * np.cos(th), mag * np.sin(th)], 1).astype(np.float32)


def train(out: str, schedule=None, lr: float = 3e-3, decay_every: int = 2000, gamma: float = 0.8,
          seed: int = 0, resume: str | None = None, minutes: float = 1e9, pool: int = 256,
          log: str | None = None, init: str | None = None, clip: float = 0.0, mix=(1, 1, 1, 1)):
    import torch

    import datagen
    from paper_2312_11093_amd import Solver

    schedule = schedule or DEFAULT_SCHEDULE
    t_end = time.time() + 60.0 * minutes
    if init and os.path.exists(init):
        w0 = np.load(init, allow_pickle=False).astype(np.float32)
    else:
        w0 = datagen.xavier_weights(16, seed)
    w = torch.tensor(w0, device="cuda", dtype=torch.float32)
    opt = torch.optim.Adam([w], lr=lr)
    sched = torch.optim.lr_scheduler.StepLR(opt, step_size=decay_every, gamma=gamma)
    state = {"stage": 0, "step": 0, "total": 0}
    if resume and os.path.exists(resume):
        ck = torch.load(resume, weights_only=True, map_location="cuda")
        w.copy_(ck["w"])
        opt.load_state_dict(ck["opt"])
        sched.load_state_dict(ck["sched"])
        state = {k: int(v) for k, v in ck["state"].items()}
    S = Solver(w.cpu().numpy(), state="f32", u="f32")
    rng = np.random.default_rng(seed + 1000 * state["total"])
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed + 7919 * state["total"] + 1)
    logf = open(log, "a") if log else None
    while state["stage"] < len(schedule):
        entry = tuple(schedule[state["stage"]]) + (0.0, 0)
        n, B, K, steps, slow_frac, kpre_max = entry[:6]
        a_pool = torch.from_numpy(coefficient_pool(n, pool, seed + state["stage"], mix)).cuda()
        u = torch.zeros((B, n, n), device="cuda")
        du = torch.empty_like(u)
        ema = None
        t0 = time.time()
        while state["step"] < steps:
            idx = torch.from_numpy(rng.integers(0, pool, B)).cuda()
            a = a_pool[idx].contiguous()
            b = random_velocity(rng, B)
            f = torch.randn((B, n, n), device="cuda", generator=gen)
            S.set_weights_device(w)
            S.setup(a, b)
            slow = slow_frac > 0 and rng.random() < slow_frac
            if slow:
                # right-hand side = residual after a few iterations of the current network
                u.zero_()
                S.forward(f, u, int(rng.integers(2, max(3, kpre_max + 1))))
                f = S.residual(f, u)
                if not bool(torch.isfinite(f).all()):
                    state["step"] += 1
                    state["total"] += 1
                    continue
            u.zero_()
            S.forward(f, u, K, record=True)
            S.loss(f, u, du)
            # per-problem log loss: mean_i log(relres_i^2).  Its gradient is the gradient of
            # relres_i^2 divided by relres_i^2, so problems whose residual is still large (or
            # growing) do not swamp the others; problems that blew up are dropped.
            rr = S.residual_norms(f, u)
            scale = np.where(np.isfinite(rr) & (rr > 0) & (rr < 1e6), 1.0 / np.maximum(rr, 1e-30) ** 2, 0.0)
            du.mul_(torch.from_numpy(scale.astype(np.float32)).cuda().view(-1, 1, 1))
            ok = scale > 0
            loss = float(np.mean(np.log10(rr[ok] ** 2))) if ok.any() else float("nan")
            g = S.backward(du)
            if not math.isfinite(loss) or not bool(torch.isfinite(g).all()):
                # skip the update of a diverged batch (huge loss); keep going
                state["step"] += 1
                state["total"] += 1
                continue
            gn = float(torch.linalg.vector_norm(g))
            if clip and gn > clip * max(1.0, loss):
                g = g * (clip * max(1.0, loss) / gn)
            w.grad = g
            opt.step()
            opt.zero_grad(set_to_none=True)
            sched.step()
            state["step"] += 1
            state["total"] += 1
            lg = loss
            key = "slow" if slow else "noise"
            if ema is None:
                ema = {}
            ema[key] = lg if key not in ema else 0.98 * ema[key] + 0.02 * lg
            if state["step"] % 250 == 0 or state["step"] == steps:
                rec = {"stage": state["stage"], "n": n, "B": B, "K": K, "step": state["step"],
                       "total": state["total"], "log10_loss_ema": {k: round(v, 3) for k, v in ema.items()}, "loss": loss,
                       "lr": opt.param_groups[0]["lr"], "sec": round(time.time() - t0, 1)}
                print(json.dumps(rec), flush=True)
                if logf:
                    logf.write(json.dumps(rec) + "\n"); logf.flush()
            if time.time() > t_end:
                break
        if time.time() > t_end:
            break
        state["stage"] += 1
        state["step"] = 0
    wn = w.detach().cpu().numpy().astype(np.float32)
    np.save(out, wn)
    ck_path = os.path.splitext(out)[0] + "_ckpt.pt"
    torch.save({"w": w.detach(), "opt": opt.state_dict(), "sched": sched.state_dict(),
                "state": {k: torch.tensor(v) for k, v in state.items()}}, ck_path)
    S.close()
    done = state["stage"] >= len(schedule)
    print(json.dumps({"saved": out, "checkpoint": ck_path, "finished": done, "state": state}), flush=True)
    return done


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--init", default=None)
    ap.add_argument("--minutes", type=float, default=1e9)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--decay-every", type=int, default=2000)
    ap.add_argument("--gamma", type=float, default=0.8)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--pool", type=int, default=256)
    ap.add_argument("--log", default=None)
    ap.add_argument("--schedule", default=None, help="json list of [n, batch, K, steps, slow_fraction, max_pre]")
    ap.add_argument("--mix", default="1,1,1,1", help="proportions of blocks, grf, checkerboard, inclusions")
    args = ap.parse_args()
    schedule = [tuple(x) for x in json.loads(args.schedule)] if args.schedule else None
    train(args.out, schedule, args.lr, args.decay_every, args.gamma, args.seed, args.resume,
          args.minutes, args.pool, args.log, args.init, 0.0, tuple(int(x) for x in args.mix.split(",")))


if __name__ == "__main__":
    main()
