"""The paper's own training protocol on the paper's own problem, run through the library's
recorded forward and hand-written reverse pass (Sec. 3.4, Eq. (19); Sec. 4.1 problem settings;
Appendix A.1, Table 5).

Problem: the non-divergence operator of Eq. (7) with v = (sin 0.5, cos 0.5) and white-noise
coefficients whose mesh Reynolds number spans [1, Re] (Re = 1000), generated fresh for every
batch, with fresh white-noise right-hand sides.

Loss: one application of the solve network from a zero guess (one iteration of Eq. (1)) and the
absolute squared residual, averaged over the batch (Eq. (19)), here divided by the node count
n^2 (a constant factor per grid size).  The log reports the mean squared relative residual
||f - A u||^2 / ||f||^2 after that iteration, which the white-noise right-hand sides make equal to
the loss per node up to sampling noise.

Schedule (Table 5): 50 epochs of 1000 batches; the grid starts at 31 x 31 with 4 levels and
batch 16, and every 10 epochs the grid side doubles (63, 127, 255, 511), the level count grows by
one (log2(n+1) - 1 levels, coarsest grid 3 x 3) and the batch halves down to 2; Adam with
learning rate 3e-3, multiplied by 0.8 every 2 epochs.

Network: C hidden channels (8 by default, the paper's standard), Xavier-uniform weights, held in
the library's 16-channel layout with the extra channels at zero: their gradients are masked, so
they stay zero and the network stays the C-channel network.

    python -m paper_2312_11093_amd.train_t5 --out DIR [--channels 8] [--batches 1000]
           [--epochs 50] [--resume] [--minutes M]

The same schedule can train on the other coefficient families of this library (--data blocks:
16 x 16 random blocks with log10 a ~ U(-2, 2); --data mixture: blocks, lognormal fields,
checkerboards and inclusions in turn; both with random velocities |b| <= 10 and the divergence
form, full-depth networks), with K > 1 unrolled iterations (--K), and from given weights
(--init; --init-noise adds small random weights to channels the given network leaves at zero,
so that they can leave the zero saddle).

Writes DIR/weights_c{C}.npy (the compact C-channel vector), DIR/weights16.npy (the library
layout), DIR/ckpt.pt (weights, Adam and scheduler state, progress) and DIR/log.jsonl.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
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

# Appendix A.1, Table 5
TABLE5 = {"epochs": 50, "batches": 1000, "lr": 3e-3, "lr_step_epochs": 2, "gamma": 0.8,
          "size_step": 10, "size": 31, "level": 4, "batch_size": 16, "max_size": 511,
          "min_batch_size": 2}
RE = 1000.0                      # Sec. 4.1: range limit of the mesh Reynolds number
DATA_STREAM = 0x7A5               # seed-sequence tag of the training data
# operator form and network depth (opts.levels) of each training family
DATA_FORM = {"paper": ("nondiv", -1), "blocks": ("div", 0), "mixture": ("div", 0)}


def stage(epoch: int, t=TABLE5):
    """(n, levels, batch) of an epoch: sizes double and batches halve every size_step epochs."""
    s = epoch // t["size_step"]
    n = t["size"]
    lev = t["level"]
    B = t["batch_size"]
    for _ in range(s):
        if 2 * n + 1 > t["max_size"]:
            break
        n, lev = 2 * n + 1, lev + 1
        B = max(t["min_batch_size"], B // 2)
    return n, lev, B


def batch_data(n: int, B: int, seed: int, step: int, kind: str = "paper"):
    """Coefficients a (B, n, n), velocities b (B, 2), right-hand sides f (B, n, n) (float32) and
    the f64 squared norms of f for training step `step`.  "paper": white noise mapped onto coef
    in [1/Re, 1] and v = (sin 0.5, cos 0.5) (Sec. 4.1); "blocks" / "mixture": the library's
    families with random velocities.  Right-hand sides are white noise (Sec. 3.4)."""
    import datagen
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, DATA_STREAM, step])))
    a = np.empty((B, n, n), np.float32)
    b = np.empty((B, 2), np.float32)
    f = np.empty((B, n, n), np.float32)
    for i in range(B):
        if kind == "paper":
            a[i] = datagen.white_noise_coef(n, rng, RE)
            b[i] = datagen.velocity(rng, "paper")
        elif kind == "blocks":
            a[i] = datagen.blocks_lognormal(n, rng)
            b[i] = datagen.velocity(rng, "random")
        elif kind == "mixture":
            j = (step * B + i) % 4
            a[i] = datagen.blocks_lognormal(n, rng) if j == 0 else datagen.mixture(n, rng)
            b[i] = datagen.velocity(rng, "random")
        else:
            raise ValueError(kind)
        f[i] = rng.standard_normal((n, n))
    f2 = np.einsum("bij,bij->b", f.astype(np.float64), f.astype(np.float64))
    return a, b, f, f2


def channel_mask(C: int) -> np.ndarray:
    """1 at the entries of the 16-channel layout that belong to the C-channel network."""
    from paper_2312_11093_amd.weights import embed_channels
    return embed_channels(np.ones(81 * C * C + 58 * C, np.float32), C)


def compact(w16: np.ndarray, C: int) -> np.ndarray:
    """Inverse of embed_channels: the C-channel flat vector held in the 16-channel layout."""
    return np.asarray(w16, np.float32)[channel_mask(C) > 0]


def train(out: str, C: int = 8, epochs: int | None = None, batches: int | None = None,
          seed: int = 0, resume: bool = False, minutes: float = 1e9, log_every: int = 250,
          init: str | None = None, data: str = "paper", K: int = 1, init_noise: float = 0.0,
          lr: float | None = None):
    import torch

    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd.weights import embed_channels

    t = dict(TABLE5)
    if lr is not None:
        t["lr"] = float(lr)
    form, net_levels = DATA_FORM[data]
    if epochs is not None:
        t["epochs"] = int(epochs)
    if batches is not None:
        t["batches"] = int(batches)
    os.makedirs(out, exist_ok=True)
    ck_path = os.path.join(out, "ckpt.pt")
    t_end = time.time() + 60.0 * minutes
    mask = torch.tensor(channel_mask(C), device="cuda")
    if init:
        w0 = embed_channels(np.load(init, allow_pickle=False).astype(np.float32))
        if init_noise > 0:
            # small random weights where the given network is zero but the C-channel one is not
            xav = embed_channels(datagen.xavier_weights(C, seed + 1), C)
            w0 = np.where(w0 == 0, init_noise * xav, w0).astype(np.float32)
        w0 = w0 * channel_mask(C)
    else:
        w0 = embed_channels(datagen.xavier_weights(C, seed), C)
    w = torch.tensor(w0, device="cuda")
    opt = torch.optim.Adam([w], lr=t["lr"])
    sched = torch.optim.lr_scheduler.StepLR(opt, step_size=t["lr_step_epochs"] * t["batches"],
                                            gamma=t["gamma"])
    step = 0
    if resume and os.path.exists(ck_path):
        ck = torch.load(ck_path, weights_only=True, map_location="cuda")
        w.copy_(ck["w"])
        opt.load_state_dict(ck["opt"])
        sched.load_state_dict(ck["sched"])
        step = int(ck["step"])
    total = t["epochs"] * t["batches"]
    logf = open(os.path.join(out, "log.jsonl"), "a")
    solvers = {}
    pool = cf.ThreadPoolExecutor(max_workers=2)

    def job(s):
        n, lev, B = stage(s // t["batches"], t)
        return s, n, lev, B, batch_data(n, B, seed, s, data)

    pending = pool.submit(job, step) if step < total else None
    skipped = 0
    acc, cnt = 0.0, 0
    t0 = time.time()
    while pending is not None:
        s, n, lev, B, (a_h, bv, f_h, f2) = pending.result()
        pending = pool.submit(job, s + 1) if s + 1 < total else None
        key = (n, B)
        if key not in solvers:
            for S_old in solvers.values():
                S_old.close()
            solvers = {key: Solver(w0, state="f32", u="f32", form=form, levels=net_levels)}
            u = torch.zeros((B, n, n), device="cuda")
            du = torch.empty_like(u)
        S = solvers[key]
        a = torch.from_numpy(a_h).cuda(non_blocking=False)
        f = torch.from_numpy(f_h).cuda(non_blocking=False)
        S.set_weights_device(w)
        S.setup(a, bv)
        u.zero_()
        S.forward(f, u, K, record=True)
        log_now = (s + 1) % log_every == 0 or s + 1 == total
        rel = S.loss(f, u, du)                      # mean_i ||r_i||^2 / ||f_i||^2
        # absolute loss of Eq. (19) per grid node: (1/B) sum_i ||r_i||^2 / n^2; its gradient is
        # the library's relative-loss gradient times ||f_i||^2 / n^2 per problem
        scale = torch.from_numpy((f2 / (n * n)).astype(np.float32)).cuda().view(B, 1, 1)
        du.mul_(scale)
        g = S.backward(du)
        g.mul_(mask)
        ok = math.isfinite(rel) and bool(torch.isfinite(g).all())
        if ok:
            w.grad = g
            opt.step()
            opt.zero_grad(set_to_none=True)
            acc += rel
            cnt += 1
        else:
            skipped += 1
        sched.step()
        step = s + 1
        if log_now or time.time() > t_end:
            rec = {"step": step, "epoch": s // t["batches"], "n": n, "levels": lev if data == "paper"
                   else int(math.log2(n + 1)), "batch": B, "K": K, "data": data,
                   "relres2_mean": acc / max(cnt, 1), "lr": opt.param_groups[0]["lr"],
                   "skipped": skipped, "sec": round(time.time() - t0, 1)}
            print(json.dumps(rec), flush=True)
            logf.write(json.dumps(rec) + "\n")
            logf.flush()
            acc, cnt = 0.0, 0
        if step % (2 * t["batches"]) == 0 or step == total or time.time() > t_end:
            torch.save({"w": w.detach(), "opt": opt.state_dict(), "sched": sched.state_dict(),
                        "step": torch.tensor(step)}, ck_path)
            w16 = w.detach().cpu().numpy().astype(np.float32)
            np.save(os.path.join(out, "weights16.npy"), w16)
            np.save(os.path.join(out, f"weights_c{C}.npy"), compact(w16, C))
        if time.time() > t_end:
            break
    pool.shutdown(wait=False, cancel_futures=True)
    for S_old in solvers.values():
        S_old.close()
    logf.close()
    print(json.dumps({"finished": step >= total, "step": step, "out": out}), flush=True)
    return step >= total


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--channels", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=None)
    ap.add_argument("--batches", type=int, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--resume", action="store_true")
    ap.add_argument("--minutes", type=float, default=1e9)
    ap.add_argument("--log-every", type=int, default=250)
    ap.add_argument("--init", default=None)
    ap.add_argument("--init-noise", type=float, default=0.0)
    ap.add_argument("--data", default="paper", choices=sorted(DATA_FORM))
    ap.add_argument("--K", type=int, default=1)
    ap.add_argument("--lr", type=float, default=None)
    args = ap.parse_args()
    train(args.out, args.channels, args.epochs, args.batches, args.seed, args.resume, args.minutes,
          args.log_every, args.init, args.data, args.K, args.init_noise, args.lr)


if __name__ == "__main__":
    main()
