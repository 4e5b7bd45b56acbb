"""Tile-shape autotuner for the 16 -> 16 convolutions (the library's mgcnn_set_tile_variant).

Every tile variant differs only in the output rows per workgroup, so all give the same results
bit for bit; which is fastest depends on the level side (occupancy against halo overhead and the
number of workgroups).  For a workload (default: 64 problems at 1023 x 1023 with random block
coefficients, f32 state, the benchmark's setting), each variant is applied to every level and
timed per operation and level side with the library's per-launch HIP events over profiled
fixed-K iterations (every launch over all problems).  The fastest variant per (operation,
storage, level side) is stored in a JSON file keyed by the device architecture; `load` fills the
library's table from it.

    python -m paper_2312_11093_amd.autotune --out paper_2312_11093_amd/tuning/gfx950.json [--state f32]

Operations tuned: the smoothers (down smoother on the coarser levels and up smoother on every
level share one table), the restriction, the finest down smoother (reChannel-in folded in) and the
prolongation (keyed by its fine side).  The setup network keeps its tiles.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

OPS = {"smoother": 0, "restrict": 1, "setup": 2, "smooth_in": 3, "prolong": 4}
VARIANTS = 5          # the same-size convs and the finest down smoother; restriction and prolongation 3
STATES = {"f32": 0, "bf16": 1}
# profiled kernel kinds -> tuned operation (level 0 of the down smoother is the separate
# reChannel-in kernel)
KIND_OP = {"smooth_down": "smoother", "smooth_up": "smoother", "restrict": "restrict",
           "smooth_in": "smooth_in", "prolong": "prolong"}
TUNED = ("smoother", "restrict", "smooth_in", "prolong")
DEFAULT_FILE = os.path.join(HERE, "tuning", "gfx950.json")


def device_arch() -> str:
    import torch
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def has_variant(L, op: str, state: str, variant: int) -> bool:
    return L.mgcnn_tile_rows(OPS[op], STATES[state], variant) > 0


def set_all(L, op: str, state: str, variant: int):
    for p in range(1, 13):
        st = L.mgcnn_set_tile_variant(OPS[op], STATES[state], (1 << p) - 1, variant)
        if st != 0:
            raise RuntimeError(f"mgcnn_set_tile_variant failed ({st})")


def tune(n: int = 1023, batch: int = 64, state: str = "f32", workload: str = "blocks1023", K: int = 2,
         reps: int = 2, log=print):
    import torch

    import datagen
    from paper_2312_11093_amd import Solver
    from paper_2312_11093_amd import mgcnn as M
    from paper_2312_11093_amd.handbuilt import vcycle_weights
    L = M.lib()
    a, b, f = datagen.make_batch(workload, n, batch, seed=0)
    S = Solver(vcycle_weights(), state=state, u="f64", f32_split=2 if state == "f32" else True)
    S.setup(torch.from_numpy(a).cuda(), b)
    df = torch.from_numpy(f).cuda()
    u = torch.zeros((batch, n, n), dtype=torch.float64, device="cuda")
    sides = []
    m = n
    while m >= 1:
        sides.append(m)
        m = (m - 1) // 2
    times = {}                                        # (op, side, variant) -> ms per launch
    for v in range(VARIANTS):
        ops_v = [op for op in TUNED if has_variant(L, op, state, v)]
        for op in TUNED:
            set_all(L, op, state, v if op in ops_v else 0)
        S.forward(df, u, 1)                           # warm-up of this variant's kernels
        best = {}
        for _ in range(reps):
            u.zero_()
            S.profile_begin()
            S.forward(df, u, K)
            for st in S.profile_end():
                op = KIND_OP.get(st["kind"])
                if op is None or op not in ops_v or (st["kind"] == "smooth_down" and st["level"] == 0):
                    continue
                # the prolongation into level l is keyed by that level's (fine) side
                key = (op, sides[st["level"]])
                per = st["ms_total"] / st["launches"]
                best.setdefault(key, []).append(per)
        for (op, side), vals in best.items():
            times[(op, side, v)] = float(np.min(vals))
        log(json.dumps({"variant": v, "rows": {op: L.mgcnn_tile_rows(OPS[op], STATES[state], v)
                                               for op in ops_v},
                        "ms": {f"{op}@{side}": round(times[(op, side, v)], 4)
                               for (op, side, vv) in times if vv == v}}))
    S.close()
    for op in TUNED:
        set_all(L, op, state, 0)
    entries = []
    for op in TUNED:
        for side in sides:
            cand = [(times[(op, side, v)], v) for v in range(VARIANTS) if (op, side, v) in times]
            if not cand:
                continue
            t0 = times.get((op, side, 0))
            tbest, vbest = min(cand)
            # keep the default unless another variant is faster by more than 2 %
            if t0 is not None and tbest > 0.98 * t0:
                tbest, vbest = t0, 0
            entries.append({"op": op, "state": state, "side": side, "variant": vbest,
                            "rows": L.mgcnn_tile_rows(OPS[op], STATES[state], vbest),
                            "ms": round(tbest, 4), "ms_default": round(t0, 4) if t0 else None})
    return entries


def save(entries, path: str, arch: str, workload: str):
    data = {}
    if os.path.exists(path):
        with open(path) as fh:
            data = json.load(fh)
    if data.get("arch") not in (None, arch):
        data = {}
    data["arch"] = arch
    keep = [e for e in data.get("entries", []) if e["state"] not in {x["state"] for x in entries}]
    data["entries"] = keep + entries
    states = sorted({e["state"] for e in data["entries"]})
    data["how"] = ("per-launch HIP events over profiled fixed-K iterations of " + workload +
                   f" (states tuned: {', '.join(states)}); fastest variant per (op, state, side), the "
                   "default unless another is 2 % faster")
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as fh:
        json.dump(data, fh, indent=1)


def load(path: str = DEFAULT_FILE, arch: str | None = None) -> int:
    """Fill the library's tile-variant table from a tuning file; returns the number of entries
    applied (0 if the file is missing or was tuned on another architecture)."""
    from paper_2312_11093_amd import mgcnn as M
    if not os.path.exists(path):
        return 0
    with open(path) as fh:
        data = json.load(fh)
    arch = arch or device_arch()
    if data.get("arch") != arch:
        return 0
    L = M.lib()
    count = 0
    for e in data.get("entries", []):
        if L.mgcnn_set_tile_variant(OPS[e["op"]], STATES[e["state"]], int(e["side"]), int(e["variant"])) == 0:
            count += 1
    return count


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_FILE)
    ap.add_argument("--state", default="f32", choices=sorted(STATES))
    ap.add_argument("--n", type=int, default=1023)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--workload", default="blocks1023")
    args = ap.parse_args()
    t0 = time.time()
    entries = tune(args.n, args.batch, args.state, args.workload)
    arch = device_arch()
    save(entries, args.out, arch, f"{args.workload} {args.batch} x {args.n}^2")
    print(json.dumps({"saved": args.out, "arch": arch, "entries": len(entries),
                      "changed": [e for e in entries if e["variant"] != 0], "sec": round(time.time() - t0, 1)}))


if __name__ == "__main__":
    main()
