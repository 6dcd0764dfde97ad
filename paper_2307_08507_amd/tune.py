"""Offline tuner of the sweep kernel's launch variants; writes tuning.json beside this file.

The variants compute the same values bit for bit (the tuner checks it on every measurement) and
differ only in speed:
  * point costs (squared Euclidean or L1, planar or d = 3): the sweep instance capped at 4 waves
    per SIMD (128 VGPRs, its Round paths spill) or at 2 (up to 256 VGPRs, no spills);
  * dense FP32 costs: the second batch of each wave's cost rows loaded straight into LDS, or into
    registers after the first batch.
For each cost type and size the tuner times a short solve of the paper's schedule (gamma_f = 2^8,
FP32 sweeps; the device time the library reports, best of three after a warm-up) under every
variant, and keeps the fastest; a variant must beat the default by more than 1 % to replace it.
Each measured size covers the sizes up to the geometric mean with the next one. The library
reads the file when a context is created (include/mdot.h, "Launch-variant tuning").

Run on the GPU:  python -m paper_2307_08507_amd.tune [--out FILE] [--quick]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tuning.json")
STAGE_DEFAULT = 2048  # the library's built-in staging threshold (tiles)
MAX_N = 131072  # MDOT_MAX_N of include/mdot.h


def _problem(code: str, n: int, dev):
    """(descriptor, r, c, kept tensors) of a grid workload of size n for cost type `code`."""
    import numpy as np
    import torch

    from . import mdot as M
    from . import workloads as W

    k = int(round(math.sqrt(n)))
    assert k * k == n
    r = torch.tensor(W.grid_problem_marginals(k, "smooth", 11), dtype=torch.float64, device=dev)
    c = torch.tensor(W.grid_problem_marginals(k, "smooth", 12), dtype=torch.float64, device=dev)
    X = W.grid_coords(k).astype(np.float64)
    kind = "sqeuclid" if code in ("f32", "pts_sq", "pts_sq2") else "l1"
    mx = 2.0 * (k - 1) ** 2 if kind == "sqeuclid" else 2.0 * (k - 1)
    if code == "f32":
        Xd = torch.tensor(X, device=dev)
        C = torch.empty((n, n), dtype=torch.float32, device=dev)
        for a in range(0, n, 1024):
            d = Xd[a:a + 1024, None, :] - Xd[None, :, :]
            C[a:a + 1024] = ((d * d).sum(-1) / mx).float()
        return M.dense_cost(C), r, c, (C,)
    d = 2 if code.endswith("2") else 3
    if d == 3:  # the grid lifted onto a tilted plane in 3-D: a genuine d = 3 cloud of the same shape
        X = np.concatenate([X, 0.25 * X[:, :1]], axis=1)
        mx = None
    XY = torch.tensor(np.concatenate([X, X]), dtype=torch.float32, device=dev).contiguous()
    desc = M.point_cost(XY, n, d, kind, scale=0.0 if mx is None else 1.0 / mx)
    return desc, r, c, (XY,)


def _time(ctx, desc, r, c, reps: int = 3):
    import torch

    from . import mdot as M

    prm = M.default_params(gamma_f=2.0**8)
    u = torch.empty(r.numel(), dtype=torch.float64, device=r.device)
    v = torch.empty_like(u)
    ctx.solve(desc, r, c, 1e-4, prm, u, v)  # warm-up (graph capture, caches)
    best, ref = math.inf, None
    for _ in range(reps):
        res = ctx.solve(desc, r, c, 1e-4, prm, u, v)
        best = min(best, res.seconds)
        ref = (res.primal_cost, res.dual_bound, res.sweeps, bytes(u.cpu().numpy().tobytes()))
    return best, ref


def tune(sizes_dense, sizes_points, codes_points, log=print):
    import torch

    from . import mdot as M

    dev = torch.device("cuda", 0)
    ctx = M.Context(0)
    entries = []
    plan = [("f32", sizes_dense, [("stage", 0), ("stage", 1)])]
    plan += [(cd, sizes_points, [("occ", 4), ("occ", 2)]) for cd in codes_points]
    for code, sizes, variants in plan:
        for i, n in enumerate(sizes):
            desc, r, c, keep = _problem(code, n, dev)
            times, refs = {}, {}
            for knob, val in variants:
                ctx.tune_override(occ=val if knob == "occ" else 0, stage=val if knob == "stage" else -1)
                times[f"{knob}{val}"], refs[f"{knob}{val}"] = _time(ctx, desc, r, c)
            ctx.tune_override(0, -1)
            if len(set(refs.values())) != 1:
                raise RuntimeError(f"{code} n={n}: launch variants gave different results")
            if code == "f32":
                tiles = ((n + 63) // 64) * ((n + 255) // 256)
                default = "stage1" if tiles > STAGE_DEFAULT else "stage0"
            else:
                default = "occ4"
            best = min(times, key=times.get)
            choice = best if times[best] < 0.99 * times[default] else default
            n_max = MAX_N if i + 1 == len(sizes) else int(math.sqrt(n * sizes[i + 1]))
            e = {"code": code, "n_max": n_max, "occ": 4, "stage_min_tiles": STAGE_DEFAULT}
            if code == "f32":
                e["stage_min_tiles"] = 0 if choice == "stage1" else 0x7FFFFFFF
            else:
                e["occ"] = int(choice[3:])
            e["measured_at_n"] = n
            e["solve_device_s"] = {k: round(t, 6) for k, t in sorted(times.items())}
            e["default"] = default
            entries.append(e)
            log(f"{code} n={n}: " + ", ".join(f"{k} {t * 1e3:.2f} ms" for k, t in sorted(times.items()))
                + f" -> {choice} (default {default})")
            del keep
    ctx.close()
    return entries


def write(entries, path):
    """One JSON object per line inside a list, in (code, n_max) order: the library reads it line by line."""
    order = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "pts_sq": 4, "pts_l1": 5, "pts_sq2": 6, "pts_l12": 7}
    entries = sorted(entries, key=lambda e: (order[e["code"]], e["n_max"]))
    with open(path, "w") as f:
        f.write("[\n")
        for k, e in enumerate(entries):
            f.write("  " + json.dumps(e, sort_keys=False) + ("," if k + 1 < len(entries) else "") + "\n")
        f.write("]\n")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="fewer sizes (a smoke run of the tuner)")
    args = ap.parse_args()
    if args.quick:
        dense, pts = [1024, 4096], [1024, 4096]
    else:
        dense, pts = [1024, 4096, 9216, 16384], [1024, 4096, 16384, 65536]
    entries = tune(dense, pts, ["pts_sq", "pts_l1", "pts_sq2", "pts_l12"],
                   log=lambda s: print(s, file=sys.stderr, flush=True))
    write(entries, args.out)
    print(args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
