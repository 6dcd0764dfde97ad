#!/usr/bin/env python3
"""Benchmark of the MDOT-PNCG hot path on one MI355X.

Workload (one "step" = one complete solve): n = 4096 OT problems on a 64 x 64 grid with the
cost stored in FP32 (squared-Euclidean and L1 pixel distances divided by their maximum),
marginals from four synthetic families (uniform-random pixels, Gaussian-smoothed random
fields, sums of Gaussian blobs, heavy-tailed Cauchy blobs), each solved from scratch to a
certified optimality gap of 1e-6 (rounded plan cost minus a c-transform lower bound). The
paper benchmarks upsampled MNIST and DOTmark images of the same size and costs; those are not
available here and these seeded families stand in for them.

Prints ONE JSON line. `value` is the mean time-to-gap per solve in seconds (lower is better),
measured over `--steps` solves after `--warmup` solves, inputs resident in HBM, bracketed by
torch.cuda.synchronize(). `roofline` reports the dominant kernel (the fused LSE sweep) timed
with HIP events on the library stream; `cpu_baseline` times the FP64 CPU oracle on a bounded
sample of the same workload and extrapolates to a full solve.

The default run (no workload flags) adds, beside the headline, the rest of the metric:
  lse_sweep_flushed      the sweep timed alone after a 512 MiB read evicts the cost from the
                         L2 and last-level caches (HBM-streamed, against the MALL-resident
                         figure of `roofline`)
  legs.f64 / legs.mixed  the same 8 problems solved once each in FP64 and in MIXED precision
  legs.batched_*         the 8 problems submitted together to the batched engine (FP32, MIXED)
  legs.projectors        PNCG against the Sinkhorn projector (Alg. 4) at fixed gamma_f on the
                         L1 problems: LSE sweeps per solve
  legs.serving           a short continuous-batching run (--leg-requests requests, Poisson
                         arrivals at 0.7 x saturation, HBM admission budget --hbm-budget);
                         tail_request: the slowest request, its latency against its own
                         solve time alone
  legs.precision_modes   the 8 problems in every precision mode against FP64 on the exact
                         cost (as --workload precision, summarised per mode)
--no-legs reports the headline alone.

Other workloads (not the default line):
  --problems 64          the full grid problem set: 8 marginal pairs of each family and cost
                         (reports mean, median, p90 and max time to gap over the problems)
  --family F             draw marginals from family F only (repeatable)
  --workload precision   every grid problem in each precision mode (FP64 on the exact cost as the
                         reference, FP32, FP16/BF16 storage, recomputed point cost, MIXED): per
                         result the relative UB difference, gap, marginal error and gamma_final
  --grid 128             n = 16384 on a 128 x 128 grid (the cost is 1 GiB in FP32)
  --cost-storage S       f32 (default), f16, bf16 (stored dense cost) or points (the cost is
                         recomputed in registers from FP32 grid coordinates, in FP64)
  --workload serving     continuous batching: Poisson arrivals of point-cloud OT requests
                         (n log-uniform in [512, 8192], d = 3, target gap in {1e-4 .. 1e-7});
                         reports throughput and p50 / p99 latency at 0.7x the measured
                         saturation rate
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# ALU roofline of the point-cost sweep (the cost is recomputed, nothing streams from HBM): the
# chip issues 256 CUs x 4 SIMDs x 16 lanes of VALU work per clock at 2.4 GHz. The peak takes the
# least work one element needs in this formulation, in lane-slots: d FP64 FMAs and one FP64 add
# (the argument, with |x|^2 and |y|^2 folded into the row and column terms), one FP64->FP32
# conversion, one v_exp_f32 at quarter rate (4 slots), one FP32 add (row sum) and one FP32 FMA
# (column sum): 8 + d. The compiled loop issues about 12.2 slots per element for d <= 2 and 13.5
# for d = 3 (per-row coordinate work, accumulator flushes, addressing).
VALU_LANE_SLOTS_PER_S = 256 * 4 * 16 * 2.4e9


POINT_DIM = 2  # grid workloads recompute the cost from 2-D pixel coordinates


def points_alu_peak_gexps(d: int) -> float:
    return VALU_LANE_SLOTS_PER_S / (8 + d) / 1e9


FAMILIES = ("uniform", "smooth", "blobs", "cauchy")
COSTS = ("sqeuclid", "l1")
BYTES = {"f32": 4, "f16": 2, "bf16": 2, "f64": 8}


def build_problems(k: int, count: int, families=FAMILIES):
    """Up to 8 marginal pairs per (family, cost): pair j of family fi and cost ci draws r and c with
    seeds 1000 (fi + 1) + 10 ci + 100 j and that + 1. Pairs are taken j-major, so the first
    len(families) x 2 problems are pair 0 of every (family, cost), and count = 64 over all four
    families is the full grid problem set."""
    from paper_2307_08507_amd import workloads as W

    probs = []
    for j in range(8):
        for fi, fam in enumerate(FAMILIES):
            if fam not in families:
                continue
            for ci, cost in enumerate(COSTS):
                if len(probs) < count:
                    seed = 1000 * (fi + 1) + 10 * ci + 100 * j
                    probs.append({"family": fam, "cost": cost, "seed": seed,
                                  "name": f"{fam}/{cost}" + (f"#{j}" if j else ""),
                                  "r": W.grid_problem_marginals(k, fam, seed),
                                  "c": W.grid_problem_marginals(k, fam, seed + 1)})
    return probs


def problem_set(args):
    return build_problems(args.grid, args.problems, tuple(args.family) if args.family else FAMILIES)


def grid_cost_device(k: int, kind: str, storage: str, dev):
    """The normalised grid cost on the device: (descriptor maker, FP64 host copy maker).
    Integer numerators are exact in FP64; num / max is rounded once, as in the generator."""
    import torch

    from paper_2307_08507_amd import mdot as M
    from paper_2307_08507_amd import workloads as W

    X = torch.tensor(W.grid_coords(k), dtype=torch.float64, device=dev)
    mx = 2.0 * (k - 1) ** 2 if kind == "sqeuclid" else 2.0 * (k - 1)
    if storage == "points":
        XY = torch.cat([X, X]).float().contiguous()
        n = k * k
        return {"desc": lambda: M.point_cost(XY, n, POINT_DIM, kind, scale=1.0 / mx), "keep": XY,
                "host64": lambda: _grid_num(X, kind).div_(mx).cpu().numpy()}
    dt = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16, "f64": torch.float64}[storage]
    C = _grid_num(X, kind).div_(mx).to(dt).contiguous()
    return {"desc": lambda: M.dense_cost(C), "keep": C, "host64": lambda: C.double().cpu().numpy()}


def _grid_num(X, kind):
    import torch

    n = X.shape[0]
    out = torch.empty((n, n), dtype=torch.float64, device=X.device)
    step = 2048
    for a in range(0, n, step):
        d = X[a:a + step, None, :] - X[None, :, :]
        out[a:a + step] = (d * d).sum(-1) if kind == "sqeuclid" else d.abs().sum(-1)
    return out


def measured_traffic(n: int, storage: str):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary, if it was taken
    on this workload with the current kernel source (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"k_sweep_n{n}_{storage}_hbm_traffic.md")
    src = os.path.join(ROOT, "paper_2307_08507_amd", "csrc", "mdot_kernels.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith((" ", "|", "#")):
            k, _, v = line.partition(":")
            fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != hashlib.sha256(open(src, "rb").read()).hexdigest():
        return None
    return int(fields["traffic_bytes_per_launch"])


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(C64, probs, gpu_counts, n_sweeps_sample: int, n_cert_sample: int, label: str):
    """Time the FP64 CPU oracle on a bounded sample (two-sided LSE sweeps and round+certify
    evaluations on one problem's cost) with all host threads and with one, and extrapolate to
    each problem's full solve from the GPU solve's sweep and certified-stage counts (the oracle
    takes the same decisions; its per-sweep cost does not depend on the marginals)."""
    import numpy as np

    from oracle import oracle as O

    p0 = probs[0]
    r, c = p0["r"], p0["c"]
    u, v = np.log(r), np.log(c)

    def sample(ns, nc):
        t0 = time.perf_counter()
        for k in range(ns):
            O.lse2(C64, u, v, 16.0 * 2 ** (k / 3))
        t_sweep = (time.perf_counter() - t0) / ns
        t0 = time.perf_counter()
        for k in range(nc):
            O.round_certify(C64, u, v, 64.0, r, c, u_prev=0.9 * u, v_prev=0.9 * v, gamma_prev=50.0)
        return t_sweep, (time.perf_counter() - t0) / nc

    threads = O.num_threads()
    t_sweep, t_cert = sample(n_sweeps_sample, n_cert_sample)
    O.set_num_threads(1)
    try:
        t_sweep1, t_cert1 = sample(max(2, n_sweeps_sample // 5), 1)
    finally:
        O.set_num_threads(0)
    per = [sw * t_sweep + st * t_cert for sw, st in gpu_counts]
    per1 = [sw * t_sweep1 + st * t_cert1 for sw, st in gpu_counts]
    return {
        "value": round(statistics.mean(per), 3),
        "unit": "s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"FP64 C oracle (gcc -O3 -march=x86-64-v3, OpenMP over rows/columns) on {label} (n={r.size}): "
                   f"{n_sweeps_sample} two-sided LSE sweeps ({t_sweep:.4f} s each) and {n_cert_sample} round+certify "
                   f"evaluations ({t_cert:.3f} s each) on {threads} threads, extrapolated to each of the "
                   f"{len(per)} problems' sweep and certified-stage counts; value = mean over the problems"),
        "cpu_model": _cpu_model(),
        "per_problem_s": [round(x, 2) for x in per],
        "one_thread": {"value": round(statistics.mean(per1), 3), "unit": "s", "cores": 1,
                       "sweep_s": round(t_sweep1, 4), "round_certify_s": round(t_cert1, 3)},
    }


def bench_grid(args) -> dict:
    import torch

    from paper_2307_08507_amd import mdot as M

    dev = torch.device("cuda", 0)
    # reference for hardware byte counters in profiling runs of this command: one plain
    # device-to-device copy of 64 MiB (64 MiB read, 64 MiB written)
    ref = torch.empty(16 << 20, dtype=torch.float32, device=dev)
    torch.empty_like(ref).copy_(ref)
    del ref
    k = args.grid
    n = k * k
    probs = problem_set(args)
    costs = {kind: grid_cost_device(k, kind, args.cost_storage, dev) for kind in {p["cost"] for p in probs}}
    for p in probs:
        p["rd"] = torch.tensor(p["r"], dtype=torch.float64, device=dev)
        p["cd"] = torch.tensor(p["c"], dtype=torch.float64, device=dev)
    ctx = M.Context(0)
    prm = M.default_params(precision=args.precision)
    u = torch.empty(n, dtype=torch.float64, device=dev)
    v = torch.empty_like(u)

    def solve(p):
        return ctx.solve(costs[p["cost"]]["desc"](), p["rd"], p["cd"], args.target, prm, u, v)

    for i in range(args.warmup):
        solve(probs[i % len(probs)])
    torch.cuda.synchronize()
    results, step_times = [], []
    per_prob = [[] for _ in probs]
    for i in range(args.steps):
        t0 = time.perf_counter()
        res = solve(probs[i % len(probs)])
        torch.cuda.synchronize()
        step_times.append(time.perf_counter() - t0)
        per_prob[i % len(probs)].append(step_times[-1])
        results.append(res)
    torch.cuda.synchronize()
    # each problem's runs are averaged first, so steps that are not a multiple of the problem
    # count do not weight some problems more than others
    prob_means = [statistics.mean(t) for t in per_prob if t]
    mean_s = statistics.mean(prob_means)
    # FP16/BF16 storage certifies the gap of the stored cost. Every plan's cost differs by at most
    # delta = max |C_stored - C_exact| between the stored and the exact FP64 cost (total mass 1),
    # so the returned plan is within gap + 2 delta of the exact problem's optimum.
    error_vs_exact = None
    if args.cost_storage in ("f16", "bf16"):
        delta = {}
        for kind, cd in costs.items():
            exact = grid_cost_device(k, kind, "f64", dev)["keep"]
            delta[kind] = float((cd["keep"].double() - exact).abs().max())
            del exact
        error_vs_exact = [{"problem": probs[i % len(probs)]["name"],
                           "certified_gap_stored_cost": res.gap, "delta": delta[probs[i % len(probs)]["cost"]],
                           "error_bound_exact_cost": res.gap + 2.0 * delta[probs[i % len(probs)]["cost"]]}
                          for i, res in enumerate(results)]

    # roofline of the dominant kernel: the fused LSE sweep at the first problem's solution
    p0 = probs[0]
    r0 = solve(p0)
    sweep_prec = "f64" if args.precision == "f64" else "f32"  # MIXED finishes on the exact cost in F32
    ms = ctx.bench_sweep(costs[p0["cost"]]["desc"](), u, v, r0.gamma_final, precision=sweep_prec, iters=200)
    if args.cost_storage == "points":
        bound, unit, peak = "alu", "Gexp/s", round(points_alu_peak_gexps(POINT_DIM), 1)
        achieved = n * n / (ms * 1e-3) / 1e9
        per_launch = {"elements_per_launch": n * n}
    else:
        bound, unit, peak = "hbm", "GB/s", HBM_PEAK_GBPS
        per_launch = {"bytes_per_launch": n * n * BYTES[args.cost_storage]}
        achieved = per_launch["bytes_per_launch"] / (ms * 1e-3) / 1e9
    roof = {"bound": bound, "achieved": round(achieved, 1), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 4) if peak else None,
            "traffic": measured_traffic(n, args.cost_storage) if sweep_prec == "f32" else None,
            "kernel": "k_sweep (fused two-sided LSE sweep)", **per_launch}
    out = {
        "metric": f"time-to-gap {args.target:g} at n={n}",
        "value": round(mean_s, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mean_s * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": (f"n={n} ({k}x{k} grid), {args.cost_storage} cost, {'/'.join(sorted(costs))} x "
                         f"{{{', '.join(sorted({p['family'] for p in probs}))}}} marginals, certified gap "
                         f"{args.target:g}"),
            "n": n,
            "target_gap": args.target,
            "problems": len(probs),
            "cost_storage": args.cost_storage,
        },
        "time_to_gap_per_problem_s": {p["name"]: round(statistics.mean(t), 6)
                                      for p, t in zip(probs, per_prob) if t},
        "time_to_gap_median_s": round(statistics.median(prob_means), 6),
        "time_to_gap_p90_s": round(sorted(prob_means)[min(len(prob_means) - 1, int(0.9 * len(prob_means)))], 6),
        "time_to_gap_max_s": round(max(prob_means), 6),
        "certified_gap_max": max(r.gap for r in results),
        "all_certified": all(r.status == 0 and r.gap <= args.target for r in results),
        "sweeps_mean": statistics.mean(r.sweeps for r in results),
        "proxy_stages_mean": statistics.mean(r.proxy_stages for r in results),
        "fp64_stage_switches": sum(r.prec_switches for r in results),
        "us_per_sweep_in_solve": round(1e6 * sum(step_times) / sum(r.sweeps for r in results), 2),
        "lse_sweep_us": round(ms * 1e3, 3),
        "roofline": roof,
    }
    if error_vs_exact is not None:
        out["error_vs_exact_cost"] = error_vs_exact
        out["error_bound_exact_cost_max"] = max(e["error_bound_exact_cost"] for e in error_vs_exact)
    if args.legs and args.cost_storage == "f32" and args.precision == "f32":
        out["lse_sweep_flushed"] = flushed_sweep(ctx, costs[p0["cost"]]["desc"](), u, v, r0.gamma_final, n,
                                                 BYTES[args.cost_storage])
    if not args.no_cpu_baseline:
        big = n > 8192
        counts = []
        for i, p in enumerate(probs):
            rs = [r for j, r in enumerate(results) if j % len(probs) == i]
            if rs:
                counts.append((rs[0].sweeps, rs[0].stages))
        out["cpu_baseline"] = cpu_baseline(costs[p0["cost"]]["host64"](), probs, counts,
                                           n_sweeps_sample=6 if big else 20, n_cert_sample=1 if big else 3,
                                           label=f"the first problem's cost ({p0['cost']})")
    ctx.close()
    return out


def flushed_sweep(ctx, desc, u, v, gamma, n, nbytes):
    """The LSE sweep timed alone after a 512 MiB read evicts the cost from the L2s and the 256 MB
    last-level cache: every sweep streams the whole matrix from HBM."""
    import torch

    flush = torch.ones(64 << 20, dtype=torch.float64, device=u.device)  # 512 MiB
    ms = ctx.bench_sweep_flushed(desc, u, v, gamma, flush, precision="f32", iters=40)
    del flush
    achieved = n * n * nbytes / (ms * 1e-3) / 1e9
    return {"us": round(ms * 1e3, 3), "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "bytes_per_launch": n * n * nbytes,
            "note": "each sweep timed alone (HIP events) after a 512 MiB read evicts the cost from L2 and MALL"}


def bench_grid_batched(args) -> dict:
    """The grid workload through the batched engine: each timed step submits the --problems
    problems together and runs them to their certified gaps. `value` = wall time of a batch /
    problems (the batched form's time-to-gap per solve); per-problem completion latencies within
    the batch are reported beside it."""
    import torch

    from paper_2307_08507_amd import mdot as M

    dev = torch.device("cuda", 0)
    k = args.grid
    n = k * k
    probs = problem_set(args)
    costs = {kind: grid_cost_device(k, kind, args.cost_storage, dev) for kind in {p["cost"] for p in probs}}
    for p in probs:
        p["rd"] = torch.tensor(p["r"], dtype=torch.float64, device=dev)
        p["cd"] = torch.tensor(p["c"], dtype=torch.float64, device=dev)
        p["u"] = torch.empty(n, dtype=torch.float64, device=dev)
        p["v"] = torch.empty_like(p["u"])
    prm = M.default_params(precision=args.precision)
    eng = M.Context(0)

    def batch():
        t0 = time.perf_counter()
        res, lat = [None] * len(probs), [0.0] * len(probs)
        tickets = {}
        for i, p in enumerate(probs):
            t = eng.submit(costs[p["cost"]]["desc"](), p["rd"], p["cd"], args.target, prm, p["u"], p["v"])
            if t is None:
                raise RuntimeError("the engine did not admit the whole batch")
            tickets[i] = t
        while tickets:
            eng.run(8)
            for i, t in list(tickets.items()):
                r = eng.poll(t)
                if r is not None:
                    res[i] = r
                    lat[i] = time.perf_counter() - t0
                    del tickets[i]
        torch.cuda.synchronize()
        return time.perf_counter() - t0, res, lat

    for _ in range(args.warmup):
        batch()
    walls, results, lats = [], [], []
    for _ in range(args.steps):
        w, rs, ls = batch()
        walls.append(w)
        results += rs
        lats += ls
    mean_wall = statistics.mean(walls)
    # one problem solved alone must give the same result bit for bit
    ctx = M.Context(0)
    p0 = probs[0]
    u0 = torch.empty_like(p0["u"])
    alone = ctx.solve(costs[p0["cost"]]["desc"](), p0["rd"], p0["cd"], args.target, prm, u0, torch.empty_like(u0))
    same = alone.primal_cost == results[0].primal_cost and alone.sweeps == results[0].sweeps and bool(
        torch.equal(u0, p0["u"]))
    lats.sort()
    return {
        "metric": f"time-to-gap {args.target:g} at n={n}, batched",
        "value": round(mean_wall / len(probs), 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mean_wall * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {
            "workload": (f"n={n} ({k}x{k} grid), {args.cost_storage} cost, {len(probs)} problems "
                         f"({'/'.join(sorted(costs))} x {{{', '.join(sorted({p['family'] for p in probs}))}}} "
                         f"marginals) submitted together to the batched engine, certified gap {args.target:g}"),
            "n": n,
            "target_gap": args.target,
            "problems": len(probs),
            "cost_storage": args.cost_storage,
        },
        "batch_wall_s": round(mean_wall, 6),
        "latency_p50_s": round(lats[len(lats) // 2], 6),
        "latency_p99_s": round(lats[min(len(lats) - 1, int(0.99 * len(lats)))], 6),
        "all_certified": all(r.status == 0 and r.gap <= args.target for r in results),
        "sweeps_mean": statistics.mean(r.sweeps for r in results),
        "sample_bitwise_equal_to_alone": same,
    }


def leg_single(args, precision: str, problems=None, target=None, **kw) -> dict:
    """Single solves (mdot_solve), each problem once after one warm-up solve: mean time-to-gap."""
    import torch

    from paper_2307_08507_amd import mdot as M

    dev = torch.device("cuda", 0)
    k = args.grid
    n = k * k
    probs = problem_set(args)
    if problems is not None:
        probs = [probs[i] for i in problems]
    costs = {kind: grid_cost_device(k, kind, args.cost_storage, dev) for kind in {p["cost"] for p in probs}}
    ctx = M.Context(0)
    prm = M.default_params(precision=precision, **kw)
    u = torch.empty(n, dtype=torch.float64, device=dev)
    v = torch.empty_like(u)
    tg = args.target if target is None else target
    out = []
    for i, p in enumerate(probs):
        rd = torch.tensor(p["r"], dtype=torch.float64, device=dev)
        cd = torch.tensor(p["c"], dtype=torch.float64, device=dev)
        if i == 0:
            ctx.solve(costs[p["cost"]]["desc"](), rd, cd, tg, prm, u, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = ctx.solve(costs[p["cost"]]["desc"](), rd, cd, tg, prm, u, v)
        torch.cuda.synchronize()
        out.append((time.perf_counter() - t0, res))
    ctx.close()
    return {"time_to_gap_s": round(statistics.mean(t for t, _ in out), 6),
            "all_certified": all(r.status == 0 and (kw.get("gamma_f") or r.gap <= tg) for _, r in out),
            "sweeps_mean": statistics.mean(r.sweeps for _, r in out),
            "per_problem": [{"problem": p["name"], "s": round(t, 5), "sweeps": r.sweeps,
                             "gap": r.gap, "status": r.status} for p, (t, r) in zip(probs, out)]}


def leg_projectors(args) -> dict:
    """PNCG against the Sinkhorn projector (Alg. 4) inside the same annealing schedule, on the L1
    grid problems (the paper's comparison uses L1 costs at n=4096): LSE sweeps and time per
    solve at fixed gamma_f (the paper's setting), both with FP32 sweeps."""
    import argparse as _ap

    a = _ap.Namespace(**vars(args))
    l1 = [i for i, p in enumerate(problem_set(args)) if p["cost"] == "l1"]
    out = {}
    for gf in (2.0**9, 2.0**12):
        pn = leg_single(a, "f32", problems=l1, gamma_f=gf)
        sk = leg_single(a, "f32", problems=l1, gamma_f=gf, projector=1)
        out[f"gamma_f=2^{int(round(math.log2(gf)))}"] = {
            "pncg_sweeps_mean": pn["sweeps_mean"], "sinkhorn_sweeps_mean": sk["sweeps_mean"],
            "sweep_ratio_sinkhorn_over_pncg": round(sk["sweeps_mean"] / pn["sweeps_mean"], 3),
            "pncg_s": pn["time_to_gap_s"], "sinkhorn_s": sk["time_to_gap_s"],
            "status_ok": all(q["status"] == 0 for q in pn["per_problem"] + sk["per_problem"])}
    return out


def run_legs(args, head: dict) -> dict:
    """The rest of the metric beside the headline: FP64 and MIXED single solves, the batched
    engine (FP32 and MIXED), PNCG against the Sinkhorn projector, a short serving run, and the
    per-result accuracy of every precision mode."""
    import argparse as _ap

    legs = {}
    t0 = time.perf_counter()
    legs["f64"] = leg_single(args, "f64")
    legs["mixed"] = leg_single(args, "mixed")
    print(f"legs: single f64/mixed done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    for prec in ("f32", "mixed"):
        a = _ap.Namespace(**vars(args))
        a.steps, a.warmup, a.precision = 2, 1, prec
        b = bench_grid_batched(a)
        legs[f"batched_{prec}"] = {k: b[k] for k in ("value", "unit", "batch_wall_s", "latency_p50_s",
                                                     "latency_p99_s", "all_certified", "sweeps_mean",
                                                     "sample_bitwise_equal_to_alone")}
    print(f"legs: batched done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    legs["projectors"] = leg_projectors(args)
    print(f"legs: projectors done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    a = _ap.Namespace(**vars(args))
    a.requests = args.leg_requests
    srv = bench_serving(a)
    legs["serving"] = {k: srv[k] for k in ("value", "unit", "saturation_rps", "latency_p50_s", "latency_p99_s",
                                           "latency_max_s", "all_certified", "sample_bitwise_equal_to_alone",
                                           "hbm_budget_bytes", "peak_bytes_in_use", "tail_request")}
    legs["serving"]["workload"] = srv["config"]["workload"]
    print(f"legs: serving done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    prec = bench_precision(_ap.Namespace(**vars(args)))
    legs["precision_modes"] = {name: {k: m[k] for k in ("all_certified", "max_ub_diff_over_bound", "max_rel_ub_vs_ref",
                                                         "max_gap", "max_marg_err_l1", "time_to_gap_mean_s")}
                               for name, m in prec["modes"].items()}
    print(f"legs: precision modes done at {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    fp32 = head["value"]
    legs["summary"] = {
        "fp32_single_s": fp32,
        "f64_single_s": legs["f64"]["time_to_gap_s"],
        "mixed_single_s": legs["mixed"]["time_to_gap_s"],
        "fp32_batched_per_solve_s": legs["batched_f32"]["value"],
        "mixed_batched_per_solve_s": legs["batched_mixed"]["value"],
        "mixed_batched_vs_fp32_single": round(legs["batched_mixed"]["value"] / fp32, 4),
    }
    return legs


def bench_serving(args) -> dict:
    import numpy as np
    import torch

    from paper_2307_08507_amd import mdot as M
    from paper_2307_08507_amd import workloads as W

    dev = torch.device("cuda", 0)
    reqs = W.serving_stream(args.requests, 1.0, seed=args.seed, d=3)
    for q in reqs:
        q.XY = torch.tensor(np.concatenate([q.x, q.y]), dtype=torch.float32, device=dev)
        q.rd = torch.tensor(q.r, dtype=torch.float64, device=dev)
        q.cd = torch.tensor(q.c, dtype=torch.float64, device=dev)
        q.u = torch.empty(q.n, dtype=torch.float64, device=dev)
        q.v = torch.empty_like(q.u)
    prm = M.default_params(precision=args.precision)
    torch.cuda.synchronize()

    peak = [0]

    def run(arrivals):
        eng = M.Context(0, hbm_budget_bytes=args.hbm_budget)
        order = sorted(range(len(reqs)), key=lambda i: arrivals[i])
        nxt, tickets, done = 0, {}, {}
        t0 = time.perf_counter()
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(order) and arrivals[order[nxt]] <= now:
                q = reqs[order[nxt]]
                t = eng.submit(M.point_cost(q.XY, q.n, 3, "sqeuclid"), q.rd, q.cd, q.target, prm, q.u, q.v)
                if t is None:
                    break
                tickets[t] = order[nxt]
                nxt += 1
            if tickets:
                peak[0] = max(peak[0], eng.inflight()[1])
                eng.run(8)
                now = time.perf_counter() - t0
                for t in list(tickets):
                    res = eng.poll(t)
                    if res is not None:
                        done[tickets.pop(t)] = (now, res)
                        if len(done) % 16 == 0:
                            print(f"served {len(done)}/{len(reqs)} at {now:.2f} s", file=sys.stderr, flush=True)
            elif nxt < len(order):
                time.sleep(max(0.0, min(1e-3, arrivals[order[nxt]] - now)))
        eng.close()
        lat = [done[i][0] - arrivals[i] for i in range(len(reqs))]
        span = max(d[0] for d in done.values()) - min(arrivals)
        return lat, span, [done[i][1] for i in range(len(reqs))]

    # saturation: every request available at t = 0
    _, span_sat, _ = run([0.0] * len(reqs))
    sat = len(reqs) / span_sat
    rate = args.load * sat
    arrivals = [q.arrival for q in reqs]  # Poisson at rate 1: rescale to `rate`
    arrivals = [a / rate for a in arrivals]
    lat, span, res = run(arrivals)
    # a sample of requests solved alone must give the same result bit for bit
    ctx = M.Context(0)
    same = True
    for i in range(0, len(reqs), max(1, len(reqs) // 4)):
        q = reqs[i]
        u, v = torch.empty_like(q.u), torch.empty_like(q.v)
        r1 = ctx.solve(M.point_cost(q.XY, q.n, 3, "sqeuclid"), q.rd, q.cd, q.target, prm, u, v)
        same &= bool(torch.equal(u, q.u) and torch.equal(v, q.v) and r1.primal_cost == res[i].primal_cost)
    # the slowest request solved alone: its latency over its own solve time is the slowdown that
    # sharing the GPU with the requests in flight cost it
    i_max = max(range(len(reqs)), key=lambda i: lat[i])
    q = reqs[i_max]
    u, v = torch.empty_like(q.u), torch.empty_like(q.v)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r1 = ctx.solve(M.point_cost(q.XY, q.n, 3, "sqeuclid"), q.rd, q.cd, q.target, prm, u, v)
    torch.cuda.synchronize()
    alone_s = time.perf_counter() - t1
    same &= bool(torch.equal(u, q.u) and torch.equal(v, q.v) and r1.primal_cost == res[i_max].primal_cost)
    tail = {"n": q.n, "target_gap": q.target, "sweeps": int(r1.sweeps), "latency_s": round(lat[i_max], 4),
            "alone_s": round(alone_s, 4), "slowdown": round(lat[i_max] / alone_s, 2)}
    ctx.close()
    lat_s = sorted(lat)
    return {
        "metric": "serving throughput, point-cloud OT requests to certified gap",
        "value": round(len(reqs) / span, 3),
        "unit": "requests/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": args.precision,
        "data": "synthetic",
        "config": {"workload": (f"{len(reqs)} requests, Poisson arrivals at {rate:.2f}/s ({args.load:g} x "
                                f"saturation), n log-uniform in [512, 8192], d=3 GMM point clouds, "
                                f"Dirichlet(1) marginals, squared-Euclidean cost / max, target gap in "
                                f"{{1e-4, 1e-5, 1e-6, 1e-7}}")},
        "saturation_rps": round(sat, 3),
        "hbm_budget_bytes": args.hbm_budget,
        "peak_bytes_in_use": peak[0],
        "latency_p50_s": round(lat_s[len(lat_s) // 2], 4),
        "latency_p99_s": round(lat_s[min(len(lat_s) - 1, int(0.99 * len(lat_s)))], 4),
        "latency_max_s": round(lat_s[-1], 4),
        "all_certified": all(r.status == 0 and r.gap <= reqs[i].target for i, r in enumerate(res)),
        "sample_bitwise_equal_to_alone": same,
        "tail_request": tail,
    }


def bench_precision(args) -> dict:
    """Per-result accuracy of every precision mode on the grid problems: each problem is solved
    with FP64 exponentials on the exact FP64 cost (the reference: the paper's precision), then in
    each other mode. Per result: |UB - UB_ref| / UB_ref, the certified gap, the marginal error and
    gamma_final; for FP16/BF16 storage also delta = max |C_stored - C_exact| and the bound
    gap + 2 delta on the exact problem (the gap there is certified on the stored cost)."""
    import torch

    from paper_2307_08507_amd import mdot as M

    dev = torch.device("cuda", 0)
    k = args.grid
    n = k * k
    probs = problem_set(args)
    for p in probs:
        p["rd"] = torch.tensor(p["r"], dtype=torch.float64, device=dev)
        p["cd"] = torch.tensor(p["c"], dtype=torch.float64, device=dev)
    ctx = M.Context(0)
    u = torch.empty(n, dtype=torch.float64, device=dev)
    v = torch.empty_like(u)
    modes = [("f64_exact_cost", "f64", "f64"), ("f32", "f32", "f32"), ("f16_storage", "f32", "f16"),
             ("bf16_storage", "f32", "bf16"), ("recompute_points", "f32", "points"), ("mixed", "mixed", "f32")]
    exact = {kind: grid_cost_device(k, kind, "f64", dev)["keep"] for kind in COSTS}
    ref, ref_gap, out = {}, {}, {}
    for name, prec, storage in modes:
        costs = {kind: grid_cost_device(k, kind, storage, dev) for kind in COSTS}
        delta = {kind: (float((costs[kind]["keep"].double() - exact[kind]).abs().max())
                        if storage in ("f16", "bf16") else 0.0) for kind in COSTS}
        prm = M.default_params(precision=prec)
        rows = []
        for p in probs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve(costs[p["cost"]]["desc"](), p["rd"], p["cd"], args.target, prm, u, v)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            if name == "f64_exact_cost":
                ref[p["name"]], ref_gap[p["name"]] = res.primal_cost, res.gap
            row = {"problem": p["name"], "s": round(dt, 5), "status": res.status, "ub": res.primal_cost,
                   "rel_ub_vs_ref": abs(res.primal_cost - ref[p["name"]]) / ref[p["name"]], "gap": res.gap,
                   "marg_err_l1": res.marg_err_l1, "gamma_final": res.gamma_final, "sweeps": res.sweeps}
            if storage in ("f16", "bf16"):
                row["delta"] = delta[p["cost"]]
                row["error_bound_exact_cost"] = res.gap + 2.0 * delta[p["cost"]]
            # both UBs lie within their certified gaps of their own problems' optima, which differ
            # by at most delta: |UB - UB_ref| <= gap + gap_ref + 2 delta
            row["ub_diff_over_bound"] = abs(res.primal_cost - ref[p["name"]]) / max(
                res.gap + ref_gap[p["name"]] + 2.0 * row.get("delta", 0.0), 1e-300)
            rows.append(row)
        out[name] = {
            "precision": prec, "cost_storage": storage,
            "all_certified": all(r["status"] == 0 and r["gap"] <= args.target for r in rows),
            "max_rel_ub_vs_ref": max(r["rel_ub_vs_ref"] for r in rows),
            "max_ub_diff_over_bound": max(r["ub_diff_over_bound"] for r in rows),
            "max_gap": max(r["gap"] for r in rows),
            "max_marg_err_l1": max(r["marg_err_l1"] for r in rows),
            "gamma_final_range": [min(r["gamma_final"] for r in rows), max(r["gamma_final"] for r in rows)],
            "time_to_gap_mean_s": round(statistics.mean(r["s"] for r in rows), 6),
            "per_problem": rows,
        }
        if storage in ("f16", "bf16"):
            out[name]["max_error_bound_exact_cost"] = max(r["error_bound_exact_cost"] for r in rows)
        del costs
        print(f"precision mode {name} done", file=sys.stderr, flush=True)
    ctx.close()
    return {
        "metric": f"per-result accuracy of the precision modes at gap {args.target:g}, n={n}",
        "value": out["f32"]["max_rel_ub_vs_ref"],
        "unit": "relative UB difference against FP64 on the exact cost (FP32 mode, max over problems)",
        "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic",
        "config": {"workload": f"n={n} ({k}x{k} grid), {len(probs)} problems, certified gap {args.target:g}"},
        "modes": out,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--target", type=float, default=1e-6)
    ap.add_argument("--grid", type=int, default=64, help="grid side k (n = k*k)")
    ap.add_argument("--problems", type=int, default=8,
                    help="problems cycled through: pair 0 of every (family, cost) first; 64 = the full set")
    ap.add_argument("--family", action="append", choices=FAMILIES,
                    help="grid workload: marginal families to draw from (repeatable; default all four)")
    ap.add_argument("--precision", default="f32", choices=("f32", "f64", "mixed"))
    ap.add_argument("--cost-storage", default="f32", choices=("f32", "f16", "bf16", "f64", "points"))
    ap.add_argument("--workload", default="grid", choices=("grid", "serving", "precision"))
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--load", type=float, default=0.7, help="arrival rate as a fraction of saturation")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched", action="store_true",
                    help="grid workload: submit the problems together to the batched engine")
    ap.add_argument("--hbm-budget", type=int, default=1 << 30,
                    help="serving: HBM bytes the engine may hold for solves in flight (admission bound)")
    ap.add_argument("--no-legs", dest="legs", action="store_false",
                    help="default workload: report the headline only (no FP64/MIXED/batched/projector/serving "
                         "legs and no flushed-cache sweep)")
    ap.add_argument("--leg-requests", type=int, default=128, help="requests of the serving leg")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the solver runs on one GPU; "
              f"row sharding across GPUs is a design, not an implementation)", file=sys.stderr)
        return 2
    if args.workload == "serving":
        out = bench_serving(args)
    elif args.workload == "precision":
        out = bench_precision(args)
    elif args.batched:
        out = bench_grid_batched(args)
    else:
        out = bench_grid(args)
        default = (args.grid == 64 and args.cost_storage == "f32" and args.precision == "f32" and args.target == 1e-6)
        if args.legs and default:
            out["legs"] = run_legs(args, out)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
