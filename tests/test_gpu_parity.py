"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Kernel level: the fused two-sided LSE sweep and the Round/certificate sweeps against
oracle.lse2 / oracle.round_certify, element by element, on sizes that span several tiles
and a ragged tail. Solve level: the annealed PNCG solve against oracle.mdot on the small
grid workload (n = 256), in schedule mode (the paper's fixed gamma_f) and in adaptive
(certified-gap) mode, plus exact LP values.

Tolerances (written per test) follow from the arithmetic:
  F64 sweeps: FP64 exp/log and FP64 sums in a different order than the oracle, so values
    agree to a few ulp of the log-sums: |d lr| <= 1e-12 (+ n-dependent reduction error).
  F32 sweeps: exponent argument in FP64, exp2 in FP32 (1 ulp) after rounding the shifted
    argument to FP32, partial sums of 4 FP32 terms: relative error of each sum <= ~1e-6,
    so |d lr| <= 2e-6.
"""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2307_08507_amd import mdot as M  # noqa: E402
from paper_2307_08507_amd import workloads as W  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = M.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def _potentials(n, seed, C, gamma):
    """Potentials of the kind the solver visits: random u, then v from one Sinkhorn
    half-step (column sums exactly 1/n), so every row and column has a moderate log-sum."""
    from scipy.special import logsumexp

    rng = np.random.default_rng(seed)
    u = rng.standard_normal(n) * 0.5 - np.log(n)
    v = -np.log(n) - logsumexp(u[:, None] - gamma * C, axis=0)
    return u, v


@pytest.mark.parametrize("n,gamma,prec", [(256, 16.0, "f64"), (256, 16.0, "f32"), (1000, 300.0, "f64"),
                                           (1000, 300.0, "f32"), (257, 2.0**12, "f64"), (333, 50.0, "f32")])
def test_lse2_random_cost(ctx, n, gamma, prec):
    print(f"lse2 random n={n} gamma={gamma} prec={prec}", flush=True)
    rng = np.random.default_rng(n)
    C = rng.random((n, n))
    Cd = dev(C, torch.float32 if prec == "f32" else torch.float64)
    C64 = Cd.double().cpu().numpy()  # the stored values are the cost
    u, v = _potentials(n, n + 1, C64, gamma)
    lr_o, lc_o = O.lse2(C64, u, v, gamma)
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    rc = ctx.lse2(M.dense_cost(Cd), dev(u), dev(v), gamma, lr, lc, precision=prec)
    torch.cuda.synchronize()
    assert rc == 0
    tol = 1e-12 * max(1.0, gamma) if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr.cpu().numpy(), lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc.cpu().numpy(), lc_o, rtol=0, atol=tol)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lse2_grid_near_solution(ctx, prec):
    # potentials of an oracle solve: the regime the solver works in (entries ~ marginals)
    C, r, c = W.grid_problem(16, "smooth", "sqeuclid", 0)
    gf = 2.0**12
    s = O.mdot(C, r, c, O.default_params(gamma_f=gf))
    lr_o, lc_o = O.lse2(C, s.u, s.v, gf)
    n = r.size
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    Cd = dev(C, torch.float32 if prec == "f32" else torch.float64)
    lr_o, lc_o = O.lse2(Cd.double().cpu().numpy(), s.u, s.v, gf)
    ctx.lse2(M.dense_cost(Cd), dev(s.u), dev(s.v), gf, lr, lc, shift=dev(lr_o + 0.3), precision=prec)
    tol = 1e-12 if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr.cpu().numpy(), lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc.cpu().numpy(), lc_o, rtol=0, atol=tol)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_round_certify_parity(ctx, dtype):
    C, r, c = W.grid_problem(16, "blobs", "l1", 4)
    Cd = dev(C, dtype)
    C64 = Cd.double().cpu().numpy()
    g1, g2 = 2.0**10 / 2 ** (1 / 3), 2.0**10
    s1 = O.mdot(C64, r, c, O.default_params(gamma_f=g1))
    s2 = O.mdot(C64, r, c, O.default_params(gamma_f=g2))
    ub_o, lb_o, me_o, _ = O.round_certify(C64, s2.u, s2.v, g2, r, c, u_prev=s1.u, v_prev=s1.v, gamma_prev=g1)
    ub, lb, me = ctx.round_certify(M.dense_cost(Cd), dev(s2.u), dev(s2.v), g2, dev(r), dev(c),
                                   u_prev=dev(s1.u), v_prev=dev(s1.v), gamma_prev=g1)
    assert ub == pytest.approx(ub_o, rel=1e-12, abs=1e-15)
    assert lb == pytest.approx(lb_o, rel=1e-12, abs=1e-15)
    assert me <= 1e-12 and me_o <= 1e-12
    # without the previous stage only the u/gamma bound is used
    ub_o2, lb_o2, _, _ = O.round_certify(C64, s2.u, s2.v, g2, r, c)
    ub2, lb2, _ = ctx.round_certify(M.dense_cost(Cd), dev(s2.u), dev(s2.v), g2, dev(r), dev(c))
    assert lb2 == pytest.approx(lb_o2, rel=1e-12, abs=1e-15)
    assert ub2 == pytest.approx(ub_o2, rel=1e-12, abs=1e-15)


def _solve(ctx, C, r, c, target=1e-4, dtype=torch.float64, **kw):
    Cd = dev(C, dtype)
    u = torch.empty(r.size, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    res = ctx.solve(M.dense_cost(Cd), dev(r), dev(c), target, M.default_params(**kw), u, v)
    return res, u.cpu().numpy(), v.cpu().numpy(), Cd.double().cpu().numpy()


def _counts(res):
    return (res.stages, res.pncg_iters, res.ls_trials, res.sweeps)


def _ocounts(s):
    R = s.result
    return (R["stages"], R["pncg_iters"], R["ls_trials"], R["sweeps"])


@pytest.mark.parametrize("cost", ["sqeuclid", "l1"])
def test_schedule_mode_f64_matches_oracle(ctx, cost):
    # The paper's schedule to a fixed gamma_f, FP64 sweeps. The two FP64 paths round differently
    # (device exp and reduction order against libm), but here every decision lands on the same
    # side of its threshold: the same stages, PNCG iterations, line-search trials and sweeps.
    # UB and LB then agree to 1e-9 relative (measured: 1e-15 for sqeuclid; for L1 about 1e-10,
    # rounding amplified inside the stopping ball of the last stage).
    C, r, c = W.grid_problem(16, "smooth", cost, 0)
    gf = 2.0**9
    print(f"schedule f64 cost={cost}", flush=True)
    res, u, v, C64 = _solve(ctx, C, r, c, gamma_f=gf, precision="f64")
    s = O.mdot(C64, r, c, O.default_params(gamma_f=gf))
    R = s.result
    print(f"gpu: {_counts(res)} UB={res.primal_cost!r} LB={res.dual_bound!r}; oracle: {_ocounts(s)} "
          f"UB={R['primal_cost']!r} LB={R['dual_bound']!r}")
    assert res.status == 0 and s.status == 0
    assert _counts(res) == _ocounts(s)
    assert res.primal_cost == pytest.approx(R["primal_cost"], rel=1e-9)
    assert res.dual_bound == pytest.approx(R["dual_bound"], rel=1e-9)
    assert res.gamma_final == R["gamma_final"]
    # potentials: gauge-invariant comparison of u_i + v_j on a sample
    np.testing.assert_allclose((u[:, None] + v[None, :])[::7, ::5], (s.u[:, None] + s.v[None, :])[::7, ::5],
                               rtol=0, atol=1e-6 * gf)


_LP = {}


def _exact(C64, r, c, key):
    from tests.exact_ot import exact_lp

    if key not in _LP:
        _LP[key] = exact_lp(C64, r, c)
    return _LP[key]


# Seeds of the small grid workload (gap 1e-4) whose FP64 solve does not take the oracle's
# decisions exactly, with the difference in (stages, PNCG iterations, line-search trials).
# Every other seed must match exactly.
ADAPTIVE_F64_DIVERGENT = {0: (0, 1, 1), 6: (0, -6, -7)}


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adaptive_config1(ctx, prec):
    # The small grid workload: n = 256, smoothed fields, squared-Euclidean cost, gap 1e-4, seeds
    # 0-9. Every seed: certified, and the exact LP inside [LB, UB]. FP64 sweeps: the oracle's
    # decisions exactly (stages, PNCG iterations, trials), except the named seeds, which must show
    # exactly the named difference. With equal decisions the iterates differ only by rounding,
    # accumulated over ~600 iterations up to gamma ~ 2^11: |dUB| <= 1e-3 target (measured
    # <= 4e-9). A seed where a stage's gradient norm crosses eps_d / 2 at another iteration
    # moves UB by up to 1e-2 target (seed 0: one more trial, 7.4e-7, the same trial the oracle
    # takes with exp perturbed by 2 ulp; seed 6: 6 iterations fewer, 7.6e-8).
    mism = []
    for seed in range(10):
        C, r, c = W.grid_problem(16, "smooth", "sqeuclid", seed)
        print(f"adaptive {prec} seed={seed}", flush=True)
        res, u, v, C64 = _solve(ctx, C, r, c, target=1e-4, dtype=torch.float32, precision=prec)
        ot = _exact(C64, r, c, ("config1", seed))
        s = O.mdot(C64, r, c, O.default_params(target_gap=1e-4))
        print(f"{prec} seed {seed}: gpu {_counts(res)} gap={res.gap:.3e} UB={res.primal_cost!r}; oracle "
              f"{_ocounts(s)} gap={s.result['gap']:.3e} UB={s.result['primal_cost']!r}; UB-OT={res.primal_cost - ot:.3e}")
        assert res.status == 0
        assert res.gap <= 1e-4
        assert res.dual_bound <= ot + 1e-12
        assert res.primal_cost >= ot - 1e-12
        assert res.primal_cost - ot <= 1e-4
        assert res.marg_err_l1 <= 1e-12
        if prec == "f64":
            delta = tuple(a - b for a, b in zip(_counts(res)[:3], _ocounts(s)[:3]))
            tol = 1e-2 * 1e-4 if seed in ADAPTIVE_F64_DIVERGENT else 1e-3 * 1e-4
            dub, dgap = abs(res.primal_cost - s.result["primal_cost"]), abs(res.gap - s.result["gap"])
            print(f"  seed {seed}: decision delta {delta}, |dUB|={dub:.2e} |dgap|={dgap:.2e}")
            if delta != ADAPTIVE_F64_DIVERGENT.get(seed, (0, 0, 0)) or dub > tol or dgap > tol:
                mism.append((seed, delta, dub, dgap))
    assert not mism, mism


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_f32_primal_within_1e6_of_oracle(ctx, seed):
    # The FP32 path (FP32 exp while the stage tolerance is >= 1e-7, FP64 exp below) solved to the
    # same certified gap as the FP64 oracle. Both primal costs lie in [OT, OT + gap], so they agree
    # to max(gap) absolute; at gap 1e-8 and UB ~ 1e-2 that is 1e-6 relative, the criterion.
    C, r, c = W.grid_problem(16, "smooth", "sqeuclid", seed)
    target = 1e-8
    res, u, v, C64 = _solve(ctx, C, r, c, target=target, dtype=torch.float32, precision="f32")
    s = O.mdot(C64, r, c, O.default_params(target_gap=target))
    R = s.result
    rel = abs(res.primal_cost - R["primal_cost"]) / R["primal_cost"]
    print(f"f32 seed {seed}: gap={res.gap:.3e} UB={res.primal_cost!r} oracle gap={R['gap']:.3e} "
          f"UB={R['primal_cost']!r} rel={rel:.2e} switches={res.prec_switches}")
    assert res.status == 0 and s.status == 0
    assert res.gap <= target and R["gap"] <= target
    assert rel <= 1e-6
    assert res.dual_bound <= R["primal_cost"] + 1e-15 and R["dual_bound"] <= res.primal_cost + 1e-15


def test_sweep_budget_matches_oracle(ctx):
    # max_sweeps: the solve stops after the sweep that spends the budget, rounds and certifies the
    # last accepted iterate and warns; the oracle reads the budget the same way
    C, r, c = W.grid_problem(16, "blobs", "sqeuclid", 2)
    kw = dict(max_sweeps=150)
    res, u, v, C64 = _solve(ctx, C, r, c, target=1e-7, precision="f64", **kw)
    s = O.mdot(C64, r, c, O.default_params(target_gap=1e-7, **kw))
    R = s.result
    print(f"budget: gpu {_counts(res)} status={res.status} UB={res.primal_cost!r} LB={res.dual_bound!r}; oracle "
          f"{_ocounts(s)} status={s.status} UB={R['primal_cost']!r} LB={R['dual_bound']!r}")
    assert res.status == M.MDOT_W_NOT_CONVERGED and s.status == 1
    assert res.sweeps == 150 and R["sweeps"] == 150
    assert _counts(res) == _ocounts(s)
    assert res.primal_cost == pytest.approx(R["primal_cost"], rel=1e-9)
    assert res.dual_bound == pytest.approx(R["dual_bound"], rel=1e-9)
    assert res.gap > 1e-7


def test_gamma_cap_matches_oracle(ctx):
    # an explicit gamma cap below what the target needs: the last stage runs at the cap and the
    # solve warns with the best certified gap it reached
    C, r, c = W.grid_problem(16, "smooth", "l1", 3)
    kw = dict(gamma_cap=2.0**8)
    res, u, v, C64 = _solve(ctx, C, r, c, target=1e-7, precision="f64", **kw)
    s = O.mdot(C64, r, c, O.default_params(target_gap=1e-7, **kw))
    R = s.result
    print(f"gamma cap: gpu {_counts(res)} status={res.status} gamma={res.gamma_final} gap={res.gap:.3e}; oracle "
          f"{_ocounts(s)} status={s.status} gamma={R['gamma_final']} gap={R['gap']:.3e}")
    assert res.status == M.MDOT_W_NOT_CONVERGED and s.status == 1
    assert _counts(res) == _ocounts(s)
    assert res.gamma_final <= 2.0**8 and res.gamma_final == R["gamma_final"]
    assert res.gap == pytest.approx(R["gap"], rel=1e-7)
    assert res.primal_cost == pytest.approx(R["primal_cost"], rel=1e-9)


def test_line_search_cap_matches_oracle(ctx):
    # at most 2 line-search trials: at the cap the step falls back to alpha_lo when it is > 0,
    # otherwise the stage ends unconverged (schedule mode then warns)
    C, r, c = W.grid_problem(16, "cauchy", "sqeuclid", 4)
    kw = dict(gamma_f=2.0**9, max_ls_trials=2)
    res, u, v, C64 = _solve(ctx, C, r, c, precision="f64", **kw)
    s = O.mdot(C64, r, c, O.default_params(**kw))
    R = s.result
    print(f"ls cap: gpu {_counts(res)} status={res.status} failures={res.ls_failures}; oracle {_ocounts(s)} "
          f"status={s.status} failures={R['ls_failures']}")
    assert res.ls_failures > 0
    assert res.status == s.status
    assert res.ls_failures == R["ls_failures"]
    assert _counts(res) == _ocounts(s)
    assert res.primal_cost == pytest.approx(R["primal_cost"], rel=1e-9)


def test_invalid_inputs(ctx):
    n = 64
    C = dev(np.random.default_rng(0).random((n, n)), torch.float32)
    r = np.full(n, 1.0 / n)
    bad = r.copy()
    bad[3] = -bad[3]
    with pytest.raises(M.MdotError) as e:
        ctx.solve(M.dense_cost(C), dev(bad), dev(r), 1e-4)
    assert e.value.code == -2
    with pytest.raises(M.MdotError) as e:
        ctx.solve(M.dense_cost(C), dev(r * 1.01), dev(r), 1e-4)
    assert e.value.code == -2
    with pytest.raises(M.MdotError) as e:
        ctx.solve(M.dense_cost(C, scale=2.0), dev(r), dev(r), 1e-4)
    assert e.value.code == -3
    with pytest.raises(M.MdotError) as e:
        ctx.solve(M.dense_cost(C), dev(r), dev(r), -1.0)
    assert e.value.code == -1
