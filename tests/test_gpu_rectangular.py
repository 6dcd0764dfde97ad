"""Rectangular problems (m sources x n targets, m != n) on the GPU against the FP64 oracle.

The paper's problems are square; the same path takes m x n costs (rows follow r, columns c).
Tolerances as in the square parity tests: FP64 sweeps to ~1e-12 of the log-sums, FP32 sweeps to
2e-6; FP64 solves take the oracle's decisions exactly at these sizes (stage, iteration, trial
and sweep counts) with UB and LB within 1e-9 relative."""
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


def _potentials(C, gamma, seed):
    from scipy.special import logsumexp

    m, n = C.shape
    rng = np.random.default_rng(seed)
    u = rng.standard_normal(m) * 0.5 - np.log(m)
    v = -np.log(n) - logsumexp(u[:, None] - gamma * C, axis=0)
    return u, v


def _lse2(ctx, desc, u, v, gamma, prec, m, n, fn=None):
    lr = torch.empty(m, dtype=torch.float64, device="cuda")
    lc = torch.empty(n, dtype=torch.float64, device="cuda")
    rc = (fn or ctx.lse2)(desc, dev(u), dev(v), gamma, lr, lc, precision=prec)
    torch.cuda.synchronize()
    assert rc == 0
    return lr.cpu().numpy(), lc.cpu().numpy()


@pytest.mark.parametrize("m,n", [(300, 1000), (1000, 300), (257, 65), (64, 4097), (1, 700), (700, 1),
                                 (20000, 300), (300, 20000)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lse2_rectangular(ctx, m, n, prec):
    print(f"rect lse2 {m}x{n} {prec}", flush=True)
    gamma = 120.0
    rng = np.random.default_rng(m * 7 + n)
    Cd = dev(rng.random((m, n)), torch.float32 if prec == "f32" else torch.float64)
    C64 = Cd.double().cpu().numpy()
    u, v = _potentials(C64, gamma, m + n)
    lr_o, lc_o = O.lse2(C64, u, v, gamma)
    lr, lc = _lse2(ctx, M.dense_cost(Cd), u, v, gamma, prec, m, n)
    tol = 1e-12 * gamma if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr, lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc, lc_o, rtol=0, atol=tol)


def test_lse2_noalloc_rectangular(ctx):
    m, n, gamma = 2000, 3500, 60.0
    rng = np.random.default_rng(5)
    Cd = dev(rng.random((m, n)), torch.float32)
    u, v = _potentials(Cd.double().cpu().numpy(), gamma, 6)
    a = _lse2(ctx, M.dense_cost(Cd), u, v, gamma, "f32", m, n)
    b = _lse2(ctx, M.dense_cost(Cd), u, v, gamma, "f32", m, n, fn=ctx.lse2_noalloc)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("shape", [(12, 16), (16, 12)])
def test_round_certify_rectangular(ctx, shape):
    C, r, c = W.grid_pair_problem(*shape, "blobs", "l1", 4)
    Cd = dev(C, torch.float64)
    g1, g2 = 2.0**9 / 2 ** (1 / 3), 2.0**9
    s1 = O.mdot(C, r, c, O.default_params(gamma_f=g1))
    s2 = O.mdot(C, r, c, O.default_params(gamma_f=g2))
    ub_o, lb_o, me_o, _ = O.round_certify(C, s2.u, s2.v, g2, r, c, u_prev=s1.u, v_prev=s1.v, gamma_prev=g1)
    ub, lb, me = ctx.round_certify(M.dense_cost(Cd), dev(s2.u), dev(s2.v), g2, dev(r), dev(c),
                                   u_prev=dev(s1.u), v_prev=dev(s1.v), gamma_prev=g1)
    assert ub == pytest.approx(ub_o, rel=1e-12, abs=1e-15)
    assert lb == pytest.approx(lb_o, rel=1e-12, abs=1e-15)
    assert me <= 1e-12


@pytest.mark.parametrize("prec_dtype", [torch.float64, torch.float32])
def test_round_certify_tall(ctx, prec_dtype):
    # 20000 rows are 313 row tiles: past 256 the finalize folds each column's partials with 8
    # lanes in its general path, in the LSE, Round and certificate sweeps alike
    m, n, gamma = 20000, 300, 200.0
    print(f"round/certify {m}x{n} {prec_dtype}", flush=True)
    rng = np.random.default_rng(20000)
    Cd = dev(rng.random((m, n)), prec_dtype)
    C64 = Cd.double().cpu().numpy()
    r = rng.dirichlet(np.ones(m))
    c = rng.dirichlet(np.ones(n))
    u, v = _potentials(C64, gamma, 3)
    up, vp = _potentials(C64, gamma / 2, 4)
    ub_o, lb_o, me_o, _ = O.round_certify(C64, u, v, gamma, r, c, u_prev=up, v_prev=vp, gamma_prev=gamma / 2)
    ub, lb, me = ctx.round_certify(M.dense_cost(Cd), dev(u), dev(v), gamma, dev(r), dev(c),
                                   u_prev=dev(up), v_prev=dev(vp), gamma_prev=gamma / 2)
    print(f"UB {ub:.15e} vs {ub_o:.15e}  LB {lb:.15e} vs {lb_o:.15e}", flush=True)
    # the Round sweeps take FP64 exponentials whatever the cost's storage
    assert ub == pytest.approx(ub_o, rel=1e-11, abs=1e-14)
    assert lb == pytest.approx(lb_o, rel=1e-11, abs=1e-14)
    assert lb <= ub
    assert me <= 1e-11


def _solve(ctx, desc, r, c, target=1e-4, **kw):
    u = torch.empty(r.size, dtype=torch.float64, device="cuda")
    v = torch.empty(c.size, dtype=torch.float64, device="cuda")
    res = ctx.solve(desc, dev(r), dev(c), target, M.default_params(**kw), u, v)
    return res, u.cpu().numpy(), v.cpu().numpy()


@pytest.mark.parametrize("shape,cost", [((12, 16), "sqeuclid"), ((16, 12), "sqeuclid"), ((16, 11), "l1")])
@pytest.mark.parametrize("variant", [{}, dict(projector=1)])
def test_schedule_mode_rectangular_matches_oracle(ctx, shape, cost, variant):
    C, r, c = W.grid_pair_problem(*shape, "smooth", cost, 0)
    gf = 2.0**9
    print(f"rect schedule {shape} {cost} {variant}", flush=True)
    res, u, v = _solve(ctx, M.dense_cost(dev(C)), r, c, gamma_f=gf, precision="f64", **variant)
    s = O.mdot(C, r, c, O.default_params(gamma_f=gf, **variant))
    R = s.result
    got = (res.stages, res.pncg_iters, res.ls_trials, res.sweeps)
    want = (R["stages"], R["pncg_iters"], R["ls_trials"], R["sweeps"])
    print(f"gpu {got} UB={res.primal_cost!r} LB={res.dual_bound!r}; oracle {want} UB={R['primal_cost']!r} "
          f"LB={R['dual_bound']!r}")
    assert res.status == 0 and s.status == 0
    assert got == want
    assert res.primal_cost == pytest.approx(R["primal_cost"], rel=1e-9)
    assert res.dual_bound == pytest.approx(R["dual_bound"], rel=1e-9)
    assert u.shape == (r.size,) and v.shape == (c.size,)
    np.testing.assert_allclose((u[:, None] + v[None, :])[::5, ::7], (s.u[:, None] + s.v[None, :])[::5, ::7],
                               rtol=0, atol=1e-6 * gf)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_adaptive_rectangular_brackets_exact_lp(ctx, prec):
    from tests.exact_ot import exact_lp

    for shape, seed in (((14, 18), 1), ((18, 13), 2)):
        C, r, c = W.grid_pair_problem(*shape, "cauchy", "sqeuclid", seed)
        Cd = dev(C, torch.float32)
        C64 = Cd.double().cpu().numpy()
        res, u, v = _solve(ctx, M.dense_cost(Cd), r, c, target=1e-5, precision=prec)
        ot = exact_lp(C64, r, c)
        print(f"rect adaptive {shape} {prec}: gap={res.gap:.3e} UB-OT={res.primal_cost - ot:.3e}")
        assert res.status == 0 and res.gap <= 1e-5
        assert res.dual_bound <= ot + 1e-12 <= res.primal_cost + 2e-12
        assert res.marg_err_l1 <= 1e-12


def test_transposed_problem_agrees(ctx):
    # OT(r, c, C) = OT(c, r, C^T): both certified solves bracket the same value
    C, r, c = W.grid_pair_problem(10, 15, "blobs", "sqeuclid", 3)
    a, _, _ = _solve(ctx, M.dense_cost(dev(C)), r, c, target=1e-6, precision="f64")
    b, _, _ = _solve(ctx, M.dense_cost(dev(np.ascontiguousarray(C.T))), c, r, target=1e-6, precision="f64")
    assert a.status == 0 and b.status == 0
    assert max(a.dual_bound, b.dual_bound) <= min(a.primal_cost, b.primal_cost) + 1e-12
    assert abs(a.primal_cost - b.primal_cost) <= 1e-6


@pytest.mark.parametrize("m,n", [(1, 50), (50, 1)])
def test_single_row_or_column(ctx, m, n):
    # one source (or one target): U(r, c) holds a single plan, found exactly
    rng = np.random.default_rng(m + n)
    C = rng.random((m, n))
    r = np.full(m, 1.0 / m)
    c = np.full(n, 1.0 / n)
    res, _, _ = _solve(ctx, M.dense_cost(dev(C)), r, c, target=1e-8, precision="f64")
    assert res.status == 0
    assert res.primal_cost == pytest.approx(float((r[:, None] * c[None, :] * C).sum()), abs=1e-12)


def test_points_rectangular(ctx):
    from tests.exact_ot import exact_lp

    m, n, d = 230, 310, 3
    x = W.gmm_points(m, d, 11)
    y = W.gmm_points(n, d, 12)
    dd = x.astype(np.float64)[:, None, :] - y.astype(np.float64)[None, :, :]
    raw = (dd * dd).sum(-1)
    scale = 1.0 / raw.max()
    C64 = raw * scale
    XY = dev(np.concatenate([x, y], 0), torch.float32)
    desc = M.point_cost(XY, n, d, "sqeuclid", scale=scale, m=m)
    gamma = 200.0
    u, v = _potentials(C64, gamma, 13)
    lr_o, lc_o = O.lse2(C64, u, v, gamma)
    lr, lc = _lse2(ctx, desc, u, v, gamma, "f64", m, n)
    np.testing.assert_allclose(lr, lr_o, rtol=0, atol=1e-11 * gamma)
    np.testing.assert_allclose(lc, lc_o, rtol=0, atol=1e-11 * gamma)
    r = W.dirichlet_marginal(m, 14)
    c = W.dirichlet_marginal(n, 15)
    res, _, _ = _solve(ctx, desc, r, c, target=1e-5, precision="f32")
    ot = exact_lp(C64, r, c)
    assert res.status == 0 and res.gap <= 1e-5
    assert res.dual_bound <= ot + 1e-9 and ot <= res.primal_cost + 1e-9


def test_engine_mixes_square_and_rectangular():
    # square and rectangular solves in one batch: each equals its solve alone bit for bit
    probs = []
    for shape, fam in (((12, 16), "smooth"), ((16, 16), "blobs"), ((17, 9), "cauchy")):
        C, r, c = W.grid_pair_problem(*shape, fam, "sqeuclid", 7)
        probs.append((dev(C, torch.float32), dev(r), dev(c)))
    prm = M.default_params()
    alone = M.Context(0)
    eng = M.Context(0)
    try:
        ref, outs, tickets = [], [], []
        for Cd, rd, cd in probs:
            u, v = torch.empty_like(rd), torch.empty_like(cd)
            ref.append((alone.solve(M.dense_cost(Cd), rd, cd, 1e-5, prm, u, v), u, v))
        for Cd, rd, cd in probs:
            u, v = torch.empty_like(rd), torch.empty_like(cd)
            outs.append((u, v))
            tickets.append(eng.submit(M.dense_cost(Cd), rd, cd, 1e-5, prm, u, v))
        assert all(t is not None for t in tickets)
        for t, (u, v), (ra, ua, va) in zip(tickets, outs, ref):
            rb = eng.poll(t, wait=True)
            assert torch.equal(u, ua) and torch.equal(v, va)
            assert (rb.primal_cost, rb.dual_bound, rb.sweeps) == (ra.primal_cost, ra.dual_bound, ra.sweeps)
            assert rb.status == 0 and rb.gap <= 1e-5
    finally:
        eng.close()
        alone.close()
