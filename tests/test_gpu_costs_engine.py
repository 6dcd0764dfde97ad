"""Parity of the HIP path for the other cost encodings and for the batched serving engine.

Cost encodings: FP16 / BF16 stored dense costs (the stored values are the cost: the oracle
runs on the decoded values) and point-cloud costs evaluated on the fly in FP64 from FP32
coordinates (the oracle runs on the same cost formed in numpy FP64; the two differ by the
summation order of d <= 3 squares, a few ulp). Tolerances as for the FP32 / FP64 sweeps.

Engine: solves advanced together by mdot_run return exactly (bit for bit) what mdot_solve
returns for each of them alone, and admission refuses work beyond the HBM budget.
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
    from scipy.special import logsumexp

    rng = np.random.default_rng(seed)
    u = rng.standard_normal(n) * 0.5 - np.log(n)
    v = -np.log(n) - logsumexp(u[:, None] - gamma * C, axis=0)
    return u, v


def _lse2(ctx, cost, u, v, gamma, prec):
    n = u.size
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    assert ctx.lse2(cost, dev(u), dev(v), gamma, lr, lc, precision=prec) == 0
    torch.cuda.synchronize()
    return lr.cpu().numpy(), lc.cpu().numpy()


@pytest.mark.parametrize("n", [300, 512])
@pytest.mark.parametrize("tdtype", ["f16", "bf16"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lse2_half_costs(ctx, n, tdtype, prec):
    print(f"lse2 {tdtype} n={n} prec={prec}", flush=True)
    gamma = 200.0
    C = np.random.default_rng(n + 7).random((n, n))
    Cd = dev(C, torch.float16 if tdtype == "f16" else torch.bfloat16)
    C64 = Cd.double().cpu().numpy()
    u, v = _potentials(n, n, C64, gamma)
    lr_o, lc_o = O.lse2(C64, u, v, gamma)
    lr, lc = _lse2(ctx, M.dense_cost(Cd), u, v, gamma, prec)
    tol = 1e-12 * gamma if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr, lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc, lc_o, rtol=0, atol=tol)


def _points(n, d, seed, kind):
    x = W.gmm_points(n, d, seed)
    y = W.gmm_points(n, d, seed + 1)
    dd = x.astype(np.float64)[:, None, :] - y.astype(np.float64)[None, :, :]
    raw = (dd * dd).sum(-1) if kind == "sqeuclid" else np.abs(dd).sum(-1)
    scale = 1.0 / raw.max()
    XY = dev(np.concatenate([x, y], 0), torch.float32)
    return XY, raw * scale, scale


@pytest.mark.parametrize("n,d,kind", [(300, 3, "sqeuclid"), (600, 2, "sqeuclid"), (512, 2, "l1"),
                                      (257, 1, "sqeuclid"), (350, 5, "sqeuclid"), (333, 8, "l1"),
                                      (400, 4, "sqeuclid"), (290, 7, "l1")])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lse2_point_costs(ctx, n, d, kind, prec):
    print(f"lse2 points n={n} d={d} {kind} prec={prec}", flush=True)
    gamma = 500.0
    XY, C64, scale = _points(n, d, 11 * n + d, kind)
    u, v = _potentials(n, n + 3, C64, gamma)
    lr_o, lc_o = O.lse2(C64, u, v, gamma)
    lr, lc = _lse2(ctx, M.point_cost(XY, n, d, kind, scale=scale), u, v, gamma, prec)
    tol = 1e-11 * gamma if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr, lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc, lc_o, rtol=0, atol=tol)


@pytest.mark.parametrize("kind", ["sqeuclid", "l1"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_planar_points_match_padded_3d(kind, prec):
    # Clouds with d <= 2 take a kernel instance without the third coordinate's arithmetic. The
    # same points with an explicit zero third coordinate take the general one; every term the
    # planar instance leaves out is an exact zero, so the sweeps must agree bit for bit. Each
    # call runs on a fresh context, so neither can replay the other's captured step graph.
    n = 700
    print(f"planar vs padded points n={n} {kind} prec={prec}", flush=True)
    XY2, C64, scale = _points(n, 2, 31, kind)
    XY3 = torch.cat([XY2.view(2 * n, 2), torch.zeros(2 * n, 1, device="cuda")], 1).contiguous().view(-1)
    gamma = 300.0
    u, v = _potentials(n, 4, C64, gamma)
    out = []
    for XY, d in ((XY2, 2), (XY3, 3)):
        c = M.Context(0)
        try:
            out.append(_lse2(c, M.point_cost(XY, n, d, kind, scale=scale), u, v, gamma, prec))
        finally:
            c.close()
    (lr2, lc2), (lr3, lc3) = out
    np.testing.assert_array_equal(lr2, lr3)
    np.testing.assert_array_equal(lc2, lc3)
    lr_o, lc_o = O.lse2(C64, u, v, gamma)
    tol = 1e-11 * gamma if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr3, lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc3, lc_o, rtol=0, atol=tol)


@pytest.mark.parametrize("kind", ["sqeuclid", "l1"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_3d_points_match_padded_8d(kind, prec):
    # Clouds with 4 <= d <= 8 take the 8-coordinate instance. A d = 3 cloud padded with five zero
    # coordinates takes it too, and every extra term is an exact zero: sweeps and Round/certificate
    # must agree bit for bit with the d = 3 instance (fresh contexts: no shared step graph).
    n = 520
    print(f"3-D vs padded 8-D points n={n} {kind} prec={prec}", flush=True)
    XY3, C64, scale = _points(n, 3, 57, kind)
    XY8 = torch.cat([XY3.view(2 * n, 3), torch.zeros(2 * n, 5, device="cuda")], 1).contiguous().view(-1)
    gamma = 300.0
    u, v = _potentials(n, 6, C64, gamma)
    r = W.dirichlet_marginal(n, 8)
    cc = W.dirichlet_marginal(n, 9)
    out = []
    for XY, d in ((XY3, 3), (XY8, 8)):
        c = M.Context(0)
        try:
            desc = M.point_cost(XY, n, d, kind, scale=scale)
            lr, lc = _lse2(c, desc, u, v, gamma, prec)
            out.append((lr, lc, c.round_certify(desc, dev(u), dev(v), gamma, dev(r), dev(cc))))
        finally:
            c.close()
    (lr3, lc3, rc3), (lr8, lc8, rc8) = out
    np.testing.assert_array_equal(lr3, lr8)
    np.testing.assert_array_equal(lc3, lc8)
    assert rc3 == rc8


@pytest.mark.parametrize("kind", ["sqeuclid", "l1"])
def test_point_dimension_change_on_one_context(kind):
    # Regression: a context caches its captured step graph, whose sweep kernel instance depends
    # on the point dimension (planar for d <= 2). Interleaving planar and d = 3 clouds of the
    # same n on one context must run the right instance every time: each result is checked
    # against the oracle on clouds whose third coordinate is non-zero.
    n = 640
    print(f"d=2 / d=3 interleaved on one context n={n} {kind}", flush=True)
    c = M.Context(0)
    try:
        for rep in range(2):
            for d in (2, 3, 6, 2, 3, 6):
                XY, C64, scale = _points(n, d, 90 + 7 * d + rep, kind)
                if d >= 3:
                    assert float(XY.view(2 * n, d)[:, d - 1].abs().max()) > 0.1
                gamma = 250.0
                u, v = _potentials(n, 5 + d, C64, gamma)
                lr, lc = _lse2(c, M.point_cost(XY, n, d, kind, scale=scale), u, v, gamma, "f32")
                lr_o, lc_o = O.lse2(C64, u, v, gamma)
                np.testing.assert_allclose(lr, lr_o, rtol=0, atol=2e-6)
                np.testing.assert_allclose(lc, lc_o, rtol=0, atol=2e-6)
                r = W.dirichlet_marginal(n, 3 + d)
                cc = W.dirichlet_marginal(n, 4 + d)
                ub, lb, me = c.round_certify(M.point_cost(XY, n, d, kind, scale=scale), dev(u), dev(v), gamma,
                                             dev(r), dev(cc))
                ub_o, lb_o, _, _ = O.round_certify(C64, u, v, gamma, r, cc)
                assert ub == pytest.approx(ub_o, rel=1e-11, abs=1e-14)
                assert lb == pytest.approx(lb_o, rel=1e-11, abs=1e-14)
    finally:
        c.close()


def test_point_cost_default_scale(ctx):
    # scale 0: the library normalises by the largest pairwise value
    n, d = 200, 3
    XY, C64, scale = _points(n, d, 5, "sqeuclid")
    gamma = 100.0
    u, v = _potentials(n, 9, C64, gamma)
    lr_o, lc_o = O.lse2(C64, u, v, gamma)
    lr, lc = _lse2(ctx, M.point_cost(XY, n, d, "sqeuclid"), u, v, gamma, "f64")
    np.testing.assert_allclose(lr, lr_o, rtol=0, atol=1e-9)
    np.testing.assert_allclose(lc, lc_o, rtol=0, atol=1e-9)


@pytest.mark.parametrize("d", [3, 6])
def test_solve_point_cloud_brackets_exact_ot(ctx, d):
    from tests.exact_ot import exact_lp

    n = 256
    XY, C64, scale = _points(n, d, 21, "sqeuclid")
    r = W.dirichlet_marginal(n, 1)
    c = W.dirichlet_marginal(n, 2)
    u = torch.empty(n, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    res = ctx.solve(M.point_cost(XY, n, d, "sqeuclid", scale=scale), dev(r), dev(c), 1e-5,
                    M.default_params(precision="f32"), u, v)
    ot = exact_lp(C64, r, c)
    print(f"points: gap={res.gap:.3e} UB-OT={res.primal_cost - ot:.3e} sweeps={res.sweeps}")
    assert res.status == 0 and res.gap <= 1e-5
    assert res.dual_bound <= ot + 1e-9 and res.primal_cost >= ot - 1e-9
    assert res.marg_err_l1 <= 1e-12


@pytest.mark.parametrize("tdtype", ["f16", "bf16"])
def test_solve_half_cost_brackets_exact_ot(ctx, tdtype):
    from tests.exact_ot import exact_lp

    C, r, c = W.grid_problem(16, "blobs", "sqeuclid", 3)
    Cd = dev(C, torch.float16 if tdtype == "f16" else torch.bfloat16)
    C64 = Cd.double().cpu().numpy()
    u = torch.empty(r.size, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    res = ctx.solve(M.dense_cost(Cd), dev(r), dev(c), 1e-5, M.default_params(precision="f32"), u, v)
    ot = exact_lp(C64, r, c)
    print(f"{tdtype}: gap={res.gap:.3e} UB-OT={res.primal_cost - ot:.3e}")
    assert res.status == 0 and res.gap <= 1e-5
    assert res.dual_bound <= ot + 1e-12 and res.primal_cost >= ot - 1e-12


# ---------------------------------------------------------------- serving engine
def _engine_problems():
    out = []
    for k, fam, cost, seed in [(16, "smooth", "sqeuclid", 1), (24, "uniform", "l1", 2), (32, "blobs", "sqeuclid", 3),
                               (17, "cauchy", "l1", 4), (40, "smooth", "l1", 5)]:
        C, r, c = W.grid_problem(k, fam, cost, seed)
        out.append((dev(C, torch.float32), dev(r), dev(c)))
    return out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_engine_bitwise_equals_solve(ctx, prec):
    probs = _engine_problems()
    prm = M.default_params(precision=prec)
    alone = []
    for C, r, c in probs:
        u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)
        res = ctx.solve(M.dense_cost(C), r, c, 1e-5, prm, u, v)
        alone.append((res, u.cpu(), v.cpu()))
    eng = M.Context(0)
    try:
        tickets, outs = [], []
        for C, r, c in probs:
            u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
            v = torch.empty_like(u)
            t = eng.submit(M.dense_cost(C), r, c, 1e-5, prm, u, v)
            assert t is not None
            tickets.append(t)
            outs.append((u, v))
        assert eng.inflight()[0] == len(probs)
        for _ in range(100000):
            if eng.inflight()[0] == 0:
                break
            eng.run(64)
        assert eng.inflight() == (0, 0)
        for t, (u, v), (ra, ua, va) in zip(tickets, outs, alone):
            rb = eng.poll(t)
            assert rb is not None
            assert torch.equal(u.cpu(), ua) and torch.equal(v.cpu(), va)
            for f in ("status", "primal_cost", "dual_bound", "gap", "gamma_final", "stages", "pncg_iters", "sweeps"):
                assert getattr(rb, f) == getattr(ra, f), f
            with pytest.raises(M.MdotError):
                eng.poll(t)  # a ticket is released once polled
    finally:
        eng.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_engine_results_against_oracle_and_exact_lp(prec):
    # engine results judged against independent references, not only against mdot_solve: three
    # problems of uneven n in one batch, each certified to gap 1e-5. The exact LP (scipy HiGHS)
    # must lie in [LB, UB] with UB - OT <= 1e-5, and the FP64 oracle's solve to the same gap must
    # agree on the primal cost to 1e-5 (both lie in [OT, OT + 1e-5]).
    from tests.exact_ot import exact_lp

    probs = []
    for k, fam, cost, seed in [(16, "smooth", "sqeuclid", 1), (17, "cauchy", "l1", 4), (24, "uniform", "l1", 2)]:
        C, r, c = W.grid_problem(k, fam, cost, seed)
        Cd = dev(C, torch.float32)
        probs.append((Cd, r, c, Cd.double().cpu().numpy()))
    prm = M.default_params(precision=prec)
    eng = M.Context(0)
    try:
        tickets, held = [], []  # the engine borrows inputs and outputs until the ticket is polled
        for Cd, r, c, _ in probs:
            rd, cd = dev(r), dev(c)
            u = torch.empty(r.size, dtype=torch.float64, device="cuda")
            v = torch.empty_like(u)
            held.append((rd, cd, u, v))
            t = eng.submit(M.dense_cost(Cd), rd, cd, 1e-5, prm, u, v)
            assert t is not None
            tickets.append(t)
        results = [eng.poll(t, wait=True) for t in tickets]
    finally:
        eng.close()
    for (Cd, r, c, C64), res in zip(probs, results):
        ot = exact_lp(C64, r, c)
        ref = O.mdot(C64, r, c, O.default_params(target_gap=1e-5)).result
        print(f"engine {prec} n={r.size}: gap={res.gap:.3e} UB-OT={res.primal_cost - ot:.3e} "
              f"oracle UB-OT={ref['primal_cost'] - ot:.3e}")
        assert res.status == 0 and res.gap <= 1e-5
        assert res.dual_bound <= ot + 1e-12 and ot <= res.primal_cost + 1e-12
        assert res.primal_cost - ot <= 1e-5
        assert abs(res.primal_cost - ref["primal_cost"]) <= 1e-5


@pytest.mark.parametrize("mix", ["planar", "mixed", "high_d"])
def test_engine_point_clouds_bitwise_equals_solve(ctx, mix):
    # Planar clouds run the planar point instance, d = 3 clouds the general one: a mixed batch
    # launches both sweeps in every step. Each result must equal its solve alone bit for bit.
    dims = {"planar": [2, 2, 2], "mixed": [2, 3, 2], "high_d": [2, 7, 3]}[mix]
    print(f"engine point clouds {mix} d={dims}", flush=True)
    probs = []
    for j, (n, d) in enumerate(zip([300, 520, 260], dims)):
        XY, _, scale = _points(n, d, 40 + j, "sqeuclid")
        probs.append((M.point_cost(XY, n, d, "sqeuclid", scale=scale), XY, dev(W.dirichlet_marginal(n, 2 * j + 1)),
                      dev(W.dirichlet_marginal(n, 2 * j + 2))))
    prm = M.default_params(precision="f32")
    alone = []
    for cost, _, r, c in probs:
        u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)
        res = ctx.solve(cost, r, c, 1e-5, prm, u, v)
        assert res.status == 0 and res.gap <= 1e-5
        alone.append((res, u.cpu(), v.cpu()))
    eng = M.Context(0)
    try:
        tickets, outs = [], []
        for cost, _, r, c in probs:
            u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
            v = torch.empty_like(u)
            tickets.append(eng.submit(cost, r, c, 1e-5, prm, u, v))
            outs.append((u, v))
        assert all(t is not None for t in tickets)
        for _ in range(100000):
            if eng.inflight()[0] == 0:
                break
            eng.run(64)
        assert eng.inflight() == (0, 0)
        for t, (u, v), (ra, ua, va) in zip(tickets, outs, alone):
            rb = eng.poll(t)
            assert torch.equal(u.cpu(), ua) and torch.equal(v.cpu(), va)
            for f in ("status", "primal_cost", "dual_bound", "gap", "sweeps"):
                assert getattr(rb, f) == getattr(ra, f), f
    finally:
        eng.close()


def test_engine_mixed_cost_types_bitwise_equals_solve(ctx):
    # One batch holding every cost type: dense FP64 / FP32 / FP16 / BF16 and point clouds of
    # both metrics, planar and not. Each step launches one sweep per type; finalize and decide
    # are shared. Every result must equal the same solve alone bit for bit.
    print("engine mixed cost types", flush=True)
    probs = []
    for k, cost, dt in [(14, "sqeuclid", torch.float64), (16, "l1", torch.float32), (18, "sqeuclid", torch.float16),
                        (15, "l1", torch.bfloat16)]:
        C, r, c = W.grid_problem(k, "blobs", cost, k)
        Cd = dev(C, dt)
        probs.append((M.dense_cost(Cd), Cd, dev(r), dev(c)))
    for n, d, kind in [(300, 3, "sqeuclid"), (280, 2, "l1"), (260, 2, "sqeuclid")]:
        XY, _, scale = _points(n, d, 60 + n, kind)
        probs.append((M.point_cost(XY, n, d, kind, scale=scale), XY, dev(W.dirichlet_marginal(n, n)),
                      dev(W.dirichlet_marginal(n, n + 1))))
    prm = M.default_params(precision="f32")
    alone = []
    for cost, _, r, c in probs:
        u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)
        res = ctx.solve(cost, r, c, 1e-5, prm, u, v)
        assert res.status == 0 and res.gap <= 1e-5
        alone.append((res, u.cpu(), v.cpu()))
    eng = M.Context(0)
    try:
        tickets, outs = [], []
        for cost, _, r, c in probs:
            u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
            v = torch.empty_like(u)
            tickets.append(eng.submit(cost, r, c, 1e-5, prm, u, v))
            outs.append((u, v))
        assert all(t is not None for t in tickets)
        assert eng.inflight()[0] == len(probs)
        for _ in range(100000):
            if eng.inflight()[0] == 0:
                break
            eng.run(64)
        assert eng.inflight() == (0, 0)
        for t, (u, v), (ra, ua, va) in zip(tickets, outs, alone):
            rb = eng.poll(t)
            assert torch.equal(u.cpu(), ua) and torch.equal(v.cpu(), va)
            for f in ("status", "primal_cost", "dual_bound", "gap", "sweeps"):
                assert getattr(rb, f) == getattr(ra, f), f
    finally:
        eng.close()


@pytest.mark.parametrize("k", [16, 33])
def test_engine_shared_cost_groups(ctx, k):
    # problems that share a cost sweep their tiles interleaved (one group per cost); every
    # result stays bit-identical to the solve alone. k = 33: n = 1089 has 18 x 5 = 90 tiles,
    # not a multiple of 8, so the groups carry idle workgroups
    print(f"engine shared-cost k={k}", flush=True)
    costs = {kind: dev(W.grid_problem(k, "smooth", kind, 0)[0], torch.float32) for kind in ("sqeuclid", "l1")}
    probs = []
    for j, fam in enumerate(["smooth", "blobs", "uniform"]):
        for kind in ("sqeuclid", "l1"):
            _, r, c = W.grid_problem(k, fam, kind, 10 + j)
            probs.append((costs[kind], dev(r), dev(c)))
    prm = M.default_params(precision="f32")
    alone = []
    for C, r, c in probs:
        u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)
        res = ctx.solve(M.dense_cost(C), r, c, 1e-5, prm, u, v)
        alone.append((res, u.cpu(), v.cpu()))
    eng = M.Context(0)
    try:
        tickets, outs = [], []
        for C, r, c in probs:
            u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
            v = torch.empty_like(u)
            tickets.append(eng.submit(M.dense_cost(C), r, c, 1e-5, prm, u, v))
            outs.append((u, v))
        assert all(t is not None for t in tickets)
        for _ in range(100000):
            if eng.inflight()[0] == 0:
                break
            eng.run(64)
        assert eng.inflight() == (0, 0)
        for t, (u, v), (ra, ua, va) in zip(tickets, outs, alone):
            rb = eng.poll(t)
            assert rb is not None and rb.status == 0
            assert torch.equal(u.cpu(), ua) and torch.equal(v.cpu(), va)
            for f in ("primal_cost", "dual_bound", "gap", "stages", "pncg_iters", "sweeps"):
                assert getattr(rb, f) == getattr(ra, f), f
    finally:
        eng.close()


def test_engine_staggered_submission(ctx):
    # a request admitted while others are half-way gets the same result as alone
    probs = _engine_problems()
    prm = M.default_params(precision="f32")
    C, r, c = probs[2]
    u0 = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
    v0 = torch.empty_like(u0)
    ref = ctx.solve(M.dense_cost(C), r, c, 1e-5, prm, u0, v0)
    eng = M.Context(0)
    try:
        keep = []
        for C1, r1, c1 in probs[:2]:
            u = torch.empty(r1.numel(), dtype=torch.float64, device="cuda")
            keep.append((u, torch.empty_like(u)))
            assert eng.submit(M.dense_cost(C1), r1, c1, 1e-5, prm, *keep[-1]) is not None
        eng.run(40)
        u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)
        t = eng.submit(M.dense_cost(C), r, c, 1e-5, prm, u, v)
        res = eng.poll(t, wait=True)
        assert torch.equal(u, u0) and torch.equal(v, v0)
        assert res.primal_cost == ref.primal_cost and res.sweeps == ref.sweeps
    finally:
        eng.close()


def test_engine_admission_budget():
    probs = _engine_problems()
    prm = M.default_params(precision="f32")
    C, r, c = probs[4]  # n = 1600
    eng = M.Context(0, hbm_budget_bytes=2_500_000)
    try:
        keep = []
        u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        keep.append((u, torch.empty_like(u)))
        t1 = eng.submit(M.dense_cost(C), r, c, 1e-5, prm, *keep[-1])
        assert t1 is not None
        _, used = eng.inflight()
        assert 0 < used <= 2_500_000
        u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        keep.append((u, torch.empty_like(u)))
        assert eng.submit(M.dense_cost(C), r, c, 1e-5, prm, *keep[-1]) is None  # over budget: busy
        res = eng.poll(t1, wait=True)
        assert res.status == 0
        t2 = eng.submit(M.dense_cost(C), r, c, 1e-5, prm, *keep[-1])
        assert t2 is not None
        assert eng.poll(t2, wait=True).primal_cost == res.primal_cost
    finally:
        eng.close()


# ---------------------------------------------------------------- MIXED precision
@pytest.mark.parametrize("cost", ["sqeuclid", "l1"])
def test_mixed_precision_certifies_on_exact_cost(ctx, cost):
    from tests.exact_ot import exact_lp

    C, r, c = W.grid_problem(16, "blobs", cost, 11)
    Cd = dev(C, torch.float32)
    C64 = Cd.double().cpu().numpy()
    u = torch.empty(r.size, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    res = ctx.solve(M.dense_cost(Cd), dev(r), dev(c), 1e-5, M.default_params(precision="mixed"), u, v)
    ref = ctx.solve(M.dense_cost(Cd), dev(r), dev(c), 1e-5, M.default_params(precision="f32"), u, v)
    ot = exact_lp(C64, r, c)
    print(f"mixed {cost}: proxy stages={res.proxy_stages} stages={res.stages} sweeps={res.sweeps} gap={res.gap:.3e} "
          f"UB-OT={res.primal_cost - ot:.3e}; f32 sweeps={ref.sweeps}")
    assert res.proxy_stages > 0
    assert res.status == 0 and res.gap <= 1e-5
    # the bound and the rounded plan refer to the exact (FP32-stored) cost
    assert res.dual_bound <= ot + 1e-12 and res.primal_cost >= ot - 1e-12
    assert res.marg_err_l1 <= 1e-12


def test_mixed_precision_rejected_where_unsupported(ctx):
    n, d = 64, 3
    XY, _, scale = _points(n, d, 3, "sqeuclid")
    r = torch.full((n,), 1.0 / n, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MdotError) as e:
        ctx.solve(M.point_cost(XY, n, d, "sqeuclid", scale=scale), r, r, 1e-4, M.default_params(precision="mixed"))
    assert e.value.code == -1
    eng = M.Context(0)
    try:
        with pytest.raises(M.MdotError) as e:
            eng.submit(M.point_cost(XY, n, d, "sqeuclid", scale=scale), r, r, 1e-4, M.default_params(precision="mixed"))
        assert e.value.code == -1
        C16 = dev(np.random.default_rng(0).random((n, n)), torch.float16)
        with pytest.raises(M.MdotError) as e:
            eng.submit(M.dense_cost(C16), r, r, 1e-4, M.default_params(precision="mixed"))
        assert e.value.code == -1
    finally:
        eng.close()


def test_engine_mixed_precision_bitwise_equals_solve(ctx):
    # MIXED solves in the engine pause at the switch to the exact cost; the engine binds the
    # exact cost at the next chunk boundary and the problem's sweeps move to the FP32 kernel
    # instance. Alongside a plain FP32 solve, each result must equal its solve alone bit for bit.
    print("engine MIXED", flush=True)
    probs = []
    for k, fam, cost, seed, prec in [(16, "blobs", "sqeuclid", 11, "mixed"), (20, "smooth", "l1", 12, "mixed"),
                                     (18, "cauchy", "sqeuclid", 13, "f32"), (24, "uniform", "sqeuclid", 14, "mixed")]:
        C, r, c = W.grid_problem(k, fam, cost, seed)
        probs.append((dev(C, torch.float32), dev(r), dev(c), prec))
    alone = []
    for C, r, c, prec in probs:
        u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)
        res = ctx.solve(M.dense_cost(C), r, c, 1e-5, M.default_params(precision=prec), u, v)
        assert res.status == 0 and res.gap <= 1e-5
        assert (res.proxy_stages > 0) == (prec == "mixed")
        alone.append((res, u.cpu(), v.cpu()))
    eng = M.Context(0)
    try:
        tickets, outs = [], []
        for C, r, c, prec in probs:
            u = torch.empty(r.numel(), dtype=torch.float64, device="cuda")
            v = torch.empty_like(u)
            tickets.append(eng.submit(M.dense_cost(C), r, c, 1e-5, M.default_params(precision=prec), u, v))
            outs.append((u, v))
        assert all(t is not None for t in tickets)
        for _ in range(100000):
            if eng.inflight()[0] == 0:
                break
            eng.run(64)
        assert eng.inflight() == (0, 0)
        for t, (u, v), (ra, ua, va) in zip(tickets, outs, alone):
            rb = eng.poll(t)
            assert torch.equal(u.cpu(), ua) and torch.equal(v.cpu(), va)
            for f in ("status", "primal_cost", "dual_bound", "gap", "sweeps", "stages", "proxy_stages"):
                assert getattr(rb, f) == getattr(ra, f), f
    finally:
        eng.close()
