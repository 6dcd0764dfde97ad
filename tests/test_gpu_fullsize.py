"""Parity at the benchmark's size and in the degenerate cases.

* Full size: the n = 4096 grid workload in the launch configuration bench.py times (FP32
  stored cost, one workgroup per 64 x 256 tile). The oracle cannot run a whole solve there in
  seconds, so the sweep is checked on sampled rows and columns (each log-sum recomputed in
  FP64 by the oracle's definition), and the solve's output is checked by the oracle's own
  Round + certificate on the returned potentials. A ragged size (n = 4097: no 16-byte rows,
  ragged last tiles) covers the other load path at scale.
* Past n = 8192 (the finalize's other instance): point-cost sweeps at n = 12000 on sampled rows
  and columns, and an n = 9000 point-cost solve re-certified by the oracle.
* The largest size (MDOT_MAX_N = 131072): point-cost sweeps in both precisions and a 64 GiB
  stored FP32 cost, on sampled rows and columns; one more is rejected.
* Degenerate cases with closed forms: n = 1, identical marginals on a cost with zero
  diagonal (OT = 0), and a separable cost C_ij = a_i + b_j (every plan costs <a, r> + <b, c>).

Inputs are seeded and synthetic (paper_2307_08507_amd.workloads); expected values come from
the oracle or from the closed forms, never from the HIP path.
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


def _sampled_lse(C, u, v, gamma, rows, cols):
    from scipy.special import logsumexp

    lr = np.array([logsumexp(u[i] + v - gamma * C[i]) for i in rows])
    lc = np.array([logsumexp(u + v[j] - gamma * C[:, j]) for j in cols])
    return lr, lc


@pytest.mark.parametrize("k,ragged", [(64, False), (64, True)])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_lse2_fullsize_sampled(ctx, k, ragged, prec):
    from scipy.special import logsumexp

    C, r, c = W.grid_problem(k, "smooth", "sqeuclid", 1000)
    if ragged:  # n = 4097: one extra point at the far corner
        n0 = C.shape[0]
        C = np.pad(C, ((0, 1), (0, 1)), constant_values=1.0)
        C[n0, n0] = 0.0
        r = np.append(r, 1e-6)
        c = np.append(c, 1e-6)
    n = C.shape[0]
    print(f"full-size lse2 n={n} prec={prec}", flush=True)
    Cd = dev(C, torch.float32)
    C64 = Cd.double().cpu().numpy()
    gamma = 300.0
    rng = np.random.default_rng(n)
    u = np.log(r) + rng.standard_normal(n) * 0.1
    v = -logsumexp(u[:, None] - gamma * C64, axis=0) + np.log(c)
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    assert ctx.lse2(M.dense_cost(Cd), dev(u), dev(v), gamma, lr, lc, precision=prec) == 0
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([rng.choice(n, 60, replace=False), [0, n - 1]]))
    cols = np.unique(np.concatenate([rng.choice(n, 60, replace=False), [0, n - 1]]))
    lr_o, lc_o = _sampled_lse(C64, u, v, gamma, rows, cols)
    tol = 1e-12 * gamma if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr.cpu().numpy()[rows], lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc.cpu().numpy()[cols], lc_o, rtol=0, atol=tol)


def test_solve_fullsize_recertified_by_oracle(ctx):
    # the benchmark's first problem (uniform marginals, squared-Euclidean grid cost, n = 4096)
    k = 64
    r = W.grid_problem_marginals(k, "uniform", 1000)
    c = W.grid_problem_marginals(k, "uniform", 1001)
    C = W.grid_cost(k, "sqeuclid")
    Cd = dev(C, torch.float32)
    C64 = Cd.double().cpu().numpy()
    u = torch.empty(k * k, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    res = ctx.solve(M.dense_cost(Cd), dev(r), dev(c), 1e-6, M.default_params(precision="f32"), u, v)
    print(f"n=4096 solve: gap={res.gap:.3e} UB={res.primal_cost!r} LB={res.dual_bound!r} "
          f"gamma=2^{np.log2(res.gamma_final):.2f} sweeps={res.sweeps}", flush=True)
    assert res.status == 0 and 0 <= res.gap <= 1e-6
    # the oracle rounds the plan of the returned potentials at gamma_final (Alg. 3) and bounds
    # OT with their c-transforms: its UB is the GPU's UB up to FP32-exp rounding, and the
    # GPU's certified bound cannot exceed a feasible plan's cost
    ub_o, lb_o, me_o, _ = O.round_certify(C64, u.cpu().numpy(), v.cpu().numpy(), res.gamma_final, r, c)
    print(f"oracle: UB={ub_o!r} LB(u/gamma)={lb_o!r} marg_err={me_o:.2e}")
    assert res.primal_cost == pytest.approx(ub_o, rel=1e-5)
    assert res.dual_bound <= ub_o + 1e-12
    assert lb_o <= res.primal_cost + 1e-12
    assert me_o <= 1e-12


_ORACLE_4096 = {}


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_solve_fullsize_schedule_mode_matches_oracle(ctx, prec):
    # The benchmark's size (n = 4096, FP32-stored squared-Euclidean grid cost, smoothed-field
    # marginals) on the paper's schedule to a short gamma_f = 2^7 (10 stages), which keeps the
    # FP64 oracle to seconds. FP64 sweeps take the oracle's decisions exactly (stages, PNCG
    # iterations, trials, sweeps) with UB and LB within 1e-9 relative. FP32 sweeps (FP32 exp)
    # follow other iterates inside each stage's stopping ball ||grad||_1 <= eps_d / 2, which at
    # gamma <= 2^7 is wide (eps_d / 2 ~ 3e-3); both paths still run the same stages and end at
    # the same gamma, and their rounded plans' costs agree to 1e-4 relative.
    k, gf = 64, 2.0**7
    C, r, c = W.grid_problem(k, "smooth", "sqeuclid", 0)
    Cd = dev(C, torch.float32)
    C64 = Cd.double().cpu().numpy()
    if "s" not in _ORACLE_4096:
        _ORACLE_4096["s"] = O.mdot(C64, r, c, O.default_params(gamma_f=gf))
    s = _ORACLE_4096["s"]
    R = s.result
    u = torch.empty(k * k, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    print(f"n=4096 schedule {prec}", flush=True)
    res = ctx.solve(M.dense_cost(Cd), dev(r), dev(c), 1e-4, M.default_params(gamma_f=gf, precision=prec), u, v)
    got = (res.stages, res.pncg_iters, res.ls_trials, res.sweeps)
    want = (R["stages"], R["pncg_iters"], R["ls_trials"], R["sweeps"])
    print(f"gpu {got} UB={res.primal_cost!r} LB={res.dual_bound!r}; oracle {want} UB={R['primal_cost']!r} "
          f"LB={R['dual_bound']!r}")
    assert res.status == 0 and s.status == 0
    assert res.stages == R["stages"] and res.gamma_final == R["gamma_final"] == gf
    if prec == "f64":
        assert got == want
        assert res.primal_cost == pytest.approx(R["primal_cost"], rel=1e-9)
        assert res.dual_bound == pytest.approx(R["dual_bound"], rel=1e-9)
    else:
        assert res.primal_cost == pytest.approx(R["primal_cost"], rel=1e-4)
        assert res.dual_bound == pytest.approx(R["dual_bound"], rel=1e-4)


def _points_problem(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.random((n, 2)).astype(np.float32)
    Y = rng.random((n, 2)).astype(np.float32)
    r = rng.random(n) + 0.1
    c = rng.random(n) + 0.1
    return X, Y, r / r.sum(), c / c.sum()


def _points_rows(X, Y, idx, scale, axis):
    """Rows (axis 0) or columns (axis 1) idx of C = scale |x_i - y_j|^2 in FP64 from the FP32
    coordinates."""
    A, B = (X, Y) if axis == 0 else (Y, X)
    A, B = A.astype(np.float64)[idx], B.astype(np.float64)
    out = np.zeros((len(A), len(B)))
    for e in range(A.shape[1]):
        d = np.subtract.outer(A[:, e], B[:, e])
        out += d * d
    return scale * out


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_lse2_large_n_points_sampled(ctx, prec):
    # past n = 8192 the finalize folds 32 partials per lane (its other kernel instance);
    # n = 12000 also leaves ragged last tiles. Point costs, scale 1/2 (C in [0, 1])
    from scipy.special import logsumexp

    n, gamma, scale = 12000, 300.0, 0.5
    print(f"large-n lse2 points n={n} prec={prec}", flush=True)
    X, Y, _, _ = _points_problem(n, 77)
    rng = np.random.default_rng(78)
    u = rng.standard_normal(n) * 0.1
    v = rng.standard_normal(n) * 0.1
    XY = dev(np.concatenate([X, Y]).ravel(), torch.float32)
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    assert ctx.lse2(M.point_cost(XY, n, 2, "sqeuclid", scale=scale), dev(u), dev(v), gamma, lr, lc,
                    precision=prec) == 0
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([rng.choice(n, 40, replace=False), [0, n - 1]]))
    cols = np.unique(np.concatenate([rng.choice(n, 40, replace=False), [0, n - 1]]))
    Cr = _points_rows(X, Y, rows, scale, 0)
    Cc = _points_rows(X, Y, cols, scale, 1)
    lr_o = logsumexp(u[rows, None] + v[None, :] - gamma * Cr, axis=1)
    lc_o = logsumexp(u[None, :] + v[cols, None] - gamma * Cc, axis=1)
    tol = 1e-12 * gamma if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr.cpu().numpy()[rows], lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc.cpu().numpy()[cols], lc_o, rtol=0, atol=tol)


MAX_N = 131072  # MDOT_MAX_N of include/mdot.h


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_lse2_max_n_points_sampled(ctx, prec):
    # the largest size the library takes: 2048 x 512 tiles, partial arrays of 9 GB in total, and
    # the finalize's general path (more row tiles than its fast path holds)
    from scipy.special import logsumexp

    n, gamma, scale = MAX_N, 200.0, 0.5
    print(f"max-n lse2 points n={n} prec={prec}", flush=True)
    X, Y, _, _ = _points_problem(n, 81)
    rng = np.random.default_rng(82)
    u = rng.standard_normal(n) * 0.1
    v = rng.standard_normal(n) * 0.1
    XY = dev(np.concatenate([X, Y]).ravel(), torch.float32)
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    assert ctx.lse2(M.point_cost(XY, n, 2, "sqeuclid", scale=scale), dev(u), dev(v), gamma, lr, lc,
                    precision=prec) == 0
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([rng.choice(n, 24, replace=False), [0, n - 1]]))
    cols = np.unique(np.concatenate([rng.choice(n, 24, replace=False), [0, n - 1]]))
    lr_o = logsumexp(u[rows, None] + v[None, :] - gamma * _points_rows(X, Y, rows, scale, 0), axis=1)
    lc_o = logsumexp(u[None, :] + v[cols, None] - gamma * _points_rows(X, Y, cols, scale, 1), axis=1)
    tol = 1e-12 * gamma if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr.cpu().numpy()[rows], lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc.cpu().numpy()[cols], lc_o, rtol=0, atol=tol)


def test_lse2_max_n_dense_sampled(ctx):
    # a stored FP32 cost at the largest size (64 GiB): row offsets past 2^32 bytes, each tile's
    # buffer range clamped below 2 GiB. Seeded uniform costs; the sampled rows and columns are
    # copied back as inputs and the log-sums formed from them by their definition.
    from scipy.special import logsumexp

    n, gamma = MAX_N, 50.0
    print(f"max-n lse2 dense f32 n={n}", flush=True)
    g = torch.Generator(device="cuda").manual_seed(83)
    C = torch.rand((n, n), generator=g, device="cuda", dtype=torch.float32)
    rng = np.random.default_rng(84)
    u = rng.standard_normal(n) * 0.1 - np.log(n)
    v = rng.standard_normal(n) * 0.1
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    assert ctx.lse2(M.dense_cost(C), dev(u), dev(v), gamma, lr, lc, precision="f32") == 0
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([rng.choice(n, 16, replace=False), [0, n - 1]]))
    cols = np.unique(np.concatenate([rng.choice(n, 16, replace=False), [0, n - 1]]))
    Cr = C[torch.as_tensor(rows, device="cuda")].double().cpu().numpy()
    Cc = C[:, torch.as_tensor(cols, device="cuda")].double().cpu().numpy().T
    del C
    torch.cuda.empty_cache()
    lr_o = logsumexp(u[rows, None] + v[None, :] - gamma * Cr, axis=1)
    lc_o = logsumexp(u[None, :] + v[cols, None] - gamma * Cc, axis=1)
    np.testing.assert_allclose(lr.cpu().numpy()[rows], lr_o, rtol=0, atol=2e-6)
    np.testing.assert_allclose(lc.cpu().numpy()[cols], lc_o, rtol=0, atol=2e-6)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_lse2_n100k_points_d3_sampled(ctx, prec):
    # the paper's largest size for costs computed on the fly (about 10^5 points): n = 100,000,
    # ragged last tiles (1563 x 391), 3-D clouds from a Gaussian mixture, scale 1 / (max |x| +
    # max |y|)^2, which keeps C in [0, 1] (the library's range pass checks it)
    from scipy.special import logsumexp

    from paper_2307_08507_amd import workloads as Wl

    n, gamma = 100_000, 300.0
    print(f"n=100000 lse2 points d=3 prec={prec}", flush=True)
    rng = np.random.default_rng(91)
    X = Wl.gmm_points(n, 3, 92).astype(np.float32)
    Y = Wl.gmm_points(n, 3, 93).astype(np.float32)
    u = rng.standard_normal(n) * 0.1 - np.log(n)
    v = rng.standard_normal(n) * 0.1
    XY = dev(np.concatenate([X, Y]).ravel(), torch.float32)
    lr = torch.empty(n, dtype=torch.float64, device="cuda")
    lc = torch.empty_like(lr)
    X64, Y64 = X.astype(np.float64), Y.astype(np.float64)
    scale = 1.0 / (np.sqrt((X64 ** 2).sum(1).max()) + np.sqrt((Y64 ** 2).sum(1).max())) ** 2
    assert ctx.lse2(M.point_cost(XY, n, 3, "sqeuclid", scale=scale), dev(u), dev(v), gamma, lr, lc,
                    precision=prec) == 0
    torch.cuda.synchronize()
    rows = np.unique(np.concatenate([rng.choice(n, 20, replace=False), [0, n - 1]]))
    cols = np.unique(np.concatenate([rng.choice(n, 20, replace=False), [0, n - 1]]))
    lr_o = logsumexp(u[rows, None] + v[None, :] - gamma * _points_rows(X, Y, rows, scale, 0), axis=1)
    lc_o = logsumexp(u[None, :] + v[cols, None] - gamma * _points_rows(X, Y, cols, scale, 1), axis=1)
    tol = 1e-12 * gamma if prec == "f64" else 2e-6
    np.testing.assert_allclose(lr.cpu().numpy()[rows], lr_o, rtol=0, atol=tol)
    np.testing.assert_allclose(lc.cpu().numpy()[cols], lc_o, rtol=0, atol=tol)


def test_size_past_max_rejected(ctx):
    # a descriptor claiming MAX_N + 1 points over a small buffer: rejected before any access
    XY = torch.zeros(16, dtype=torch.float32, device="cuda")
    u = torch.zeros(4, dtype=torch.float64, device="cuda")
    desc = M.CostDesc(n=MAX_N + 1, d=2, kind=M.COST_POINTS_SQEUCLID, dtype=0, data=XY.data_ptr(), scale=1.0)
    with pytest.raises(M.MdotError) as e:
        ctx.lse2(desc, u, u, 1.0, u, u)
    assert e.value.code == -1


def test_solve_large_n_points_recertified_by_oracle(ctx):
    # a solve past n = 8192 (n = 9000, ragged tiles), checked by the oracle's Round and
    # certificate on the returned potentials
    n, scale = 9000, 0.5
    X, Y, r, c = _points_problem(n, 79)
    XY = dev(np.concatenate([X, Y]).ravel(), torch.float32)
    u = torch.empty(n, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    res = ctx.solve(M.point_cost(XY, n, 2, "sqeuclid", scale=scale), dev(r), dev(c), 1e-4,
                    M.default_params(precision="f32"), u, v)
    print(f"n={n} points solve: gap={res.gap:.3e} UB={res.primal_cost!r} sweeps={res.sweeps}", flush=True)
    assert res.status == 0 and 0 <= res.gap <= 1e-4
    C64 = _points_rows(X, Y, np.arange(n), scale, 0)
    ub_o, lb_o, me_o, _ = O.round_certify(C64, u.cpu().numpy(), v.cpu().numpy(), res.gamma_final, r, c)
    print(f"oracle: UB={ub_o!r} LB(u/gamma)={lb_o!r} marg_err={me_o:.2e}")
    assert res.primal_cost == pytest.approx(ub_o, rel=1e-5)
    assert res.dual_bound <= ub_o + 1e-12
    assert lb_o <= res.primal_cost + 1e-12
    assert me_o <= 1e-12


def test_engine_equals_solve_with_xcd_finalize_order(ctx):
    # n = 5120: 16 lanes per column entry and 400 finalize workgroups, so a solve alone runs
    # its finalize in the XCD-aware workgroup order; the batched finalize does not. Everything a
    # workgroup computes depends on its virtual index only, so the two must agree bit for bit.
    n = 5120
    rng = np.random.default_rng(5120)
    Cd = dev(rng.random((n, n)), torch.float32)
    r = dev(W.dirichlet_marginal(n, 11))
    c = dev(W.dirichlet_marginal(n, 12))
    prm = M.default_params(precision="f32")
    u_a = torch.empty(n, dtype=torch.float64, device="cuda")
    v_a = torch.empty_like(u_a)
    ra = ctx.solve(M.dense_cost(Cd), r, c, 1e-4, prm, u_a, v_a)
    print(f"alone n={n}: status={ra.status} gap={ra.gap:.3e} sweeps={ra.sweeps}", flush=True)
    assert ra.status == 0 and ra.gap <= 1e-4
    eng = M.Context(0)
    try:
        u_b = torch.empty_like(u_a)
        v_b = torch.empty_like(u_a)
        t = eng.submit(M.dense_cost(Cd), r, c, 1e-4, prm, u_b, v_b)
        assert t is not None
        for _ in range(100000):
            if eng.inflight()[0] == 0:
                break
            eng.run(64)
        rb = eng.poll(t)
        assert rb is not None
        assert torch.equal(u_a, u_b) and torch.equal(v_a, v_b)
        for f in ("status", "primal_cost", "dual_bound", "gap", "gamma_final", "stages", "pncg_iters", "sweeps"):
            assert getattr(rb, f) == getattr(ra, f), f
    finally:
        eng.close()


@pytest.mark.parametrize("sizes", [((20000, 83), (9000, 84)), ((9000, 85), (12000, 86))])
def test_engine_past_256_row_tiles_bitwise_equals_solve(ctx, sizes):
    # Past 256 row tiles (m > 16384) the finalize folds each entry's partials in its general
    # path; in the engine the batched finalize serves that problem beside one whose entries take
    # the 32-partial fast path. n = 20000 (313 row tiles) beside n = 9000 (141 row tiles): the
    # batch runs the finalize instance for any size, while n = 9000 alone runs the one for at
    # most 256 row tiles. n = 9000 beside n = 12000: the batch runs that instance too. The engine
    # must return each problem's solve-alone result bit for bit.
    prm = M.default_params(precision="f32")
    probs = []
    for n, seed in sizes:
        X, Y, r, c = _points_problem(n, seed)
        probs.append((n, dev(np.concatenate([X, Y]).ravel(), torch.float32), dev(r), dev(c)))
    alone = []
    for n, XY, r, c in probs:
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)
        res = ctx.solve(M.point_cost(XY, n, 2, "sqeuclid", scale=0.5), r, c, 1e-4, prm, u, v)
        print(f"alone n={n}: status={res.status} gap={res.gap:.3e} sweeps={res.sweeps}", flush=True)
        assert res.status == 0 and res.gap <= 1e-4
        alone.append((res, u.cpu(), v.cpu()))
    eng = M.Context(0)
    try:
        tickets, outs = [], []
        for n, XY, r, c in probs:
            u = torch.empty(n, dtype=torch.float64, device="cuda")
            v = torch.empty_like(u)
            t = eng.submit(M.point_cost(XY, n, 2, "sqeuclid", scale=0.5), r, c, 1e-4, prm, u, v)
            assert t is not None
            tickets.append(t)
            outs.append((u, v))
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
    finally:
        eng.close()


def test_single_point(ctx):
    C = dev(np.array([[0.375]]), torch.float64)
    one = dev(np.array([1.0]))
    res = ctx.solve(M.dense_cost(C), one, one, 1e-6)
    assert res.status == 0
    assert res.primal_cost == pytest.approx(0.375, abs=1e-12)
    assert res.dual_bound == pytest.approx(0.375, abs=1e-9)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_identical_marginals_zero_diagonal(ctx, prec):
    # r = c and C_ii = 0 <= C_ij: the identity coupling is optimal, OT = 0
    C, r, _ = W.grid_problem(16, "blobs", "l1", 21)
    Cd, rd = dev(C, torch.float32), dev(r)  # keep the device buffers alive during the call
    res = ctx.solve(M.dense_cost(Cd), rd, rd, 1e-6, M.default_params(precision=prec))
    assert res.status == 0 and res.gap <= 1e-6
    assert res.dual_bound <= 1e-12
    assert 0.0 <= res.primal_cost <= 1e-6


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_separable_cost(ctx, prec):
    # C_ij = a_i + b_j: every coupling costs <a, r> + <b, c>
    n = 300
    rng = np.random.default_rng(5)
    a, b = rng.random(n) * 0.5, rng.random(n) * 0.5
    C = a[:, None] + b[None, :]
    r = W.dirichlet_marginal(n, 7)
    c = W.dirichlet_marginal(n, 8)
    exact = float(a @ r + b @ c)
    Cd, rd, cd = dev(C, torch.float64), dev(r), dev(c)  # keep the device buffers alive during the call
    res = ctx.solve(M.dense_cost(Cd), rd, cd, 1e-8, M.default_params(precision=prec))
    assert res.status == 0
    assert res.primal_cost == pytest.approx(exact, abs=1e-10)
    assert res.dual_bound == pytest.approx(exact, abs=1e-8)
