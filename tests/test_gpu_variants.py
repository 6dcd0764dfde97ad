"""GPU parity of the variants the paper compares MDOT-PNCG against, each against the same
variant of the FP64 oracle: the Sinkhorn projector (Alg. 4), the diagonal-Hessian direction
with the [0.01, 100] switch (Sec. 4.3, eq. (s-tilde)), the epsilon-scaling warm start
(Sec. 4.2.1), fixed smoothing (App. D), log n in the tolerance (App. C), and the plain copy
warm start.

Workload: the n = 256 grid (16 x 16, smoothed-field marginals, squared-Euclidean cost), FP64
sweeps, the paper's schedule to a fixed gamma_f. The two FP64 paths round differently (device
exp and reduction order against libm). At this size the differences stay far inside every
decision threshold: the GPU takes the oracle's decisions exactly (stage, iteration, trial and
sweep counts, the switch between s and s~), and UB and LB agree to 1e-11 relative (measured:
about 1e-14)."""
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


def _gpu(ctx, C, r, c, target, **kw):
    Cd = dev(C, torch.float64)
    u = torch.empty(r.size, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    res = ctx.solve(M.dense_cost(Cd), dev(r), dev(c), target, M.default_params(**kw), u, v)
    return res, u.cpu().numpy(), v.cpu().numpy()


VARIANTS = {
    "sinkhorn": dict(projector=1),
    "precond": dict(precond=1),
    "eps_scaling": dict(warm_start=2),
    "copy_start": dict(warm_start=0),
    "fixed_smoothing": dict(smoothing=1),
    "log_n_tol": dict(tol_log_n=1),
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_variant_schedule_mode_matches_oracle(ctx, name):
    kw = VARIANTS[name]
    C, r, c = W.grid_problem(16, "smooth", "sqeuclid", 0)
    gf = 2.0**9
    print(f"variant {name} schedule gamma_f={gf}", flush=True)
    res, u, v = _gpu(ctx, C, r, c, 1e-4, gamma_f=gf, precision="f64", **kw)
    s = O.mdot(C, r, c, O.default_params(gamma_f=gf, **kw))
    R = s.result
    tilde_o = sum(st["tilde_iters"] for st in s.stages)
    print(f"gpu: stages={res.stages} iters={res.pncg_iters} trials={res.ls_trials} sweeps={res.sweeps} "
          f"tilde={res.tilde_iters} UB={res.primal_cost!r} LB={res.dual_bound!r}; oracle: stages={R['stages']} "
          f"iters={R['pncg_iters']} trials={R['ls_trials']} sweeps={R['sweeps']} tilde={tilde_o} "
          f"UB={R['primal_cost']!r} LB={R['dual_bound']!r}")
    assert res.status == 0 and s.status == 0
    assert res.stages == R["stages"]
    assert res.gamma_final == R["gamma_final"]
    assert (res.pncg_iters, res.ls_trials, res.sweeps) == (R["pncg_iters"], R["ls_trials"], R["sweeps"])
    assert res.tilde_iters == tilde_o
    if name == "precond":
        assert tilde_o > 0
    assert res.primal_cost == pytest.approx(R["primal_cost"], rel=1e-11)
    assert res.dual_bound == pytest.approx(R["dual_bound"], rel=1e-11)
    np.testing.assert_allclose((u[:, None] + v[None, :])[::7, ::5], (s.u[:, None] + s.v[None, :])[::7, ::5],
                               rtol=0, atol=1e-6 * gf)


def test_sinkhorn_adaptive_brackets_exact_ot(ctx):
    # the Sinkhorn projector inside the certified-gap loop, FP32 sweeps: the certificate holds
    from tests.exact_ot import exact_lp

    C, r, c = W.grid_problem(16, "blobs", "l1", 3)
    Cd = dev(C, torch.float32)
    C64 = Cd.double().cpu().numpy()
    ot = exact_lp(C64, r, c)
    u = torch.empty(r.size, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    res = ctx.solve(M.dense_cost(Cd), dev(r), dev(c), 1e-4, M.default_params(projector=1), u, v)
    print(f"sinkhorn adaptive: gap={res.gap:.3e} UB-OT={res.primal_cost - ot:.3e} sweeps={res.sweeps}")
    assert res.status == 0 and res.gap <= 1e-4
    assert res.dual_bound <= ot + 1e-12 <= res.primal_cost + 2e-12
    assert res.pncg_iters > 0 and res.ls_trials == 0


def test_variant_parameters_are_checked(ctx):
    C, r, c = W.grid_problem(8, "smooth", "sqeuclid", 0)
    for bad in (dict(projector=2), dict(precond=1, projector=1), dict(warm_start=3), dict(smoothing=-1),
                dict(tol_log_n=2)):
        with pytest.raises(M.MdotError) as e:
            _gpu(ctx, C, r, c, 1e-4, **bad)
        assert e.value.code == -1
