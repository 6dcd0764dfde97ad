"""The allocation-free LSE entry point (mdot_lse2_noalloc) against mdot_lse2.

Both run the same sweep kernels on the same tiles, so the log-sums must be bit-identical;
the first call is also checked against the FP64 oracle (tolerances as in the sweep parity
tests). Calls come in a row with shrinking n on one context, so a value the static array
kept from the previous call would show up. Sizes above the entry point's maximum are
rejected on the host before any kernel runs."""
from __future__ import annotations

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from paper_2307_08507_amd import mdot as M  # noqa: E402

NOALLOC_MAX_N = 4096


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = M.Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


def _inputs(n, seed, gamma):
    from scipy.special import logsumexp

    rng = np.random.default_rng(seed)
    C = rng.random((n, n))
    u = rng.standard_normal(n) * 0.5 - np.log(n)
    v = -np.log(n) - logsumexp(u[:, None] - gamma * C, axis=0)
    return C, u, v


def _both(ctx, cost, u, v, gamma, prec, shift=None):
    n = u.numel()
    outs = []
    for fn in (ctx.lse2, ctx.lse2_noalloc):
        lr = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        lc = torch.full_like(lr, np.nan)
        rc = fn(cost, u, v, gamma, lr, lc, shift=shift, precision=prec)
        torch.cuda.synchronize()
        outs.append((rc, lr.cpu().numpy(), lc.cpu().numpy()))
    return outs


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_noalloc_matches_lse2_two_calls(ctx, prec):
    gamma = 300.0
    # first call: the largest size it takes (n = 4096, 64 x 16 tiles), second: smaller and ragged
    for n, seed in ((NOALLOC_MAX_N, 1), (1000, 2)):
        print(f"noalloc lse2 n={n} prec={prec}", flush=True)
        C, u, v = _inputs(n, seed, gamma)
        Cd = dev(C, torch.float32 if prec == "f32" else torch.float64)
        cost = M.dense_cost(Cd)
        (rc0, lr0, lc0), (rc1, lr1, lc1) = _both(ctx, cost, dev(u), dev(v), gamma, prec)
        assert rc0 == rc1 == 0
        assert np.array_equal(lr0, lr1) and np.array_equal(lc0, lc1)
        if n == 1000:
            C64 = Cd.double().cpu().numpy()
            lr_o, lc_o = O.lse2(C64, u, v, gamma)
            tol = 1e-12 * gamma if prec == "f64" else 2e-6
            np.testing.assert_allclose(lr1, lr_o, rtol=0, atol=tol)
            np.testing.assert_allclose(lc1, lc_o, rtol=0, atol=tol)


def test_noalloc_with_shift_and_points(ctx):
    # a given shift (no row-max pass), then a smaller point cloud whose scale the call resolves
    n, gamma = 2500, 80.0
    C, u, v = _inputs(n, 5, gamma)
    Cd = dev(C, torch.float32)
    shift = torch.full((n,), float(np.log(1.0 / n)), dtype=torch.float64, device="cuda")
    print(f"noalloc lse2 with shift n={n}", flush=True)
    (rc0, lr0, lc0), (rc1, lr1, lc1) = _both(ctx, M.dense_cost(Cd), dev(u), dev(v), gamma, "f32", shift=shift)
    assert rc0 == rc1 and rc0 in (0, M.MDOT_W_RANGE)
    assert np.array_equal(lr0, lr1) and np.array_equal(lc0, lc1)
    rng = np.random.default_rng(7)
    m, d = 777, 3
    XY = dev(rng.standard_normal((2 * m, d)), torch.float32)
    cost = M.point_cost(XY, m, d, "sqeuclid", scale=0.0)
    uu = dev(rng.standard_normal(m) * 0.1 - np.log(m))
    vv = dev(rng.standard_normal(m) * 0.1 - np.log(m))
    print(f"noalloc lse2 points n={m} d={d}", flush=True)
    (rc0, lr0, lc0), (rc1, lr1, lc1) = _both(ctx, cost, uu, vv, 40.0, "f32")
    assert rc0 == rc1 == 0
    assert np.array_equal(lr0, lr1) and np.array_equal(lc0, lc1)


def test_noalloc_rejects_sizes_above_its_maximum(ctx):
    # rejected by the host-side size check: no kernel is launched
    n = NOALLOC_MAX_N + 1
    Cd = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    z = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MdotError) as ei:
        ctx.lse2_noalloc(M.dense_cost(Cd), z, z, 1.0, z.clone(), z.clone())
    assert ei.value.code == -1 and "4096" in str(ei.value)
