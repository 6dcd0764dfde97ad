"""Properties of the seeded synthetic workloads (CPU): marginals on the simplex with the
stated floor, costs in [0, 1] with the stated closed-form maxima, determinism per seed."""
from __future__ import annotations

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

from paper_2307_08507_amd import workloads as W


@settings(max_examples=25, deadline=None)
@given(k=st.integers(2, 12), seed=st.integers(0, 10_000), fam=st.sampled_from(sorted(W.FAMILIES)))
def test_marginals_on_simplex(k, seed, fam):
    r = W.FAMILIES[fam](k, seed)
    assert r.shape == (k * k,)
    assert np.all(r > 0)
    assert abs(r.sum() - 1.0) < 1e-12
    np.testing.assert_array_equal(r, W.FAMILIES[fam](k, seed))  # deterministic


@pytest.mark.parametrize("k", [2, 5, 16, 64])
@pytest.mark.parametrize("kind,maxnum", [("sqeuclid", lambda k: 2 * (k - 1) ** 2), ("l1", lambda k: 2 * (k - 1))])
def test_grid_cost_range(k, kind, maxnum):
    num, mx = W.grid_cost_numerators(k, kind)
    assert mx == maxnum(k) == num.max()
    C = W.grid_cost(k, kind)
    assert C.min() == 0.0 and C.max() == 1.0
    np.testing.assert_array_equal(np.diag(C), 0.0)
    np.testing.assert_array_equal(C, C.T)
    assert np.all(num == np.round(num))  # integer numerators


def test_grid_cost_is_distance():
    k = 6
    x = W.grid_coords(k).astype(np.float64)
    C = W.grid_cost(k, "l1")
    i, j = 7, 29
    assert C[i, j] == pytest.approx((abs(x[i] - x[j]).sum()) / (2 * (k - 1)))


def test_point_cloud_and_dirichlet():
    x = W.gmm_points(500, 3, 1)
    assert x.shape == (500, 3) and x.dtype == np.float32
    r = W.dirichlet_marginal(500, 2)
    assert abs(r.sum() - 1) < 1e-12 and np.all(r > 0)
    num, mx = W.sqeuclid_cost_from_points(x[:50], x[50:100])
    assert mx == num.max() > 0


def test_serving_stream():
    reqs = W.serving_stream(20, rate=100.0, seed=3)
    assert len(reqs) == 20
    ts = [q.arrival for q in reqs]
    assert ts == sorted(ts)
    for q in reqs:
        assert 512 <= q.n <= 8192
        assert q.target in (1e-4, 1e-5, 1e-6, 1e-7)
        assert q.x.shape == (q.n, 3) and q.r.shape == (q.n,)
