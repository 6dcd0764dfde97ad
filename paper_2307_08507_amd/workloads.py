"""Seeded synthetic OT workloads (inputs only; none of the solver's arithmetic).

Both the HIP path and the CPU oracle take their inputs from here, so this module
holds input construction only: grids, point clouds, cost matrices and marginals.

The paper benchmarks on upsampled MNIST, DOTmark and DALL-E colour-transfer images
(Sec. 5.1, App. H); none of them is available here. The families below stand in
for them at the same sizes and cost definitions:

* cost: L1 or squared-L2 distance between pixel locations of a k x k grid,
  divided by its maximum so C lies in [0, 1] (Sec. 5.1); point-cloud costs use the
  squared Euclidean distance between 3-D points divided by the maximum over pairs
  (the synthetic generator of App. C uses the same construction);
* marginals: uniform-random pixels (a white-noise image), Gaussian-smoothed random
  fields (smooth random images), sums of 1-5 Gaussian blobs, heavy-tailed Cauchy
  blobs; point-cloud marginals are Dirichlet(1) weights.

Every generator takes an explicit seed and uses numpy's default_rng.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

FLOOR = 1e-6  # added to every pixel intensity before normalising


def grid_coords(k: int) -> np.ndarray:
    """Integer pixel coordinates of a k x k grid, row-major, shape (k*k, 2), float32."""
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    return np.stack([ii.ravel(), jj.ravel()], axis=1).astype(np.float32)


def grid_cost_numerators(k: int, kind: str) -> tuple[np.ndarray, float]:
    """Integer cost numerators between pixels of a k x k grid and their maximum.

    kind = "sqeuclid": (di^2 + dj^2), max 2 (k-1)^2;  kind = "l1": |di| + |dj|, max 2 (k-1).
    Returns (numerators as float64 (n, n), max).
    """
    x = grid_coords(k).astype(np.float64)
    d = x[:, None, :] - x[None, :, :]
    if kind == "sqeuclid":
        num = (d * d).sum(-1)
        mx = 2.0 * (k - 1) ** 2
    elif kind == "l1":
        num = np.abs(d).sum(-1)
        mx = 2.0 * (k - 1)
    else:
        raise ValueError(f"unknown grid cost kind {kind!r}")
    return num, mx


def grid_cost(k: int, kind: str, dtype=np.float64) -> np.ndarray:
    """Normalised grid cost C = numerator / max, entries in [0, 1], shape (k*k, k*k)."""
    num, mx = grid_cost_numerators(k, kind)
    if mx == 0:
        return np.zeros_like(num, dtype=dtype)
    return (num / mx).astype(dtype)


def _gauss_kernel(sigma: float, truncate: float = 4.0) -> np.ndarray:
    rad = int(truncate * sigma + 0.5)
    x = np.arange(-rad, rad + 1, dtype=np.float64)
    w = np.exp(-0.5 * (x / sigma) ** 2)
    return w / w.sum()


def _blur(img: np.ndarray, sigma: float) -> np.ndarray:
    """Separable Gaussian blur with reflect boundary (truncated at 4 sigma)."""
    w = _gauss_kernel(sigma)
    rad = (len(w) - 1) // 2
    out = img
    for axis in (0, 1):
        pad = [(0, 0), (0, 0)]
        pad[axis] = (rad, rad)
        p = np.pad(out, pad, mode="symmetric")
        acc = np.zeros_like(out)
        for t, wt in enumerate(w):
            sl = [slice(None), slice(None)]
            sl[axis] = slice(t, t + out.shape[axis])
            acc += wt * p[tuple(sl)]
        out = acc
    return out


def _normalise(img: np.ndarray) -> np.ndarray:
    a = np.abs(np.asarray(img, dtype=np.float64)).ravel() + FLOOR
    return a / a.sum()


def smoothed_field(k: int, seed: int, sigma: float = 2.0) -> np.ndarray:
    """N(0,1) field on a k x k grid, Gaussian-smoothed (sigma px), abs, +floor, normalised."""
    rng = np.random.default_rng(seed)
    return _normalise(_blur(rng.standard_normal((k, k)), sigma))


def uniform_random(k: int, seed: int) -> np.ndarray:
    """Independent U(0,1) pixel intensities (+floor), normalised."""
    rng = np.random.default_rng(seed)
    return _normalise(rng.random((k, k)))


def gaussian_blobs(k: int, seed: int) -> np.ndarray:
    """Sum of K ~ U{1..5} isotropic Gaussian blobs; centres U[0,k)^2, sigma ~ U[2,12] px
    (scaled by k/64), weights U[0.5, 1]."""
    rng = np.random.default_rng(seed)
    kk = int(rng.integers(1, 6))
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    img = np.zeros((k, k))
    s = k / 64.0
    for _ in range(kk):
        ci, cj = rng.random(2) * k
        sig = rng.uniform(2.0, 12.0) * s
        wt = rng.uniform(0.5, 1.0)
        img += wt * np.exp(-0.5 * ((ii - ci) ** 2 + (jj - cj) ** 2) / sig**2)
    return _normalise(img)


def cauchy_blobs(k: int, seed: int) -> np.ndarray:
    """Sum of K ~ U{1..5} heavy-tailed blobs with profile (1 + d^2/s^2)^(-3/2),
    s ~ U[1, 6] px (scaled by k/64), weights U[0.5, 1]."""
    rng = np.random.default_rng(seed)
    kk = int(rng.integers(1, 6))
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    img = np.zeros((k, k))
    s0 = k / 64.0
    for _ in range(kk):
        ci, cj = rng.random(2) * k
        s = rng.uniform(1.0, 6.0) * s0
        wt = rng.uniform(0.5, 1.0)
        img += wt * (1.0 + ((ii - ci) ** 2 + (jj - cj) ** 2) / s**2) ** -1.5
    return _normalise(img)


FAMILIES = {
    "uniform": uniform_random,
    "smooth": smoothed_field,
    "blobs": gaussian_blobs,
    "cauchy": cauchy_blobs,
}


def grid_problem(k: int, family: str, cost: str, seed: int, dtype=np.float64):
    """One OT problem on a k x k grid: (C, r, c) with r, c from `family` (seeds seed, seed+1)."""
    gen = FAMILIES[family]
    r = gen(k, seed)
    c = gen(k, seed + 1)
    return grid_cost(k, cost, dtype), r, c


def grid_pair_problem(k1: int, k2: int, family: str, cost: str, seed: int, dtype=np.float64):
    """A rectangular OT problem between images of two resolutions: r on a k1 x k1 grid, c on a
    k2 x k2 grid (both from `family`, seeds seed and seed + 1), pixel centres placed in the unit
    square ((i + 1/2) / k), cost = squared-Euclidean or L1 distance between centres divided by its
    maximum. Returns (C of shape (k1^2, k2^2), r, c)."""
    gen = FAMILIES[family]
    r = gen(k1, seed)
    c = gen(k2, seed + 1)
    x = (grid_coords(k1).astype(np.float64) + 0.5) / k1
    y = (grid_coords(k2).astype(np.float64) + 0.5) / k2
    d = x[:, None, :] - y[None, :, :]
    if cost == "sqeuclid":
        num = (d * d).sum(-1)
    elif cost == "l1":
        num = np.abs(d).sum(-1)
    else:
        raise ValueError(f"unknown grid cost kind {cost!r}")
    return (num / num.max()).astype(dtype), r, c


def grid_problem_marginals(k: int, family: str, seed: int) -> np.ndarray:
    """The marginal `grid_problem` draws from `family` with `seed` (the cost is formed apart)."""
    return FAMILIES[family](k, seed)


def gmm_points(n: int, d: int, seed: int) -> np.ndarray:
    """n points in R^d from a K ~ U{1..8}-component Gaussian mixture: means N(0, 4 I),
    covariances A A^T / 3 + 0.1 I, equal component weights. float32 (n, d)."""
    rng = np.random.default_rng(seed)
    kk = int(rng.integers(1, 9))
    means = rng.standard_normal((kk, d)) * 2.0
    covs = []
    for _ in range(kk):
        a = rng.standard_normal((d, d))
        covs.append(a @ a.T / 3.0 + 0.1 * np.eye(d))
    comp = rng.integers(0, kk, size=n)
    pts = np.empty((n, d))
    for t in range(kk):
        idx = np.nonzero(comp == t)[0]
        if idx.size:
            pts[idx] = rng.multivariate_normal(means[t], covs[t], size=idx.size)
    return pts.astype(np.float32)


def dirichlet_marginal(n: int, seed: int) -> np.ndarray:
    """Dirichlet(1_n) weights (float64), floored and renormalised."""
    rng = np.random.default_rng(seed)
    w = rng.dirichlet(np.ones(n)) + 1e-12
    return w / w.sum()


def sqeuclid_cost_from_points(x: np.ndarray, y: np.ndarray) -> tuple[np.ndarray, float]:
    """Squared Euclidean cost between point sets (float64) and its maximum over pairs."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = x[:, None, :] - y[None, :, :]
    num = (d * d).sum(-1)
    return num, float(num.max())


@dataclass
class Request:
    """One serving request: arrival time (s), size, point clouds, marginals, target."""

    arrival: float
    n: int
    x: np.ndarray
    y: np.ndarray
    r: np.ndarray
    c: np.ndarray
    target: float
    seed: int


def serving_stream(num: int, rate: float, seed: int, n_lo: int = 512, n_hi: int = 8192, d: int = 3):
    """Poisson arrivals at `rate` per second; n = round(exp(U(ln n_lo, ln n_hi)));
    3-D GMM point clouds; Dirichlet(1) marginals; target gap uniform over
    {1e-4, 1e-5, 1e-6, 1e-7}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    targets = (1e-4, 1e-5, 1e-6, 1e-7)
    for k in range(num):
        t += rng.exponential(1.0 / rate)
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        s = int(seed * 100003 + k * 7 + 1)
        out.append(
            Request(
                arrival=t,
                n=n,
                x=gmm_points(n, d, s),
                y=gmm_points(n, d, s + 1),
                r=dirichlet_marginal(n, s + 2),
                c=dirichlet_marginal(n, s + 3),
                target=float(targets[int(rng.integers(0, 4))]),
                seed=s,
            )
        )
    return out
