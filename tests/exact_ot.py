"""Exact OT references used to pin the oracle (test infrastructure).

* exact_lp: the transportation LP min <P, C> s.t. P1 = r, P^T 1 = c, P >= 0, solved by
  scipy's HiGHS (an independent library, run here, not copied).
* birkhoff: for uniform marginals the optimum is attained at a permutation matrix
  (Birkhoff-von Neumann), so OT = min over permutations of mean C_{i, sigma(i)}.
* monotone_1d: on the real line with a convex cost of |x - y| the monotone (north-west
  corner on sorted supports) coupling is optimal.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
from scipy.optimize import linprog


def exact_lp(C, r, c) -> float:
    C = np.asarray(C, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    c = c * (r.sum() / c.sum())
    n, m = C.shape
    # the n + m equalities have rank n + m - 1: drop the last column constraint, which the
    # others imply, so rounding in the sums cannot make the system look inconsistent
    A = sp.vstack([sp.kron(sp.eye(n), np.ones((1, m))), sp.kron(np.ones((1, n)), sp.eye(m))]).tocsr()[:-1]
    res = linprog(C.ravel(), A_eq=A, b_eq=np.concatenate([r, c])[:-1], bounds=(0, None), method="highs")
    assert res.status == 0, res.message
    return float(res.fun)


def birkhoff(C) -> float:
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    best = np.inf
    idx = np.arange(n)
    for perm in itertools.permutations(range(n)):
        best = min(best, C[idx, list(perm)].sum() / n)
    return best


def monotone_1d(x, r, y, c, power: float) -> float:
    """Cost of the monotone coupling between (x, r) and (y, c) for |x - y|^power."""
    ox, oy = np.argsort(x, kind="stable"), np.argsort(y, kind="stable")
    xs, rs = np.asarray(x, dtype=np.float64)[ox], np.asarray(r, dtype=np.float64)[ox].copy()
    ys, cs = np.asarray(y, dtype=np.float64)[oy], np.asarray(c, dtype=np.float64)[oy].copy()
    cs *= rs.sum() / cs.sum()
    i = j = 0
    total = 0.0
    while i < len(xs) and j < len(ys):
        m = min(rs[i], cs[j])
        total += m * abs(xs[i] - ys[j]) ** power
        rs[i] -= m
        cs[j] -= m
        if rs[i] <= cs[j]:
            i += 1
        else:
            j += 1
    return total
