"""ctypes wrapper of the FP64 CPU oracle (oracle/mdot_oracle.c).

TEST INFRASTRUCTURE. Only tests, the smoke check and the CPU-baseline leg of the
benchmark may import this module. The product path never does.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdot_oracle.c")
_LIB = os.path.join(_HERE, "_build", "libmdot_oracle.so")

_dp = ct.POINTER(ct.c_double)


class Params(ct.Structure):
    _fields_ = [
        ("p", ct.c_double),
        ("q", ct.c_double),
        ("gamma_i", ct.c_double),
        ("gamma_f", ct.c_double),
        ("target_gap", ct.c_double),
        ("gamma_cap", ct.c_double),
        ("ls_c1", ct.c_double),
        ("ls_c2", ct.c_double),
        ("max_ls_trials", ct.c_int32),
        ("max_pncg_iters", ct.c_int32),
        ("max_sweeps", ct.c_int64),
        ("projector", ct.c_int32),
        ("warm_start", ct.c_int32),
        ("precond", ct.c_int32),
        ("smoothing", ct.c_int32),
        ("tol_log_n", ct.c_int32),
        ("pad_", ct.c_int32),
    ]


class Result(ct.Structure):
    _fields_ = [
        ("primal_cost", ct.c_double),
        ("dual_bound", ct.c_double),
        ("gap", ct.c_double),
        ("gamma_final", ct.c_double),
        ("marg_err_l1", ct.c_double),
        ("grad_norm", ct.c_double),
        ("stages", ct.c_int32),
        ("status", ct.c_int32),
        ("pncg_iters", ct.c_int64),
        ("ls_trials", ct.c_int64),
        ("sweeps", ct.c_int64),
        ("cg_resets", ct.c_int64),
        ("ls_failures", ct.c_int64),
    ]


class StageLog(ct.Structure):
    _fields_ = [
        ("gamma", ct.c_double),
        ("eps_d", ct.c_double),
        ("smooth_w", ct.c_double),
        ("grad_norm", ct.c_double),
        ("ub", ct.c_double),
        ("lb", ct.c_double),
        ("grad_norm0", ct.c_double),
        ("pncg_iters", ct.c_int64),
        ("ls_trials", ct.c_int64),
        ("sweeps", ct.c_int64),
        ("cg_resets", ct.c_int64),
        ("tilde_iters", ct.c_int64),
    ]


# -O3 for the AVX2/FMA subset every current x86-64 server has (x86-64-v3): the library is built
# on one machine and run on another, so -march=native could emit instructions the other lacks.
# -ffp-contract=off keeps every a*b+c a rounded product and a rounded sum, as written: no FMA
# contraction changes the oracle's arithmetic.
CFLAGS = ["-O3", "-march=x86-64-v3", "-ffp-contract=off", "-std=c11", "-fopenmp", "-fPIC"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (CFLAGS, OpenMP over independent rows and columns)."""
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", *CFLAGS, "-shared", "-o", _LIB, _SRC, "-lm"])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ct.CDLL(_LIB)
        L.orc_default_params.argtypes = [ct.POINTER(Params)]
        L.orc_entropy.restype = ct.c_double
        L.orc_entropy.argtypes = [ct.c_int, _dp]
        L.orc_lse2.argtypes = [ct.c_int, ct.c_int, _dp, _dp, _dp, ct.c_double, _dp, _dp]
        L.orc_dual_objective.restype = ct.c_double
        L.orc_dual_objective.argtypes = [ct.c_int, ct.c_int, _dp, _dp, _dp, ct.c_double, _dp, _dp]
        L.orc_round.argtypes = [ct.c_int, ct.c_int, _dp, _dp, _dp, _dp]
        L.orc_ctransform_bound.restype = ct.c_double
        L.orc_ctransform_bound.argtypes = [ct.c_int, ct.c_int, _dp, _dp, _dp, _dp, _dp]
        L.orc_round_certify.restype = ct.c_int
        L.orc_round_certify.argtypes = [ct.c_int, ct.c_int, _dp, _dp, _dp, ct.c_double, _dp, _dp, ct.c_double,
                                        _dp, _dp, _dp, _dp, _dp, _dp]
        L.orc_project.restype = ct.c_int
        L.orc_project.argtypes = [ct.c_int, ct.c_int, _dp, ct.c_double, _dp, _dp, ct.c_double, _dp,
                                  ct.POINTER(Params), ct.POINTER(ct.c_int64), _dp]
        L.orc_mdot.restype = ct.c_int
        L.orc_mdot.argtypes = [ct.c_int, ct.c_int, _dp, _dp, _dp, ct.POINTER(Params), _dp, _dp,
                               ct.POINTER(Result), ct.POINTER(StageLog), ct.c_int]
        L.orc_num_threads.restype = ct.c_int
        L.orc_set_num_threads.argtypes = [ct.c_int]
        L.orc_set_ls_log.argtypes = [_dp, ct.c_int64]
        L.orc_ls_log_count.restype = ct.c_int64
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(k: int) -> None:
    """Threads of the oracle's parallel loops (k < 1: the OpenMP default)."""
    lib().orc_set_num_threads(int(k))


class LineSearchLog:
    """Context manager recording every accepted line-search step of the oracle as rows
    (phi'(0), phi'(alpha), alpha, how); how = 0 for an approximate-Wolfe acceptance, 1 for the
    trial cap's fallback to alpha_lo."""

    def __init__(self, cap: int = 1 << 20):
        self.buf = np.zeros((cap, 4))

    def __enter__(self):
        lib().orc_set_ls_log(_d(self.buf), self.buf.shape[0])
        return self

    def __exit__(self, *exc):
        self.count = int(lib().orc_ls_log_count())
        lib().orc_set_ls_log(None, 0)
        self.rows = self.buf[:min(self.count, self.buf.shape[0])].copy()
        return False


def default_params(**kw) -> Params:
    p = Params()
    lib().orc_default_params(ct.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def entropy(r) -> float:
    r = _f64(r)
    return lib().orc_entropy(r.size, _d(r))


def _shape(C, r=None, c=None):
    """(m, n) of an m x n cost (rows follow r, columns follow c)."""
    if C.ndim != 2:
        raise ValueError("C must be a matrix")
    m, n = C.shape
    if (r is not None and r.size != m) or (c is not None and c.size != n):
        raise ValueError("marginal sizes do not match the cost")
    return m, n


def lse2(C, u, v, gamma: float):
    """(log r(P), log c(P)) of P = exp(u_i + v_j - gamma C_ij), FP64 two-pass; C is m x n."""
    C, u, v = _f64(C), _f64(u), _f64(v)
    m, n = _shape(C, u, v)
    lr = np.empty(m)
    lc = np.empty(n)
    lib().orc_lse2(m, n, _d(C), _d(u), _d(v), float(gamma), _d(lr), _d(lc))
    return lr, lc


def dual_objective(C, u, v, gamma, r, c) -> float:
    C, u, v, r, c = map(_f64, (C, u, v, r, c))
    m, n = _shape(C, r, c)
    return lib().orc_dual_objective(m, n, _d(C), _d(u), _d(v), float(gamma), _d(r), _d(c))


def round_plan(P, r, c) -> np.ndarray:
    P, r, c = _f64(P), _f64(r), _f64(c)
    m, n = _shape(P, r, c)
    G = np.empty((m, n))
    lib().orc_round(m, n, _d(P), _d(r), _d(c), _d(G))
    return G


def ctransform_bound(C, f, g, r, c) -> float:
    C, f, g, r, c = map(_f64, (C, f, g, r, c))
    m, n = _shape(C, r, c)
    return lib().orc_ctransform_bound(m, n, _d(C), _d(f), _d(g), _d(r), _d(c))


def round_certify(C, u, v, gamma, r, c, want_plan: bool = False, u_prev=None, v_prev=None,
                  gamma_prev: float = 0.0):
    """(UB, LB, marginal error, G or None) for the plan P(u, v; gamma)."""
    C, u, v, r, c = map(_f64, (C, u, v, r, c))
    m, n = _shape(C, r, c)
    ub, lb, me = ct.c_double(), ct.c_double(), ct.c_double()
    G = np.empty((m, n)) if want_plan else None
    up = _f64(u_prev) if u_prev is not None else None
    vp = _f64(v_prev) if v_prev is not None else None
    rc = lib().orc_round_certify(m, n, _d(C), _d(u), _d(v), float(gamma), _d(up) if up is not None else None,
                                 _d(vp) if vp is not None else None, float(gamma_prev), _d(r), _d(c), ct.byref(ub),
                                 ct.byref(lb), ct.byref(me), _d(G) if want_plan else None)
    if rc != 0:
        raise RuntimeError(f"orc_round_certify failed: {rc}")
    return ub.value, lb.value, me.value, G


def project(C, gamma, rt, ct_, tol, u, v, params: Params | None = None):
    """KL projection at fixed gamma (PNCG, or Sinkhorn with params.projector=1).
    Returns (u, v, status, counts[pncg_iters, ls_trials, sweeps, cg_resets, ls_failures, tilde_iters], gnorm)."""
    C, rt, ct_ = _f64(C), _f64(rt), _f64(ct_)
    m, n = _shape(C, rt, ct_)
    z = np.concatenate([_f64(u), _f64(v)])
    prm = params or default_params()
    counts = (ct.c_int64 * 6)()
    gn = ct.c_double()
    st = lib().orc_project(m, n, _d(C), float(gamma), _d(rt), _d(ct_), float(tol), _d(z), ct.byref(prm),
                           counts, ct.byref(gn))
    return z[:m].copy(), z[m:].copy(), st, list(counts), gn.value


@dataclass
class Solve:
    u: np.ndarray
    v: np.ndarray
    status: int
    result: dict
    stages: list


def mdot(C, r, c, params: Params | None = None, max_stages: int = 256) -> Solve:
    """Run MDOT (Alg. 1) on an m x n cost; returns potentials, status, result, stage log."""
    C, r, c = _f64(C), _f64(r), _f64(c)
    m, n = _shape(C, r, c)
    prm = params or default_params()
    u = np.zeros(m)
    v = np.zeros(n)
    res = Result()
    logs = (StageLog * max_stages)()
    st = lib().orc_mdot(m, n, _d(C), _d(r), _d(c), ct.byref(prm), _d(u), _d(v), ct.byref(res), logs,
                        max_stages)
    rd = {f: getattr(res, f) for f, _ in Result._fields_}
    stages = [{f: getattr(logs[k], f) for f, _ in StageLog._fields_} for k in range(min(res.stages, max_stages))]
    return Solve(u, v, st, rd, stages)
