"""Python binding of libmdot (include/mdot.h): argument marshalling only.

Every step of the solve runs in the HIP library; this module turns torch tensors into
device pointers and the current torch stream into the library's HIP stream. It raises
if the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libmdot.so")

MDOT_OK = 0
MDOT_W_NOT_CONVERGED = 1
MDOT_W_RANGE = 2
ERRORS = {-1: "MDOT_E_ARG", -2: "MDOT_E_MARGINAL", -3: "MDOT_E_COST", -4: "MDOT_E_NOMEM",
          -5: "MDOT_E_DEVICE", -6: "MDOT_E_BUSY"}

COST_DENSE, COST_POINTS_SQEUCLID, COST_POINTS_L1 = 0, 1, 2
DT_F64, DT_F32, DT_F16, DT_BF16 = 0, 1, 2, 3
PREC_F64, PREC_F32, PREC_MIXED = 0, 1, 2


class CostDesc(ct.Structure):
    _fields_ = [("n", ct.c_int32), ("d", ct.c_int32), ("kind", ct.c_int), ("dtype", ct.c_int),
                ("data", ct.c_void_p), ("scale", ct.c_double), ("m", ct.c_int32), ("reserved", ct.c_int32)]


class Params(ct.Structure):
    _fields_ = [("p", ct.c_double), ("q", ct.c_double), ("gamma_i", ct.c_double), ("gamma_f", ct.c_double),
                ("gamma_cap", ct.c_double), ("ls_c1", ct.c_double), ("ls_c2", ct.c_double),
                ("max_ls_trials", ct.c_int32), ("max_pncg_iters", ct.c_int32), ("max_sweeps", ct.c_int64),
                ("precision", ct.c_int), ("warm_start", ct.c_int32), ("mixed_switch", ct.c_double),
                ("projector", ct.c_int32), ("precond", ct.c_int32), ("smoothing", ct.c_int32),
                ("tol_log_n", ct.c_int32)]


class Result(ct.Structure):
    _fields_ = [("primal_cost", ct.c_double), ("dual_bound", ct.c_double), ("gap", ct.c_double),
                ("gamma_final", ct.c_double), ("marg_err_l1", ct.c_double), ("grad_norm", ct.c_double),
                ("seconds", ct.c_double), ("stages", ct.c_int32), ("status", ct.c_int32),
                ("pncg_iters", ct.c_int64), ("ls_trials", ct.c_int64), ("sweeps", ct.c_int64),
                ("cg_resets", ct.c_int64), ("ls_failures", ct.c_int64), ("fp64_retries", ct.c_int64),
                ("cert_sweeps", ct.c_int64), ("prec_switches", ct.c_int64), ("proxy_stages", ct.c_int64),
                ("tilde_iters", ct.c_int64)]


class MdotError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libmdot.so; raise when it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2307_08507_amd.build_lib`")
        L = ct.CDLL(LIB_PATH)
        vp, dp = ct.c_void_p, ct.c_void_p
        L.mdot_version.restype = ct.c_char_p
        L.mdot_default_params.argtypes = [ct.POINTER(Params)]
        L.mdot_last_error.restype = ct.c_char_p
        L.mdot_last_error.argtypes = [vp]
        L.mdot_ctx_create.argtypes = [ct.c_int, vp, ct.c_size_t, ct.POINTER(vp)]
        L.mdot_ctx_destroy.argtypes = [vp]
        L.mdot_solve.argtypes = [vp, ct.POINTER(CostDesc), dp, dp, ct.c_double, ct.POINTER(Params), dp, dp,
                                 ct.POINTER(Result)]
        L.mdot_lse2.argtypes = [vp, ct.POINTER(CostDesc), dp, dp, ct.c_double, dp, ct.c_int, dp, dp]
        L.mdot_lse2_noalloc.argtypes = [vp, ct.POINTER(CostDesc), dp, dp, ct.c_double, dp, ct.c_int, dp, dp]
        L.mdot_round_certify.argtypes = [vp, ct.POINTER(CostDesc), dp, dp, ct.c_double, dp, dp, ct.c_double,
                                         dp, dp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double),
                                         ct.POINTER(ct.c_double)]
        L.mdot_bench_sweep.argtypes = [vp, ct.POINTER(CostDesc), dp, dp, ct.c_double, ct.c_int, ct.c_int,
                                       ct.POINTER(ct.c_double)]
        L.mdot_bench_sweep_flushed.argtypes = [vp, ct.POINTER(CostDesc), dp, dp, ct.c_double, ct.c_int, ct.c_int,
                                               vp, ct.c_size_t, ct.POINTER(ct.c_double)]
        L.mdot_tune_override.argtypes = [vp, ct.c_int, ct.c_int]
        L.mdot_tune_variant.argtypes = [vp, ct.POINTER(CostDesc), ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)]
        L.mdot_submit.argtypes = [vp, ct.POINTER(CostDesc), dp, dp, ct.c_double, ct.POINTER(Params), dp, dp,
                                  ct.POINTER(ct.c_uint64)]
        L.mdot_run.argtypes = [vp, ct.c_int, ct.POINTER(ct.c_int)]
        L.mdot_poll.argtypes = [vp, ct.c_uint64, ct.c_int, ct.POINTER(Result)]
        L.mdot_inflight.argtypes = [vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_size_t)]
        _lib = L
    return _lib


def version() -> str:
    return lib().mdot_version().decode()


def default_params(**kw) -> Params:
    p = Params()
    lib().mdot_default_params(ct.byref(p))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"f32": PREC_F32, "f64": PREC_F64, "mixed": PREC_MIXED}[v]
        setattr(p, k, v)
    return p


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


_DTYPES = None


def _dtype_code(t) -> int:
    global _DTYPES
    import torch

    if _DTYPES is None:
        _DTYPES = {torch.float64: DT_F64, torch.float32: DT_F32, torch.float16: DT_F16, torch.bfloat16: DT_BF16}
    return _DTYPES[t.dtype]


def dense_cost(C, scale: float = 1.0) -> CostDesc:
    """Descriptor of a dense m x n cost tensor (device, contiguous, f64/f32/f16/bf16): row i is
    source i (marginal r), column j target j (marginal c)."""
    assert C.is_cuda and C.dim() == 2 and C.is_contiguous()
    desc = CostDesc(n=C.shape[1], m=C.shape[0], d=0, kind=COST_DENSE, dtype=_dtype_code(C), data=C.data_ptr(),
                    scale=scale)
    desc._tensor = C  # the descriptor holds a raw pointer: keep the tensor alive with it
    return desc


def point_cost(XY, n: int, d: int, kind: str = "sqeuclid", scale: float = 0.0, m: int | None = None) -> CostDesc:
    """Descriptor of a point-cloud cost: XY is a contiguous FP32 device tensor holding X (m x d,
    the sources; m = n unless given) followed by Y (n x d, the targets). scale 0 lets the library
    normalise by the largest pairwise value."""
    import torch

    m = n if m is None else m
    assert XY.is_cuda and XY.dtype == torch.float32 and XY.is_contiguous() and XY.numel() == (m + n) * d
    k = COST_POINTS_SQEUCLID if kind == "sqeuclid" else COST_POINTS_L1
    desc = CostDesc(n=n, m=m, d=d, kind=k, dtype=DT_F32, data=XY.data_ptr(), scale=scale)
    desc._tensor = XY  # the descriptor holds a raw pointer: keep the tensor alive with it
    return desc


@dataclass
class SolveResult:
    status: int
    primal_cost: float
    dual_bound: float
    gap: float
    gamma_final: float
    marg_err_l1: float
    grad_norm: float
    seconds: float
    stages: int
    pncg_iters: int
    ls_trials: int
    sweeps: int
    cg_resets: int
    ls_failures: int
    fp64_retries: int
    cert_sweeps: int
    prec_switches: int
    proxy_stages: int
    tilde_iters: int


class Context:
    """An mdot context bound to one device and the torch stream current at creation."""

    def __init__(self, device: int = 0, stream=None, hbm_budget_bytes: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible")
        self.device = device
        with torch.cuda.device(device):
            s = stream if stream is not None else torch.cuda.current_stream(device)
        self.stream = s
        h = ct.c_void_p()
        rc = lib().mdot_ctx_create(device, ct.c_void_p(s.cuda_stream), hbm_budget_bytes, ct.byref(h))
        if rc != 0:
            raise MdotError(rc, "mdot_ctx_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().mdot_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, allow=(MDOT_OK, MDOT_W_NOT_CONVERGED, MDOT_W_RANGE)) -> int:
        if rc not in allow:
            raise MdotError(rc, lib().mdot_last_error(self._h).decode())
        return rc

    def solve(self, cost: CostDesc, r, c, target_gap: float = 1e-6, params: Params | None = None,
              u_out=None, v_out=None) -> SolveResult:
        res = Result()
        rc = lib().mdot_solve(self._h, ct.byref(cost), _ptr(r), _ptr(c), float(target_gap),
                              ct.byref(params) if params is not None else None, _ptr(u_out), _ptr(v_out),
                              ct.byref(res))
        self._check(rc)
        return SolveResult(status=rc, **{f: getattr(res, f) for f, _ in Result._fields_ if f != "status"})

    def lse2(self, cost: CostDesc, u, v, gamma: float, lr_out, lc_out, shift=None, precision: str = "f32") -> int:
        prec = PREC_F64 if precision == "f64" else PREC_F32
        rc = lib().mdot_lse2(self._h, ct.byref(cost), _ptr(u), _ptr(v), float(gamma), _ptr(shift), prec,
                             _ptr(lr_out), _ptr(lc_out))
        return self._check(rc)

    def lse2_noalloc(self, cost: CostDesc, u, v, gamma: float, lr_out, lc_out, shift=None,
                     precision: str = "f32") -> int:
        """mdot_lse2 without device allocation (n <= MDOT_NOALLOC_MAX_N = 4096)."""
        prec = PREC_F64 if precision == "f64" else PREC_F32
        rc = lib().mdot_lse2_noalloc(self._h, ct.byref(cost), _ptr(u), _ptr(v), float(gamma), _ptr(shift), prec,
                                     _ptr(lr_out), _ptr(lc_out))
        return self._check(rc)

    # ---- serving: continuous batching
    def submit(self, cost: CostDesc, r, c, target_gap: float = 1e-6, params: Params | None = None,
               u_out=None, v_out=None) -> int | None:
        """Admit one solve; returns its ticket, or None when no slot / HBM budget is free."""
        t = ct.c_uint64()
        rc = lib().mdot_submit(self._h, ct.byref(cost), _ptr(r), _ptr(c), float(target_gap),
                               ct.byref(params) if params is not None else None, _ptr(u_out), _ptr(v_out),
                               ct.byref(t))
        if rc == -6:
            return None
        self._check(rc)
        return t.value

    def run(self, steps: int = 8) -> int:
        """Advance all solves in flight; returns how many finished."""
        nd = ct.c_int()
        self._check(lib().mdot_run(self._h, int(steps), ct.byref(nd)))
        return nd.value

    def poll(self, ticket: int, wait: bool = False) -> SolveResult | None:
        res = Result()
        rc = lib().mdot_poll(self._h, ct.c_uint64(ticket), 1 if wait else 0, ct.byref(res))
        if rc == 2:
            return None
        self._check(rc)
        return SolveResult(status=res.status, **{f: getattr(res, f) for f, _ in Result._fields_ if f != "status"})

    def inflight(self) -> tuple[int, int]:
        a, b = ct.c_int(), ct.c_size_t()
        self._check(lib().mdot_inflight(self._h, ct.byref(a), ct.byref(b)))
        return a.value, b.value

    def bench_sweep(self, cost: CostDesc, u, v, gamma: float, precision: str = "f32", iters: int = 100) -> float:
        """Mean milliseconds per fused LSE sweep (HIP events on the context stream)."""
        ms = ct.c_double()
        prec = PREC_F64 if precision == "f64" else PREC_F32
        rc = lib().mdot_bench_sweep(self._h, ct.byref(cost), _ptr(u), _ptr(v), float(gamma), prec, int(iters),
                                    ct.byref(ms))
        self._check(rc)
        return ms.value

    def bench_sweep_flushed(self, cost: CostDesc, u, v, gamma: float, flush, precision: str = "f32",
                            iters: int = 20) -> float:
        """Mean milliseconds per fused LSE sweep, each timed alone after reading `flush` (a device
        tensor larger than the last-level cache) to evict the cost from the caches."""
        ms = ct.c_double()
        prec = PREC_F64 if precision == "f64" else PREC_F32
        rc = lib().mdot_bench_sweep_flushed(self._h, ct.byref(cost), _ptr(u), _ptr(v), float(gamma), prec,
                                            int(iters), flush.data_ptr(), flush.numel() * flush.element_size(),
                                            ct.byref(ms))
        self._check(rc)
        return ms.value

    def tune_override(self, occ: int = 0, stage: int = -1) -> None:
        """Force a sweep launch variant (occ 2 or 4, stage 0/1) for later calls; 0/-1: the table's."""
        self._check(lib().mdot_tune_override(self._h, int(occ), int(stage)))

    def tune_variant(self, cost: CostDesc) -> tuple[int, int]:
        """(waves per SIMD, staging threshold in tiles) a call on `cost` takes."""
        o, s = ct.c_int(), ct.c_int()
        self._check(lib().mdot_tune_variant(self._h, ct.byref(cost), ct.byref(o), ct.byref(s)))
        return o.value, s.value

    def round_certify(self, cost: CostDesc, u, v, gamma: float, r, c, u_prev=None, v_prev=None,
                      gamma_prev: float = 0.0):
        ub, lb, me = ct.c_double(), ct.c_double(), ct.c_double()
        rc = lib().mdot_round_certify(self._h, ct.byref(cost), _ptr(u), _ptr(v), float(gamma), _ptr(u_prev),
                                      _ptr(v_prev), float(gamma_prev), _ptr(r), _ptr(c), ct.byref(ub),
                                      ct.byref(lb), ct.byref(me))
        self._check(rc)
        return ub.value, lb.value, me.value
