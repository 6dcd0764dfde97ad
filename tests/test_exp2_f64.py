"""Pin of the FP64 exponential the F64 sweeps use (exp2_f64 in mdot_kernels.hip), on the CPU.

2^x = 2^k * 2^f with k = round(x), |f| <= 1/2 and 2^f = 1 + f q(f), q of degree 9. The
coefficients are the kernel's own fit (weighted least squares driven to equal ripple), not a
library's. Checked here against 2^f in 60-digit arithmetic (mpmath):
  * the polynomial with the committed FP64 coefficients, evaluated exactly, has a relative
    error below 4e-16 on [-1/2, 1/2] (the bound the kernel's comment states);
  * the kernel's FP64 Horner evaluation (fused multiply-adds, each rounded once) stays within
    4 ulp of 2^f;
  * the scalar and the four-way versions use the same coefficients in the same order.
"""
from __future__ import annotations

import os
import re

import numpy as np
import pytest

mpmath = pytest.importorskip("mpmath")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2307_08507_amd", "csrc", "mdot_kernels.hip")


def _coefficients():
    src = open(SRC).read()
    c9 = float.fromhex(re.search(r"kExp2C9 = (0x[0-9a-fp.+-]+);", src).group(1))
    body = src[src.index("double exp2_f64(double x, double c9)"):]
    body = body[:body.index("\n}\n")]
    scalar = [float.fromhex(h) for h in re.findall(r"fma_sc\([^;]*?(0x[0-9a-fp.+-]+)\)", body)]
    body4 = src[src.index("void exp2_f64x4("):]
    body4 = body4[:body4.index("\n}\n")]
    four = [float.fromhex(h) for h in re.findall(r"fma4_sc\(q, f, (0x[0-9a-fp.+-]+)\)", body4)]
    return c9, scalar, four


def test_scalar_and_fourway_share_coefficients():
    c9, scalar, four = _coefficients()
    assert len(scalar) == 9 and scalar == four
    assert c9 > 0


def _grid():
    # a dense uniform grid plus the ends and points near 0 (where f q(f) is tiny)
    g = np.linspace(-0.5, 0.5, 4001)
    return np.unique(np.concatenate([g, [-0.5, 0.5, 1e-9, -1e-9, 2.0**-30]]))


def test_polynomial_relative_error_below_4e16():
    mpmath.mp.dps = 60
    c9, coef, _ = _coefficients()
    cs = [mpmath.mpf(c9)] + [mpmath.mpf(c) for c in coef]  # q's coefficients, highest first
    worst = mpmath.mpf(0)
    for f in _grid():
        fm = mpmath.mpf(float(f))
        q = cs[0]
        for c in cs[1:]:
            q = q * fm + c
        p = 1 + fm * q
        exact = mpmath.power(2, fm)
        worst = max(worst, abs(p / exact - 1))
    print(f"max relative error of the polynomial: {float(worst):.3e}")
    assert worst < mpmath.mpf("4e-16")


def _fma(a: float, b: float, c: float) -> float:
    # a * b + c rounded once to FP64 (exact in 60-digit arithmetic, then one rounding)
    return float(mpmath.mpf(a) * mpmath.mpf(b) + mpmath.mpf(c))


def test_fp64_horner_within_4_ulp():
    mpmath.mp.dps = 60
    c9, coef, _ = _coefficients()
    worst = 0.0
    for f in _grid()[::4]:
        f = float(f)
        q = _fma(f, c9, coef[0])
        for c in coef[1:]:
            q = _fma(q, f, c)
        p = _fma(q, f, 1.0)
        exact = mpmath.power(2, mpmath.mpf(f))
        ulp = float(np.spacing(float(exact)))
        worst = max(worst, abs(float(mpmath.mpf(p) - exact)) / ulp)
    print(f"max error of the FP64 evaluation: {worst:.2f} ulp")
    assert worst <= 4.0
