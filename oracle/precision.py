"""Floating-point formats of Table 1.1 and rounding to them (test infrastructure).

``unit_roundoff`` returns u = 2^-t for t significand bits (including the implicit bit), as
listed in Table 1.1.  ``fl(x, fmt)`` rounds float64 values to the nearest value of the
target format, ties to even, keeping subnormals (the reading taken for the paper's silence
on rounding mode); values above the format's largest finite number become +-inf.  This is
the elementwise "chop" model the paper used to simulate bf16 (Section 4).

fp16 uses NumPy's IEEE binary16 conversion.  bf16 (8 significand bits, binary32's
exponent range) is rounded by ``round_to_format``, written here from the format's
definition; the pins test it against independent library conversions.
"""
from __future__ import annotations

import numpy as np

FORMATS = ("fp64", "fp32", "fp16", "bf16")

# (t, e) from Table 1.1: significand bits including the implicit bit, exponent bits.
_BITS = {"bf16": (8, 8), "fp16": (11, 5), "fp32": (24, 8), "fp64": (53, 11)}


def unit_roundoff(fmt: str) -> float:
    """u = 2^-t (Table 1.1): bf16 3.91e-3, fp16 4.88e-4, fp32 5.96e-8, fp64 1.11e-16."""
    return 2.0 ** (-_BITS[fmt][0])


def x_max(fmt: str) -> float:
    """Largest finite number (Table 1.1)."""
    t, e = _BITS[fmt]
    emax = 2 ** (e - 1) - 1
    return float((2.0 - 2.0 ** (1 - t)) * 2.0 ** emax)


def x_min(fmt: str) -> float:
    """Smallest positive normalised number (Table 1.1)."""
    e = _BITS[fmt][1]
    return float(2.0 ** (2 - 2 ** (e - 1)))


def round_to_format(x, t: int, emin: int, xmax: float) -> np.ndarray:
    """Round float64 values to a binary format with t significand bits (implicit bit
    included), smallest normal exponent ``emin`` (x_min = 2^emin) and largest finite value
    ``xmax``: round to nearest, ties to even, gradual underflow, overflow to +-inf."""
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()
    finite = np.isfinite(x) & (x != 0)
    xf = x[finite]
    _, ex = np.frexp(xf)                  # xf = mant * 2^ex, 0.5 <= |mant| < 1
    # ulp of the binade [2^(ex-1), 2^ex) is 2^(ex-t); below x_min the ulp is 2^(emin+1-t)
    ulp_exp = np.maximum(ex - 1, emin) + 1 - t
    scaled = np.ldexp(xf, -ulp_exp)       # exact power-of-two scaling
    y = np.ldexp(np.round(scaled), ulp_exp)   # np.round: half to even
    y = np.where(np.abs(y) > xmax, np.copysign(np.inf, y), y)
    out[finite] = y
    return out


def _bf16_round(x) -> np.ndarray:
    t, e = _BITS["bf16"]
    return round_to_format(x, t, 2 - 2 ** (e - 1), x_max("bf16"))


def fl(x, fmt: str) -> np.ndarray:
    """Round float64 array ``x`` to format ``fmt`` (RNE, subnormals kept); returns float64."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "fp64":
        return x
    if fmt == "fp32":
        with np.errstate(over="ignore"):
            return x.astype(np.float32).astype(np.float64)
    if fmt == "fp16":
        with np.errstate(over="ignore"):
            return x.astype(np.float16).astype(np.float64)
    if fmt == "bf16":
        return _bf16_round(x)
    raise ValueError(f"unknown format {fmt!r}")


def matmul(a, b, fmt: str) -> np.ndarray:
    """Product at precision ``fmt``: operands rounded to ``fmt``; for the reduced formats
    the products are accumulated in binary32 and the result is rounded to ``fmt`` (operands
    at the solver precision, binary32 accumulation); fp64 is a plain float64 product."""
    if fmt == "fp64":
        return np.asarray(a, np.float64) @ np.asarray(b, np.float64)
    a32 = fl(a, fmt).astype(np.float32)
    b32 = fl(b, fmt).astype(np.float32)
    return fl((a32 @ b32).astype(np.float64), fmt)
