"""Floating-point formats of Table 1.1 and rounding to them (test infrastructure).

``unit_roundoff`` returns u = 2^-t for t significand bits (including the implicit bit), as
listed in Table 1.1.  ``fl(x, fmt)`` rounds float64 values to the nearest value of the
target format, ties to even, keeping subnormals (the reading taken for the paper's silence
on rounding mode); values above the format's largest finite number become +-inf.  This is
the elementwise "chop" model the paper used to simulate bf16 (Section 4).

fp16 uses NumPy's IEEE binary16 conversion.  bf16 (8 significand bits, binary32's
exponent range) is rounded by ``round_to_format``, written here from the format's
definition; the pins test it against independent library conversions.

Range (fp16's x_max = 65504, Table 1.1): values held at a reduced solver precision are
stored as a power of two times a value of the format (``fl_scaled``): the scale is chosen
per array (or per column) so that the largest magnitude lies in [1/2, 1), which is exact in
binary arithmetic and keeps large iterates, inverses and products out of overflow.  This is
the reading taken for the paper's silence on fp16 range (its half precision was bf16, which
has binary32's range); products take their operands this way and accumulate in binary32.
"""
from __future__ import annotations

import numpy as np

FORMATS = ("fp64", "fp32", "fp16", "bf16")  # Table 1.1 (the split format is separate)

# The split-operand format "fp16x2" (not in the paper; the hi/lo operand splitting of
# Markidis et al. 2018 and Ootomo and Yokota 2022): a value is held as a pair of binary16
# numbers, x ~ hi + 2^-11 lo with hi = fl16(x) and lo = fl16(2^11 (x - hi)), so products
# on binary16 matrix cores, hi*hi + 2^-11 (hi*lo + lo*hi) accumulated in binary32, approach
# binary32 accuracy.  22 significand bits: unit roundoff 2^-22.
SPLIT = 2.0 ** 11

# (t, e) from Table 1.1: significand bits including the implicit bit, exponent bits.
_BITS = {"bf16": (8, 8), "fp16": (11, 5), "fp32": (24, 8), "fp64": (53, 11)}


def unit_roundoff(fmt: str) -> float:
    """u = 2^-t (Table 1.1): bf16 3.91e-3, fp16 4.88e-4, fp32 5.96e-8, fp64 1.11e-16; the
    split format fp16x2 2^-22."""
    if fmt == "fp16x2":
        return 2.0 ** -22
    return 2.0 ** (-_BITS[fmt][0])


def split16(x):
    """(hi, lo) with hi = fl16(x), lo = fl16(2^11 (x - hi)): x ~ hi + 2^-11 lo."""
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(over="ignore", invalid="ignore"):
        hi = x.astype(np.float16).astype(np.float64)
        lo = (SPLIT * (x - hi)).astype(np.float16).astype(np.float64)
    return hi, lo


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
    if fmt == "fp16x2":
        hi, lo = split16(x)
        return hi + lo / SPLIT
    raise ValueError(f"unknown format {fmt!r}")


def pow2_exponent(amax) -> np.ndarray:
    """e with 2^(e-1) <= amax < 2^e (elementwise; 0 where amax is 0 or not finite)."""
    amax = np.asarray(amax, np.float64)
    ok = np.isfinite(amax) & (amax > 0)
    _, e = np.frexp(np.where(ok, amax, 1.0))
    return np.where(ok, e, 0).astype(np.int64)


def _scale_exponents(x, axis):
    """Per-array (axis None) or per-column (axis 0) exponents of the largest magnitude."""
    if x.size == 0:
        return np.zeros(() if axis is None else x.shape[1], np.int64)
    if axis is None:
        return pow2_exponent(np.max(np.abs(x)))
    return pow2_exponent(np.max(np.abs(x), axis=0))


def fl_scaled(x, fmt: str, axis=None) -> np.ndarray:
    """Round to ``fmt`` with a power-of-two scale: 2^e fl(2^-e x), where 2^-e maps the largest
    magnitude of the array (axis None) or of each column (axis 0) into [1/2, 1).  The same as
    ``fl`` inside the format's range apart from where gradual underflow starts; never
    overflows for finite x.  fp64 and fp32 are rounded plainly (their range is not at issue
    here).  Non-finite arrays are rounded plainly so that inf / NaN propagate."""
    x = np.asarray(x, dtype=np.float64)
    if fmt in ("fp64", "fp32") or x.size == 0 or not np.all(np.isfinite(x)):
        return fl(x, fmt)
    e = _scale_exponents(x, axis)
    return np.ldexp(fl(np.ldexp(x, -e), fmt), e)


def matmul(a, b, fmt: str) -> np.ndarray:
    """Product at precision ``fmt``: operands rounded to ``fmt``; for the reduced formats
    the products are accumulated in binary32 and the result is rounded to ``fmt`` (operands
    at the solver precision, binary32 accumulation); fp64 is a plain float64 product.
    For fp16 / bf16 the left operand is taken with one power-of-two scale and the right one
    with one per column (``fl_scaled``); the exact scales are applied to the binary32 sums."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if fmt == "fp64":
        return a @ b
    if fmt == "fp32":
        a32 = fl(a, fmt).astype(np.float32)
        b32 = fl(b, fmt).astype(np.float32)
        return fl((a32 @ b32).astype(np.float64), fmt)
    if not (np.all(np.isfinite(a)) and np.all(np.isfinite(b))):
        with np.errstate(invalid="ignore", over="ignore"):
            return fl(fl(a, fmt) @ fl(b, fmt), fmt)
    ea = _scale_exponents(a, None)
    eb = _scale_exponents(b, 0) if b.ndim == 2 else _scale_exponents(b[:, None], 0)[0]
    if fmt == "fp16x2":
        # three binary16 products, hi*hi and the two cross terms, each summed in binary32
        ah, al = (v.astype(np.float32) for v in split16(np.ldexp(a, -ea)))
        bh, bl = (v.astype(np.float32) for v in split16(np.ldexp(b, -eb)))
        hh = (ah @ bh).astype(np.float64)
        cross = (ah @ bl + al @ bh).astype(np.float64)
        prod = np.ldexp(hh + cross / SPLIT, ea + eb)
        return fl_scaled(prod, fmt, axis=0 if prod.ndim == 2 else None)
    a32 = fl(np.ldexp(a, -ea), fmt).astype(np.float32)
    b32 = fl(np.ldexp(b, -eb), fmt).astype(np.float32)
    prod = np.ldexp((a32 @ b32).astype(np.float64), ea + eb)
    return fl_scaled(prod, fmt, axis=0 if prod.ndim == 2 else None)
