"""Pins for the split-operand binary16 format fp16x2 of the oracle (x ~ hi + 2^-11 lo, hi and
lo binary16; products hi*hi + 2^-11 (hi*lo + lo*hi) in binary32): its representation error,
the accuracy of its products against exact float64 products, and IR with it as the solver
precision (the bound of Table 3.1 with u_s = 2^-22)."""
import numpy as np
import pytest

import lyapgen
from oracle import exact as E
from oracle import refine as IR
from oracle import residual as R
from oracle import signnewton as SN
from oracle.precision import fl, matmul, split16, unit_roundoff


def test_split_representation_error_is_22_bits():
    rng = np.random.default_rng(0)
    x = rng.uniform(0.5, 1.0, 100000) * rng.choice([-1.0, 1.0], 100000)
    hi, lo = split16(x)
    # hi is binary16, lo is binary16, and the pair carries 22 significand bits
    assert np.array_equal(hi, hi.astype(np.float16).astype(np.float64))
    assert np.array_equal(lo, lo.astype(np.float16).astype(np.float64))
    err = np.abs(x - (hi + lo / 2048.0))
    assert np.all(err <= 2.0 ** -22 * np.abs(x))
    assert np.max(err / np.abs(x)) > 2.0 ** -26      # not exact: 22 bits, not 24 or 53
    # binary16 numbers are represented exactly (lo = 0)
    h = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(fl(h, "fp16x2"), h)
    assert unit_roundoff("fp16x2") == 2.0 ** -22


@pytest.mark.parametrize("K", [16, 200])
def test_split_products_approach_binary32(K):
    rng = np.random.default_rng(K)
    a = rng.standard_normal((40, K))
    b = rng.standard_normal((K, 30))
    exact = a @ b
    absprod = np.abs(a) @ np.abs(b)
    e16 = np.abs(matmul(a, b, "fp16") - exact)
    ex2 = np.abs(matmul(a, b, "fp16x2") - exact)
    # operands at 2^-22 each, binary32 sums, the result stored at fp16x2
    assert np.all(ex2 <= (3 * 2.0 ** -22 + K * 2.0 ** -24) * absprod)
    assert np.median(ex2 / absprod) * 100 < np.median(e16 / absprod)


def test_ir_with_split_solver_reaches_the_exact_solution():
    A, L = lyapgen.random_shift(1, 64, 2)
    X = E.kron_solve(A, L @ L.T)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("fp16x2", "fp64", "fp64", "fp64"), tol=1e-13)
    assert info.status == "OK"
    assert R.relres(A, L, None, Z, d) <= 1e-13
    assert np.linalg.norm((Z * d) @ Z.T - X) <= 1e-10 * np.linalg.norm(X)
    # Newton counts sit between the binary32 and binary16 solvers' (tau_N = 10 sqrt(n u_s))
    k32 = SN.a_sequence(A, "fp32").K
    k16 = SN.a_sequence(A, "fp16").K
    assert k16 <= info.inversions <= k32 + 1
    # fewer refinements than with binary16 operands
    _, _, i16 = IR.ir_ldlt(A, L, None, prec=("fp16", "fp64", "fp64", "fp64"), tol=1e-13)
    assert info.refinements <= i16.refinements
