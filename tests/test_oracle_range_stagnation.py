"""Pins for the oracle's fp16 range handling (Table 1.1 x_max; scaled casts of A_k, factors
and products), for the early stop of eq (4.2), and for the construction of the n = 4096
workload (the triangular factor's off-diagonal scale)."""
import numpy as np
import pytest

import lyapgen
from oracle import exact as E
from oracle import refine as IR
from oracle import residual as R
from oracle import signnewton as SN
from oracle.precision import fl, fl_scaled, matmul, unit_roundoff, x_max


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ------------------------------------------------------------------- scaled storage
def test_fl_scaled_keeps_large_values_finite_and_equals_fl_in_range():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((40, 7))
    # inside the range the power-of-two scale changes nothing but where underflow starts
    assert np.array_equal(fl_scaled(x, "fp16"), fl(x, "fp16"))
    big = x * 2.0 ** 30                      # far above fp16's x_max = 65504
    assert np.all(np.isinf(fl(big, "fp16")[np.abs(big) > x_max("fp16")]))
    y = fl_scaled(big, "fp16")
    assert np.all(np.isfinite(y))
    # exact equivariance under powers of two, per array and per column
    assert np.array_equal(y, 2.0 ** 30 * fl_scaled(x, "fp16"))
    cols = x * (2.0 ** np.arange(0, 70, 10))[None, :]
    yc = fl_scaled(cols, "fp16", axis=0)
    assert np.array_equal(yc, fl_scaled(x, "fp16", axis=0) * (2.0 ** np.arange(0, 70, 10)))
    # relative rounding error is fp16's unit roundoff for the largest entries of each column
    top = np.argmax(np.abs(cols), axis=0)
    j = np.arange(cols.shape[1])
    assert np.all(np.abs(yc[top, j] - cols[top, j]) <= unit_roundoff("fp16") * np.abs(cols[top, j]))


@pytest.mark.parametrize("fmt", ["fp16", "bf16"])
def test_matmul_reduced_is_exactly_scale_equivariant(fmt):
    rng = np.random.default_rng(1)
    a = rng.standard_normal((30, 20))
    b = rng.standard_normal((20, 6))
    p = matmul(a, b, fmt)
    q = matmul(2.0 ** -12 * a, b * (2.0 ** np.array([20, 0, -5, 9, 14, 3]))[None, :], fmt)
    assert np.array_equal(q, p * 2.0 ** -12 * (2.0 ** np.array([20, 0, -5, 9, 14, 3]))[None, :])
    assert _rel(p, a @ b) <= 4 * 20 * unit_roundoff(fmt)


def test_fp16_first_solve_on_graded_family_is_not_dropped():
    """The n = 4096 workload's construction at n = 256 (diag down to 1e-3, kappa ~ 1e3): the
    fp16 solver's truncations form R Y R^T with entries far above 65504.  With unscaled fp16
    storage every eigenvalue became inf and the whole factor was dropped (X_hat = 0, relative
    error 1); with scaled storage the first solve is within kappa u_s of X."""
    A, L, Q, T = lyapgen.schur_family(3, 256, 8, lo=-3.0, upper_std_scale=0.003)
    s = lyapgen.indefinite_signs(1003, 8)
    X = E.schur_solve(Q, T, E.form_w(L, s))
    Z, Y, seq, info = SN.sign_newton_ldlt(A, L, s, "fp16", psd=False)
    assert Z.shape[1] >= 8 and min(info.columns) > 0
    err = _rel(Z @ Y @ Z.T, X)
    assert err <= 1e3 * unit_roundoff("fp16")          # kappa ~ 1e3 times u_s = 0.49
    assert R.relres(A, L, s, Z, np.diag(Y)) <= 1e-2


def test_fp16_solve_is_scale_invariant():
    """A <- 2^-10 A, L <- 2^6 L gives X <- 2^22 X: the scaled Newton step removes the scale
    of A after one step, and power-of-two scaled storage rounds the same significands."""
    A, L = lyapgen.random_shift(1, 64, 2)
    Z, Y, _, _ = SN.sign_newton_ldlt(A, L, np.ones(2), "fp16", psd=True)
    Zs, Ys, _, _ = SN.sign_newton_ldlt(2.0 ** -10 * A, 2.0 ** 6 * L, np.ones(2), "fp16", psd=True)
    X, Xs = Z @ Y @ Z.T, Zs @ Ys @ Zs.T
    assert np.all(np.isfinite(Xs))
    assert _rel(Xs, 2.0 ** 22 * X) <= 10 * unit_roundoff("fp16")
    Zi, di, info = IR.ir_ldlt(2.0 ** -10 * A, 2.0 ** 6 * L, None, prec=("fp16", "fp64", "fp64", "fp64"))
    assert info.status == "OK"
    Xe = E.kron_solve(2.0 ** -10 * A, 2.0 ** 12 * L @ L.T)
    assert _rel((Zi * di) @ Zi.T, Xe) <= 1e-11


def test_rank_trunc_rejects_non_finite_eigenvalues():
    Z = np.array([[1.0, np.inf], [0.0, 1.0]])
    with pytest.raises((SN.NonFiniteError, np.linalg.LinAlgError, ValueError)):
        SN.rank_trunc_ldlt(Z, np.eye(2), "fp16", psd=True)


# --------------------------------------------------------------------- eq (4.2)
@pytest.mark.parametrize("hist,expect", [
    ([1.0, 0.95, 0.9], True),             # theta = 0.95, 0.947: twice above 0.9
    ([1.0, 0.95, 0.5], False),            # once
    ([1.0, 0.5, 0.49], False),            # theta = 0.5, then 0.98: once
    ([1.0, 0.91], False),                 # one ratio only
    ([1e-8, 1e-12, 1e-16, 0.95e-16, 0.9e-16], True),
    ([1e-8, 1e-12, 0.9e-12, 0.1e-12, 0.095e-12], False),   # two ratios above, not consecutive
    ([1.0, 0.9, 0.81], False),            # exactly 0.9 is not above it
])
def test_stagnation_rule_constructed_histories(hist, expect):
    assert IR.stagnated(hist, 0.9) is expect


@pytest.mark.parametrize("us", ["fp64", "fp32", "fp16"])
def test_refinement_with_zero_tolerance_stops_by_stagnation(us):
    """tau_I = 0 is never met: the residual levels off at the rounding level of the FP64
    residual and update, and eq (4.2) must end the loop (not i_max), at the first step where
    the rule holds, with a valid iterate."""
    A, L = lyapgen.random_shift(1, 64, 2)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=(us, "fp64", "fp64", "fp64"), tol=0.0)
    h = info.res_hist
    assert info.status == "STAGNATED"
    assert IR.stagnated(h, 0.9)
    assert not any(IR.stagnated(h[:k], 0.9) for k in range(len(h)))
    assert len(h) < 50
    assert R.relres(A, L, None, Z, d) <= 1e-14


def test_refinement_i_max_one_is_not_converged():
    A, L = lyapgen.random_shift(1, 64, 2)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("fp16", "fp64", "fp64", "fp64"), tol=1e-13, i_max=1)
    assert info.status == "NOT_CONVERGED"
    assert info.refinements == 0 and len(info.res_hist) == 1
    assert info.res > 1e-13


# ------------------------------------------------------- the n = 4096 workload's T
@pytest.mark.slow
def test_large_workload_off_diagonal_scale():
    """With diag(T) = -logspace(-3, 0, 4096), strict-upper entries of std 0.1/sqrt(n) are
    larger than the leading diagonal entries (1e-3), and the leading 64 x 64 block of T alone
    has an inverse of norm above 1e12 (the sign iteration cannot converge).  At
    0.003/sqrt(n) that block's inverse stays within a small factor of the diagonal's,
    ||diag^-1|| ~ 8e3, as for a normal matrix with the same spectrum."""
    norms = {}
    for scale in (0.1, 0.003):
        T = lyapgen.schur_family(3, 4096, 8, lo=-3.0, upper_std_scale=scale)[3]
        B = T[:64, :64]
        norms[scale] = np.linalg.norm(np.linalg.inv(B))
        diag_norm = np.linalg.norm(1.0 / np.diag(B))
    assert norms[0.1] >= 1e12
    assert norms[0.003] <= 2.0 * diag_norm
