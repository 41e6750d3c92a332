"""Pins for oracle.exact / oracle.residual: the three solution routes agree with each other,
with SciPy's independent Lyapunov solver and with closed forms."""
import numpy as np
import pytest
import scipy.linalg as sla

import lyapgen
from oracle import exact as E
from oracle import residual as R


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,m,seed", [(12, 2, 11), (40, 3, 12), (64, 2, 1)])
def test_kronecker_matches_bartels_stewart(n, m, seed):
    A, L = lyapgen.random_shift(seed, n, m)
    W = L @ L.T
    Xk = E.kron_solve(A, W)
    Xb = E.bartels_stewart(A, W)
    assert _rel(Xb, Xk) <= 1e-12
    assert R.relres_dense(A, W, Xk) <= 1e-14


def test_bartels_stewart_matches_scipy_library_solver():
    A, L = lyapgen.random_shift(21, 150, 4)
    W = L @ L.T
    Xb = E.bartels_stewart(A, W)
    Xs = sla.solve_continuous_lyapunov(A, -W)   # A X + X A^H = Q with Q = -W
    assert _rel(Xb, Xs) <= 1e-11


def test_schur_recurrence_matches_general_bartels_stewart():
    A, L, Q, T = lyapgen.schur_family(5, 160, 3, lo=-2.0)
    W = L @ L.T
    Xs = E.schur_solve(Q, T, W)
    Xb = E.bartels_stewart(A, W)
    assert _rel(Xs, Xb) <= 1e-10
    assert R.relres_dense(A, W, Xs) <= 1e-15


def test_diagonal_closed_form():
    rng = np.random.default_rng(7)
    a = -rng.uniform(0.1, 3.0, 30)
    L = rng.standard_normal((30, 3))
    W = L @ L.T
    X = E.diag_closed_form(a, W)
    assert _rel(E.kron_solve(np.diag(a), W), X) <= 1e-13
    assert _rel(E.bartels_stewart(np.diag(a), W), X) <= 1e-13


def test_shift_closed_form():
    rng = np.random.default_rng(8)
    L = rng.standard_normal((25, 2))
    W = L @ L.T
    X = E.shift_closed_form(1.7, W)
    assert _rel(E.bartels_stewart(-1.7 * np.eye(25), W), X) <= 1e-13


def test_solution_symmetric_psd_for_psd_rhs():
    A, L = lyapgen.random_shift(9, 80, 3)
    X = E.bartels_stewart(A, L @ L.T)
    assert np.linalg.norm(X - X.T) <= 1e-15 * np.linalg.norm(X)
    w = np.linalg.eigvalsh(X)
    assert w.min() >= -1e-13 * w.max()


def test_indefinite_rhs_gives_indefinite_solution():
    A, L = lyapgen.random_shift(10, 50, 4)
    s = np.array([1.0, -1.0, 1.0, -1.0])
    W = E.form_w(L, s)
    X = E.bartels_stewart(A, W)
    assert _rel(E.kron_solve(A, W), X) <= 1e-12
    w = np.linalg.eigvalsh(X)
    assert w.min() < 0 < w.max()


def test_residual_definitions_consistent():
    A, L = lyapgen.random_shift(13, 30, 2)
    rng = np.random.default_rng(0)
    Z = rng.standard_normal((30, 5))
    d = rng.standard_normal(5)
    Rm = R.residual_matrix(A, L, None, Z, d)
    X = (Z * d) @ Z.T
    assert np.allclose(Rm, A @ X + X @ A.T + L @ L.T, rtol=0, atol=1e-12)
    den = np.linalg.norm(L @ L.T) + 2 * np.linalg.norm(X) * np.linalg.norm(A)
    assert R.relres(A, L, None, Z, d) == pytest.approx(np.linalg.norm(Rm) / den, rel=1e-13)


def test_planted_transpose_mistake_is_caught():
    # A solver that forgot the transpose (solved AX + XA + W = 0) fails the pins above.
    A, L = lyapgen.random_shift(14, 20, 2)
    W = L @ L.T
    X_wrong = sla.solve_sylvester(A, A, -W)
    assert R.relres_dense(A, W, X_wrong) > 1e-6


def test_bartels_stewart_lapack_triangular_step_equals_recurrence():
    # the ztrsyl path (used above n = 512) and the column recurrence give the same solution
    import lyapgen
    from oracle import exact as E
    A, L = lyapgen.random_shift(9, 150, 3)
    W = L @ L.T
    a = E.bartels_stewart(A, W, recurrence=True)
    b = E.bartels_stewart(A, W, recurrence=False)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)
    X = E.kron_solve(A[:40, :40], W[:40, :40])
    assert np.linalg.norm(E.bartels_stewart(A[:40, :40], W[:40, :40], recurrence=False) - X) \
        <= 1e-12 * np.linalg.norm(X)
