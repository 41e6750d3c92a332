"""Pins for the low-rank ADI inner solver of the oracle (the second solver the refinement
framework admits, Section 3 and the Conclusions): the residual identity of the
residual-factor recurrence, the closed form of the ADI error for a diagonal A, the one-step
exact case, the equioscillation that characterises Wachspress's optimal shifts, the power
iteration on a matrix with known spectrum, and refinement with ADI reaching tau_I."""
import math

import numpy as np
import pytest

import lyapgen
from oracle import adi as AD
from oracle import exact as E
from oracle import refine as IR
from oracle import residual as R


def _fixed_sequence(A, shifts):
    n = A.shape[0]
    seq = AD.ADISequence(fmt="fp64", a=0.0, b=0.0, shifts=list(shifts))
    seq.inverses = [np.linalg.inv(A + p * np.eye(n)) for p in shifts]
    return seq


def _recurrence(A, G, s, shifts, steps):
    """The dense residual A X_j + X_j A^T + G S G^T after each step, and W_j S W_j^T from the
    oracle's factors (recomputed here from its V blocks)."""
    seq = _fixed_sequence(A, shifts)
    out = []
    for j in range(1, steps + 1):
        Z, d, _ = AD.lr_adi_ldlt(A, G, s, "fp64", seq, psd=False, rho=10.0, max_steps=j,
                                 tol_inner=0.0)
        X = (Z * d) @ Z.T
        out.append((X, A @ X + X @ A.T + (G * s) @ G.T))
    return out


def test_residual_is_the_factored_residual():
    # A X_j + X_j A^T + G S G^T = W_j S W_j^T with W_j = W_{j-1} - 2 p_j V_j: build W_j here
    # by the textbook recurrence and compare with the dense residual of the oracle's X_j
    rng = np.random.default_rng(3)
    n = 30
    A = -np.eye(n) * 2.0 + 0.3 * rng.standard_normal((n, n))
    assert np.max(np.linalg.eigvals(A).real) < 0
    G = rng.standard_normal((n, 3))
    s = np.array([1.0, -2.0, 0.5])
    shifts = [-0.7, -3.1, -1.6, -5.0]
    W = G.copy()
    for j, (X, Res) in enumerate(_recurrence(A, G, s, shifts, 4)):
        p = shifts[j]
        V = np.linalg.solve(A + p * np.eye(n), W)
        W = W - 2.0 * p * V
        np.testing.assert_allclose(Res, (W * s) @ W.T, atol=1e-11 * np.linalg.norm(G) ** 2)


def test_diagonal_a_error_has_the_closed_form():
    # diagonal A: X_ik = -W_ik / (a_i + a_k) and the ADI error after the steps p_1 .. p_J is
    # X_ik prod_l r_l(a_i) r_l(a_k) with r_l(x) = (x - p_l) / (x + p_l)
    rng = np.random.default_rng(5)
    a = -np.geomspace(0.05, 4.0, 12)
    A = np.diag(a)
    G = rng.standard_normal((12, 2))
    W = G @ G.T
    X = -W / (a[:, None] + a[None, :])
    shifts = [-0.1, -1.0, -3.0]
    Z, d, _ = AD.lr_adi_ldlt(A, G, np.ones(2), "fp64", _fixed_sequence(A, shifts), psd=True,
                             rho=10.0, max_steps=3)
    r = np.ones(12)
    for p in shifts:
        r *= (a - p) / (a + p)
    np.testing.assert_allclose(X - (Z * d) @ Z.T, X * np.outer(r, r), atol=1e-14, rtol=1e-10)


def test_one_shift_at_the_eigenvalue_is_exact():
    # A = alpha I with p = alpha: V = G / (2 alpha), X_1 = -2 alpha V S V^T = -G S G^T / (2 alpha)
    alpha = -1.7
    rng = np.random.default_rng(1)
    G = rng.standard_normal((9, 2))
    s = np.array([1.0, -1.0])
    A = alpha * np.eye(9)
    Z, d, info = AD.lr_adi_ldlt(A, G, s, "fp64", _fixed_sequence(A, [alpha]), psd=False)
    assert info.steps == 1 and info.res_hist[0] <= 1e-15
    np.testing.assert_allclose((Z * d) @ Z.T, -(G * s) @ G.T / (2.0 * alpha), rtol=1e-14)


@pytest.mark.parametrize("a,b,J", [(1e-3, 1.0, 7), (0.2, 5.0, 3), (1e-2, 1.0, 12)])
def test_wachspress_shifts_equioscillate(a, b, J):
    # the optimal shifts make |prod (x - q_i)/(x + q_i)| equioscillate on [a, b]: J + 1 equal
    # local maxima (the endpoints included) -- a mistake in the elliptic parametrisation
    # (modulus, the odd multiples of K / (2J), the scale b) breaks the equality
    q = -AD.wachspress_shifts(a, b, J)
    assert np.all((q >= a * (1 - 1e-12)) & (q <= b * (1 + 1e-12)))
    x = np.geomspace(a, b, 400001)
    r = AD.adi_error_function(x, q)
    inner = np.where((r[1:-1] >= r[:-2]) & (r[1:-1] >= r[2:]))[0] + 1
    peaks = np.concatenate([[r[0]], r[inner], [r[-1]]])
    assert peaks.size == J + 1
    assert np.max(peaks) <= np.min(peaks) * (1 + 1e-4)


@pytest.mark.parametrize("a,b", [(1e-3, 1.0), (0.3, 2.0)])
@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-8])
def test_shift_count_meets_the_bound(a, b, eps):
    J = AD.shift_count(a, b, eps)
    x = np.geomspace(a, b, 200001)
    assert np.max(AD.adi_error_function(x, AD.wachspress_shifts(a, b, J))) <= eps
    if J > 1:
        # and one shift fewer is not enough (within the factor 4 of the asymptotic bound)
        assert np.max(AD.adi_error_function(x, AD.wachspress_shifts(a, b, J - 1))) > eps / 4


def test_power_iteration_on_a_known_spectrum():
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = -np.concatenate([[10.0], np.linspace(0.1, 5.0, 39)])
    A = (Q * lam) @ Q.T
    assert AD.power_rho(A) == pytest.approx(10.0, rel=1e-6)
    a, b = AD.spectral_interval(A, "fp64")
    assert b == pytest.approx(10.0, rel=1e-6)
    # rho(A^-1) = 10 with its eigenvalue close to the next (1/0.1 vs 1/0.226): slower, looser
    assert a == pytest.approx(0.1, rel=0.05)


@pytest.mark.parametrize("us", ["fp64", "fp32", "fp16"])
def test_refinement_with_adi_reaches_tau(us):
    A, L = lyapgen.random_shift(1, 64, 2)
    X = E.kron_solve(A, L @ L.T)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=(us, "fp64", "fp64", "fp64"), solver="adi")
    assert info.status == "OK"
    assert R.relres(A, L, None, Z, d) <= 1e-13
    assert np.linalg.norm((Z * d) @ Z.T - X) / np.linalg.norm(X) <= 1e-11
    # J + 1 inversions (the interval's included), done once for every solve
    assert info.inversions == len(info.mus) + 1
    assert (info.refinements == 0) == (us == "fp64")


def test_adi_with_indefinite_s_and_the_adjoint():
    A, L = lyapgen.random_shift(4, 48, 3)
    s = np.array([1.0, -1.0, 2.0])
    Zi, di, info = IR.ir_ldlt(A, L, s, prec=("fp32", "fp64", "fp64", "fp64"), solver="adi")
    assert info.status == "OK"
    assert R.relres_dense(A, (L * s) @ L.T, (Zi * di) @ Zi.T) <= 1e-13
    # the transposed products solve A^T Y + Y A + G S G^T = 0 on the same sequence
    seq = AD.adi_sequence(A, "fp64")
    Zt, dt, _ = AD.lr_adi_ldlt(A, L, s, "fp64", seq, psd=False, trans=True)
    Y = E.kron_solve(A.T, (L * s) @ L.T)
    assert np.linalg.norm((Zt * dt) @ Zt.T - Y) / np.linalg.norm(Y) <= 1e-12
