"""Pins for oracle.signnewton (Section 3): closed forms, the dense iteration (3.1), the
factored invariants of (3.2)/(3.3), Roberts' block identity, Table 4.1 Newton counts and the
rank-truncation guarantees."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import lyapgen
from oracle import exact as E
from oracle import signnewton as SN
from oracle.precision import unit_roundoff

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table_4_1_newton_counts.json")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_shift_reaches_minus_identity_in_one_scaled_step():
    alpha = 2.5
    n = 16
    A = -alpha * np.eye(n)
    seq = SN.a_sequence(A, "fp64")
    assert seq.mus[0] == pytest.approx(1.0 / alpha, rel=1e-15)
    assert seq.onenorms[0] == 0.0
    # the step that meets the test is followed by one further step
    assert seq.K == 2
    L = np.random.default_rng(0).standard_normal((n, 2))
    W = L @ L.T
    Z, Y, _, _ = SN.sign_newton_ldlt(A, L, np.ones(2), seq=seq)
    assert _rel(Z @ Y @ Z.T, W / (2 * alpha)) <= 1e-14
    Zc, _, _ = SN.sign_newton_chol(A, L, seq=seq)
    assert _rel(Zc @ Zc.T, W / (2 * alpha)) <= 1e-14


def test_a_iteration_converges_to_minus_identity():
    A, _ = lyapgen.random_shift(3, 60, 1)
    seq = SN.a_sequence(A, "fp64")
    assert np.linalg.norm(seq.A_last + np.eye(60), 1) <= 1e-10
    assert np.trace(seq.A_last) == pytest.approx(-60.0, abs=1e-10)


def test_dense_iteration_limits():
    # A_k -> -I and W_k -> 2X for the dense form (3.1), with the oracle's scalings.
    A, L = lyapgen.random_shift(4, 30, 2)
    W = L @ L.T
    seq = SN.a_sequence(A, "fp64")
    As, Ws = SN.dense_iteration(A, W, seq.mus)
    assert np.linalg.norm(As[-1] + np.eye(30)) <= 1e-12
    assert _rel(Ws[-1] / 2, E.bartels_stewart(A, W)) <= 1e-12


@pytest.mark.parametrize("form", ["chol", "ldlt"])
def test_factored_iterates_reproduce_dense_iterates(form):
    # Z_k Z_k^T = W_k (3.2) and Z_k Y_k Z_k^T = W_k (3.3) while nothing is truncated.
    n, m = 40, 2
    A, L = lyapgen.random_shift(5, n, m)
    W = L @ L.T
    seq = SN.a_sequence(A, "fp64")
    _, Ws = SN.dense_iteration(A, W, seq.mus)
    for k in range(1, seq.K + 1):
        sub = SN.ASequence(fmt="fp64", inverses=seq.inverses[:k], mus=seq.mus[:k])
        if form == "chol":
            Z, _, info = SN.sign_newton_chol(A, L, rho=1e9, seq=sub)
            Xk = 2.0 * Z @ Z.T            # the solver returns Z_k / sqrt(2)
        else:
            Z, Y, _, info = SN.sign_newton_ldlt(A, L, np.ones(m), rho=1e9, seq=sub)
            Xk = Z @ (2.0 * Y) @ Z.T      # the solver returns Y_k / 2
        assert info.truncations == 0
        assert _rel(Xk, Ws[k]) <= 1e-12, k


def test_y_iterate_has_kronecker_structure():
    n, m = 30, 3
    A, L = lyapgen.random_shift(6, n, m)
    S = np.array([1.0, -2.0, 0.5])
    seq = SN.a_sequence(A, "fp64")
    _, Y, _, _ = SN.sign_newton_ldlt(A, L, S, psd=False, rho=1e9, seq=seq)
    assert np.allclose(Y * 2.0, SN.kron_y_structure(seq.mus, S), rtol=1e-14, atol=0)


def test_roberts_block_sign_identity():
    # sign([[A, W], [0, -A^T]]) = [[-I, 2X], [0, I]]; the sign is taken by SciPy's signm.
    n = 24
    A, L = lyapgen.random_shift(7, n, 2)
    W = L @ L.T
    B = np.block([[A, W], [np.zeros((n, n)), -A.T]])
    Sg = sla.signm(B)
    X = E.bartels_stewart(A, W)
    assert np.linalg.norm(Sg[:n, :n] + np.eye(n)) <= 1e-8
    assert _rel(Sg[:n, n:] / 2.0, X) <= 1e-8
    Z, Y, _, _ = SN.sign_newton_ldlt(A, L, np.ones(2))
    assert _rel(Z @ Y @ Z.T, Sg[:n, n:] / 2.0) <= 1e-8


@pytest.mark.parametrize("n", [100, 1000])
@pytest.mark.parametrize("us", ["fp64", "fp32"])
def test_table_4_1_newton_counts(n, us):
    g = json.load(open(GOLD))
    want = g["alpha"][f"n{n}_us_{us}"]
    got = [SN.a_sequence(lyapgen.paper_family(n, q)[0], us).K for q in g["q"]]
    assert got == want


@pytest.mark.parametrize("form", ["chol", "ldlt"])
def test_fp64_solver_matches_exact_solution(form):
    A, L = lyapgen.random_shift(8, 64, 2)
    X = E.kron_solve(A, L @ L.T)
    if form == "chol":
        Z, _, _ = SN.sign_newton_chol(A, L)
        Xh = Z @ Z.T
    else:
        Z, Y, _, _ = SN.sign_newton_ldlt(A, L, np.ones(2))
        Xh = Z @ Y @ Z.T
    assert _rel(Xh, X) <= 1e-12


def test_rank_trunc_chol_bound():
    rng = np.random.default_rng(9)
    n, c = 200, 60
    U, _ = np.linalg.qr(rng.standard_normal((n, c)))
    s = np.logspace(0, -12, c)
    Z = U * s[None, :]
    Zr = SN.rank_trunc_chol(Z, "fp64")
    u = unit_roundoff("fp64")
    err = np.linalg.norm(Z @ Z.T - Zr @ Zr.T, 2)
    # the dropped block contributes at most u ||Z||^2; the QR itself adds O(c u ||Z||^2)
    assert err <= 10 * u * np.linalg.norm(Z, 2) ** 2
    assert Zr.shape[1] < c
    # every singular value of Z well above sqrt(u) * ||Z|| survives
    assert Zr.shape[1] >= int((s > 1e3 * math.sqrt(u)).sum())


def test_rank_trunc_ldlt_keeps_above_threshold():
    rng = np.random.default_rng(10)
    n, c = 150, 40
    Z = rng.standard_normal((n, c))
    lam = np.concatenate([np.logspace(0, -20, c - 5), -np.logspace(-1, -3, 5)])
    Q, _ = np.linalg.qr(rng.standard_normal((c, c)))
    Y = Q @ np.diag(lam) @ Q.T
    Zr, Yr = SN.rank_trunc_ldlt(Z, Y, "fp64", psd=False)
    assert np.allclose(Zr.T @ Zr, np.eye(Zr.shape[1]), atol=1e-13)
    X = Z @ Y @ Z.T
    assert np.linalg.norm(X - Zr @ Yr @ Zr.T, 2) <= 1e-13 * np.linalg.norm(X, 2)
    assert np.any(np.diag(Yr) < 0)
    Zp, Yp = SN.rank_trunc_ldlt(Z, Y, "fp64", psd=True)
    assert np.all(np.diag(Yp) > 0)


def test_singular_and_unstable_inputs():
    A = np.diag([-1.0, -2.0, 0.0, -3.0])
    with pytest.raises(np.linalg.LinAlgError):
        SN.a_sequence(A, "fp64")
    # one eigenvalue in the right half-plane: the iteration converges to sign(A) != -I
    A2 = np.diag([-1.0, -2.0, 0.1, -3.0, -0.5])
    try:
        seq = SN.a_sequence(A2, "fp64")
        assert abs(np.trace(seq.A_last) + 5.0) > 1.0
    except SN.NotStableError:
        pass


def test_gauss_jordan_emulation_is_an_inverse():
    A, _ = lyapgen.random_shift(11, 50, 1)
    Xi = SN.gauss_jordan_inverse(A, "fp64")
    assert _rel(Xi, np.linalg.inv(A)) <= 1e-13
    X16 = SN.inverse_at(A, "fp16")
    k = np.linalg.cond(A)
    assert _rel(X16, np.linalg.inv(A)) <= 50 * k * unit_roundoff("fp16")
    assert _rel(X16, np.linalg.inv(A)) >= 0.1 * unit_roundoff("fp16")
