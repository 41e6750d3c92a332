"""Pins for the oracle's optional paths: the alternative Newton scalings of Section 3
(determinantal, 2-norm, spectral), refinement from a given starting factor (the first line of
Alg 2.1 / 2.2 accepts any X_0), precision escalation along Table 1.1's order, working
precision u = fp32 (Table 3.1's rows with u = fp32) and a full symmetric S (diagonalised
once, an exact orthogonal change of L)."""
import math

import numpy as np
import pytest

import lyapgen
from oracle import exact as E
from oracle import refine as IR
from oracle import residual as R
from oracle import signnewton as SN
from oracle.precision import fl, unit_roundoff


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# ----------------------------------------------------------------------------- scalings
@pytest.mark.parametrize("kind", SN.SCALINGS)
def test_scaled_identity_reaches_minus_identity_in_one_step(kind):
    # A = -alpha I: every scaling gives mu_0 = 1/alpha (|det A|^(-1/n) = ||A^-1||/||A|| ratio
    # = rho ratio = 1/alpha^2 under the square root), and A_1 = -I exactly.
    alpha = 3.0
    A = -alpha * np.eye(24)
    seq = SN.a_sequence(A, "fp64", scaling_kind=kind)
    assert seq.mus[0] == pytest.approx(1.0 / alpha, rel=1e-13)
    np.testing.assert_allclose(seq.inverses[0], -np.eye(24) / alpha, rtol=1e-15)
    assert seq.onenorms[0] <= 1e-15


def test_determinantal_scaling_of_a_diagonal_matrix():
    # det of a diagonal matrix is the product of its entries: mu = (prod |a_i|)^(-1/n)
    a = -np.array([0.5, 2.0, 7.0, 0.01, 3.0, 40.0])
    A = np.diag(a)
    mu = SN.scaling_mu(A, np.diag(1.0 / a), "det")
    assert mu == pytest.approx(float(np.prod(np.abs(a))) ** (-1.0 / a.size), rel=1e-14)


def test_combined_scaling_of_a_diagonal_matrix():
    # combined scaling: mu_0 determinantal, later steps Frobenius.  For diagonal A every
    # iterate is diagonal, b -> (mu b + 1/(mu b)) / 2 entrywise, so both scalings have closed
    # forms: mu_0 = (prod |a_i|)^(-1/n), mu_1 = sqrt(||1/b||_2 / ||b||_2)
    a = -np.array([0.5, 2.0, 7.0, 0.01, 3.0, 40.0, 0.2, 9.0])
    seq = SN.a_sequence(np.diag(a), "fp64", scaling_kind="combined")
    mu0 = float(np.prod(np.abs(a))) ** (-1.0 / a.size)
    b = 0.5 * (mu0 * a + 1.0 / (mu0 * a))
    mu1 = math.sqrt(np.linalg.norm(1.0 / b) / np.linalg.norm(b))
    assert seq.mus[0] == pytest.approx(mu0, rel=1e-13)
    assert seq.mus[1] == pytest.approx(mu1, rel=1e-12)
    # and not the determinantal value at step 1 (it differs for this spectrum)
    mu1_det = float(np.prod(np.abs(b))) ** (-1.0 / b.size)
    assert abs(mu1 - mu1_det) > 1e-3 * mu1


@pytest.mark.parametrize("kind", ["2norm", "spectral"])
def test_norm_and_spectral_scaling_of_a_symmetric_matrix(kind):
    # symmetric negative definite A with spectrum in [-b, -a]: ||A||_2 = rho(A) = b and
    # ||A^-1||_2 = rho(A^-1) = 1/a, so mu = 1/sqrt(a b) (the scaling that maps the extreme
    # eigenvalues symmetrically about -1); with a b != 1 a swapped ratio would give sqrt(a b)
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    lam = -np.geomspace(0.2, 50.0, 30)
    A = (Q * lam) @ Q.T
    mu = SN.scaling_mu(A, np.linalg.inv(A), kind)
    assert mu == pytest.approx(1.0 / math.sqrt(0.2 * 50.0), rel=1e-10)


@pytest.mark.parametrize("kind", SN.SCALINGS)
def test_every_scaling_solves_the_small_workload(kind):
    A, L = lyapgen.random_shift(1, 64, 2)
    X = E.kron_solve(A, L @ L.T)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("fp32", "fp64", "fp64", "fp64"), tol=1e-13,
                            scaling=kind)
    assert info.status == "OK"
    assert R.relres(A, L, None, Z, d) <= 1e-13
    assert _rel((Z * d) @ Z.T, X) <= 1e-10
    seq = SN.a_sequence(A, "fp64", scaling_kind=kind)
    assert np.trace(seq.A_last) == pytest.approx(-64.0, abs=1e-8)


# -------------------------------------------------------------------------- warm start
def _exact_factor(A, L, S=None):
    X = E.bartels_stewart(A, E.form_w(L, S))
    w, V = np.linalg.eigh(0.5 * (X + X.T))
    keep = np.abs(w) > 1e-15 * np.abs(w).max()
    return V[:, keep], w[keep], X


def test_warm_start_from_the_solution_needs_no_correction():
    A, L = lyapgen.random_shift(2, 48, 3)
    Z0, d0, X = _exact_factor(A, L)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("fp16", "fp64", "fp64", "fp64"), tol=1e-13,
                            Z0=Z0, d0=d0)
    assert info.status == "OK" and info.refinements == 0 and info.inversions == 0
    assert len(info.res_hist) == 1 and info.res_hist[0] <= 1e-13


def test_warm_start_from_a_perturbed_solution_refines_it():
    A, L = lyapgen.random_shift(2, 48, 3)
    Z0, d0, X = _exact_factor(A, L)
    rng = np.random.default_rng(1)
    Zp = Z0 + 1e-5 * rng.standard_normal(Z0.shape)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("fp32", "fp64", "fp64", "fp64"), tol=1e-13,
                            Z0=Zp, d0=d0)
    assert info.res_hist[0] > 1e-9
    assert info.status == "OK" and info.refinements >= 1 and info.inversions > 0
    assert _rel((Z * d) @ Z.T, X) <= 1e-10


# -------------------------------------------------------------------------- escalation
def test_escalation_rescues_bf16_beyond_its_condition_bound():
    # Table 3.1: bf16 fails far beyond kappa ~ 1e3 (see test_oracle_refine); escalating
    # through fp16 to fp32 converges and reports the precision that finished.
    A, L = lyapgen.paper_family(60, 6.0, seed=3)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("bf16", "fp64", "fp64", "fp64"), tol=1e-13,
                            escalate=True)
    assert info.status == "OK" and info.escalations >= 1
    assert info.u_s_final in ("fp16", "fp32", "fp64")
    assert R.relres(A, L, None, Z, d) <= 1e-13


def test_escalation_is_not_used_when_the_first_precision_converges():
    A, L = lyapgen.random_shift(1, 64, 2)
    _, _, info = IR.ir_ldlt(A, L, None, prec=("fp16", "fp64", "fp64", "fp64"), tol=1e-13,
                            escalate=True)
    assert info.status == "OK" and info.escalations == 0 and info.u_s_final == "fp16"


# ------------------------------------------------------------------ working precision fp32
@pytest.mark.parametrize("us", ["fp32", "fp16"])
def test_working_precision_fp32_stores_binary32_factors(us):
    A, L = lyapgen.random_shift(3, 64, 2)
    X = E.kron_solve(A, L @ L.T)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=(us, "fp32", "fp32", "fp32"), tol=1e-7)
    assert info.status == "OK"
    # stored at u: every entry is a binary32 number
    assert np.array_equal(fl(Z, "fp32"), Z) and np.array_equal(fl(d, "fp32"), d)
    res = R.relres(A, L, None, Z, d)
    assert res <= 1e-7
    # the limiting accuracy is binary32's: far above binary64 rounding, within kappa u_32
    assert _rel((Z * d) @ Z.T, X) <= 1e3 * unit_roundoff("fp32")


def test_working_precision_fp32_stagnates_at_the_binary32_level():
    # Table 3.1: with u = fp32 a residual of 1e-13 is out of reach; refinement stalls near
    # the binary32 level and the eq (4.2) rule ends it
    A, L = lyapgen.random_shift(3, 64, 2)
    _, _, info = IR.ir_ldlt(A, L, None, prec=("fp32", "fp32", "fp32", "fp32"), tol=1e-13)
    assert info.status == "STAGNATED"
    assert 1e-10 < info.res < 1e-6


# ------------------------------------------------------------------------------ full S
def test_full_symmetric_s_equals_its_diagonalisation():
    rng = np.random.default_rng(11)
    A, L = lyapgen.random_shift(4, 40, 3)
    B = rng.standard_normal((3, 3))
    S = B + B.T  # symmetric, indefinite in general
    X = E.kron_solve(A, L @ S @ L.T)
    Z, d, info = IR.ir_ldlt(A, L, S, prec=("fp32", "fp64", "fp64", "fp64"), tol=1e-13)
    assert info.status == "OK"
    assert _rel((Z * d) @ Z.T, X) <= 1e-10
    assert R.relres_dense(A, L @ S @ L.T, (Z * d) @ Z.T) <= 1e-13


# ------------------------------------------------------------- adaptive inner tolerances
@pytest.mark.parametrize("us", ["fp32", "fp16"])
def test_adaptive_tolerances_keep_the_accuracy_and_not_the_rank(us):
    # Inexact inner solves (Conclusions): the correction truncated at eta_r/10 and the update
    # at omega res_i still reach tau_I, the solution is as accurate, and the factor is not
    # larger than with the fixed thresholds (up to the rounding path: a few columns)
    A, L, Q, T = lyapgen.schur_family(3, 200, 4, lo=-3.0, upper_std_scale=0.003)
    X = E.schur_solve(Q, T, L @ L.T)
    Zf, df, fixed = IR.ir_ldlt(A, L, None, prec=(us, "fp64", "fp64", "fp64"))
    Za, da, adapt = IR.ir_ldlt(A, L, None, prec=(us, "fp64", "fp64", "fp64"), adaptive=True,
                               omega=1e-3)
    assert fixed.status == adapt.status == "OK"
    assert R.relres(A, L, None, Za, da) <= 1e-13
    assert adapt.rank <= 1.05 * fixed.rank + 2
    assert _rel((Za * da) @ Za.T, X) <= 1e-10
    # the update threshold follows the residual: a larger omega drops more
    Zb, db, loose = IR.ir_ldlt(A, L, None, prec=(us, "fp64", "fp64", "fp64"), adaptive=True,
                               omega=1e-1)
    assert loose.status == "OK" and loose.rank < fixed.rank
    assert R.relres(A, L, None, Zb, db) <= 1e-13



def test_adaptive_thresholds_fall_back_when_a_step_does_not_contract():
    # an update threshold far too loose (omega = 1e4 drops nearly everything) makes a step fail
    # to halve the residual; the inexact thresholds are then switched off and the refinement
    # still reaches tau_I (without the fallback it stagnates: eq 4.2)
    A, L, Q, T = lyapgen.schur_family(3, 120, 3, lo=-2.0, upper_std_scale=0.003)
    X = E.schur_solve(Q, T, L @ L.T)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("fp32", "fp64", "fp64", "fp64"), adaptive=True,
                            omega=1e4)
    h = info.res_hist
    assert any(h[i] > 0.5 * h[i - 1] for i in range(1, len(h)))
    assert info.status == "OK" and info.res_hist[-1] <= 1e-13
    assert _rel((Z * d) @ Z.T, X) <= 1e-10


@pytest.mark.parametrize("us", ["fp64", "fp16"])
def test_zero_right_hand_side_gives_the_zero_solution(us):
    # W = 0: X = 0 solves the equation exactly; eq (4.1) is 0/0 there and is read as 0
    A, _ = lyapgen.random_shift(1, 32, 2)
    Z, d, info = IR.ir_ldlt(A, np.zeros((32, 2)), None, prec=(us, "fp64", "fp64", "fp64"))
    assert info.status == "OK" and info.rank == 0 and info.res_hist == [0.0]
    assert R.relres(A, np.zeros((32, 2)), None, Z, d) == 0.0


@pytest.mark.parametrize("us", ["fp64", "fp32", "fp16", "bf16"])
def test_order_one_equation(us):
    # n = 1: a x + x a + l^2 s = 0, x = -l^2 s / (2 a)
    Z, d, info = IR.ir_ldlt(np.array([[-3.0]]), np.array([[2.0, 1.0]]), np.array([1.0, -2.0]),
                            prec=(us, "fp64", "fp64", "fp64"))
    assert info.status == "OK"
    assert float(((Z * d) @ Z.T)[0, 0]) == pytest.approx((4.0 - 2.0) / 6.0, rel=1e-13)
