"""Pins for oracle.refine (Section 2): the residual factorisations reproduce the explicit
residual, the solution updates reproduce X_i + X^D before truncation, and the IR loops reach
the exact solution (Kronecker / Bartels-Stewart) at every solver precision of Table 3.1."""
import numpy as np
import pytest

import lyapgen
from oracle import exact as E
from oracle import refine as IR
from oracle import residual as R
from oracle.precision import unit_roundoff


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _approx_solution(A, L, seed, scale=1e-3):
    """A perturbed LDL^T factorisation of the true solution (a refinement iterate)."""
    X = E.bartels_stewart(A, L @ L.T)
    w, V = np.linalg.eigh(X)
    keep = w > 1e-14 * w.max()
    Z, y = V[:, keep], w[keep]
    rng = np.random.default_rng(seed)
    return Z + scale * rng.standard_normal(Z.shape) / np.sqrt(Z.shape[0]), y


def test_res_fac_ldlt_reproduces_explicit_residual():
    A, L = lyapgen.random_shift(1, 60, 2)
    Z, y = _approx_solution(A, L, 0)
    S = np.eye(2)
    Ld, sd, normR = IR.res_fac_ldlt(A, L, S, Z, np.diag(y), eta_r=0.0)
    Rm = R.residual_matrix(A, L, None, Z, y)
    assert normR == pytest.approx(np.linalg.norm(Rm), rel=1e-10)
    assert np.linalg.norm(Ld @ np.diag(sd) @ Ld.T - Rm) <= 1e-12 * np.linalg.norm(Rm)
    # truncation at eta_r drops at most sqrt(p) eta_r ||Lambda||_2 in Frobenius norm
    Ld, sd, _ = IR.res_fac_ldlt(A, L, S, Z, np.diag(y), eta_r=1e-4)
    p = 2 * Z.shape[1] + 2
    err = np.linalg.norm(Ld @ np.diag(sd) @ Ld.T - Rm)
    assert err <= np.sqrt(p) * 1e-4 * np.abs(np.linalg.eigvalsh(Rm)).max()


def test_res_fac_chol_reproduces_explicit_residual():
    A, L = lyapgen.random_shift(2, 50, 3)
    Zs, y = _approx_solution(A, L, 1)
    Z = Zs * np.sqrt(y)[None, :]
    Lp, Lm, normR = IR.res_fac_chol(A, L, Z, eta_r=0.0)
    Rm = R.residual_matrix(A, L, None, Z)
    assert normR == pytest.approx(np.linalg.norm(Rm), rel=1e-10)
    assert np.linalg.norm(Lp @ Lp.T - Lm @ Lm.T - Rm) <= 1e-12 * np.linalg.norm(Rm)


def test_sol_upt_ldlt_reproduces_sum_before_truncation():
    rng = np.random.default_rng(3)
    n = 80
    Z = np.linalg.qr(rng.standard_normal((n, 10)))[0]
    Y = np.diag(np.logspace(0, -3, 10))
    Zd = rng.standard_normal((n, 6))
    Yd = np.diag(rng.standard_normal(6) * 1e-2)
    Zn, Yn = IR.sol_upt_ldlt(Z, Y, Zd, Yd, eta_s=0.0, psd=False)
    Xs = Z @ Y @ Z.T + Zd @ Yd @ Zd.T
    assert _rel(Zn @ Yn @ Zn.T, Xs) <= 1e-13
    assert np.allclose(Zn.T @ Zn, np.eye(Zn.shape[1]), atol=1e-13)
    # with projection the negative part is removed: the result is the PSD part of the sum
    Zp, Yp = IR.sol_upt_ldlt(Z, Y, Zd, Yd, eta_s=0.0, psd=True)
    w, V = np.linalg.eigh(Xs)
    Xplus = (V * np.maximum(w, 0)) @ V.T
    assert _rel(Zp @ Yp @ Zp.T, Xplus) <= 1e-12


def test_sol_upt_chol_projects_onto_psd_cone():
    rng = np.random.default_rng(4)
    n = 60
    Z = rng.standard_normal((n, 8))
    Zp = 0.1 * rng.standard_normal((n, 3))
    Zm = 0.1 * rng.standard_normal((n, 2))
    Zn = IR.sol_upt_chol(Z, Zp, Zm, eta_s=0.0)
    Xs = Z @ Z.T + Zp @ Zp.T - Zm @ Zm.T
    w, V = np.linalg.eigh(Xs)
    assert _rel(Zn @ Zn.T, (V * np.maximum(w, 0)) @ V.T) <= 1e-12


@pytest.mark.parametrize("us", ["fp64", "fp32", "fp16", "bf16"])
def test_ir_ldlt_reaches_exact_solution(us):
    A, L = lyapgen.random_shift(1, 64, 2)
    X = E.kron_solve(A, L @ L.T)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=(us, "fp64", "fp64", "fp64"), tol=1e-13)
    assert info.status == "OK"
    res = R.relres(A, L, None, Z, d)
    assert res <= 1e-13
    assert info.res == pytest.approx(res, rel=1e-3, abs=1e-16)
    assert _rel((Z * d) @ Z.T, X) <= 1e-11
    assert info.inversions == info.newton_max   # cache-fit: inverses computed once
    if us == "fp64":
        assert info.refinements == 0


def test_ir_chol_matches_ldlt():
    A, L = lyapgen.random_shift(1, 64, 2)
    X = E.kron_solve(A, L @ L.T)
    Z, info = IR.ir_chol(A, L, prec=("fp32", "fp64", "fp64", "fp64"), tol=1e-13)
    assert info.status == "OK"
    assert R.relres(A, L, None, Z) <= 1e-13
    assert _rel(Z @ Z.T, X) <= 1e-11


def test_ir_indefinite_rhs():
    A, L = lyapgen.random_shift(2, 48, 4)
    s = np.array([1.0, -1.0, -1.0, 1.0])
    X = E.kron_solve(A, E.form_w(L, s))
    Z, d, info = IR.ir_ldlt(A, L, s, prec=("fp16", "fp64", "fp64", "fp64"), tol=1e-13)
    assert info.status == "OK"
    assert np.any(d < 0) and np.any(d > 0)
    assert _rel((Z * d) @ Z.T, X) <= 1e-11


def test_ir_working_precision_fp32_limits_residual():
    # Table 3.1: with u = fp32 the limiting residual is fp32-level.
    A, L = lyapgen.random_shift(3, 64, 2)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("fp32", "fp32", "fp32", "fp32"),
                            tol=64 * unit_roundoff("fp32"))
    assert info.status == "OK"
    assert R.relres(A, L, None, Z, d) <= 1e-5


def test_ir_bf16_beyond_condition_bound_does_not_converge():
    # Table 3.1: bf16 needs kappa_F(L) below about 1e3; far beyond it IR cannot reach 1e-13.
    # Either the bf16 A-iteration itself never meets its stopping test, or refinement stalls.
    A, L = lyapgen.paper_family(60, 6.0, seed=3)
    Z, d, info = IR.ir_ldlt(A, L, None, prec=("bf16", "fp64", "fp64", "fp64"), tol=1e-13)
    assert info.status in ("STAGNATED", "NOT_CONVERGED", "NOT_STABLE", "NONFINITE")
    if info.res_hist:
        assert info.res > 1e-13
