"""Mixed-precision iterative refinement for low-rank Lyapunov equations (test infrastructure).

Section 2 of the paper:

* ``res_fac_chol``  -- Fragment 2.1: F = [Z, AZ, L], thin QR F = U T, H = T P T^T with
  P = [[0, I, 0], [I, 0, 0], [0, 0, I_m]], H = Q Lambda Q^T, split into the PSD/NSD parts
  L+ = U Q+ Lambda+^(1/2), L- = U Q- (-Lambda-)^(1/2) with truncation at eta_r.
* ``sol_upt_chol``  -- Fragment 2.2: G = [Z, Z+, Z-], G = V Gamma, K = Gamma J Gamma^T with
  J = blkdiag(I, I, -I), K = Theta Sigma Theta^T, keep sigma >= eta_s (PSD projection),
  Z = V Theta_t Sigma_t^(1/2).
* ``res_fac_ldlt``  -- Fragment 2.3: H = T N T^T with N = [[0, Y, 0], [Y, 0, 0], [0, 0, S]],
  keep |lambda| >= eta_r, L^D = U Q_t, S^D = Lambda_t.
* ``sol_upt_ldlt``  -- Fragment 2.4: G = [Z, Z^D], Upsilon = blkdiag(Y, Y^D), K = Gamma
  Upsilon Gamma^T, keep sigma >= eta_s, Z = V Theta_t, Y = Sigma_t.
* ``ir_chol``/``ir_ldlt`` -- Alg 2.1 / Alg 2.2 with the sign-function Newton solver, the
  cache-fit reuse of the inverse sequence (Section 3.4) and the Section 4.1 parameters:
  tau_I (default 1e-13), i_max = 50, k_max = 50, rho = 0.1, eta_s = 10u, eta_r = 1e-4, and
  the stagnation test (4.2): stop when res_i/res_{i-1} > 0.9 twice in a row.

Readings taken where the paper is terse:
* the truncation thresholds eta_r and eta_s are relative to the largest eigenvalue
  magnitude (the analysis bounds the dropped part relative to ||Lambda||);
* the stopping test compares the relative residual of eq (4.1) with tau_I;
* on ``break`` the current (Z_i, Y_i) is returned;
* for an indefinite S the PSD projection is switched off: the solution update keeps
  |sigma| >= eta_s max|sigma| with signs, and RankTruncLdlt keeps |lambda|;
* a non-diagonal S is diagonalised once (S = Q_s diag(s) Q_s^T, L <- L Q_s);
* the reduced-precision correction is solved for 2^-e times the residual factor (a power of
  two making the largest |S^D| about 1) and the solution factor is scaled back by 2^e in
  the working precision, so residual-sized values stay in the fp16 range; for the Cholesky
  form the factors L+ and L- are scaled by 2^-e (the right-hand side by 2^-2e).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .precision import fl, fl_scaled, unit_roundoff
from .adi import adi_sequence, lr_adi_ldlt
from .signnewton import NonFiniteError, NotStableError, a_sequence, sign_newton_chol, sign_newton_ldlt


def _qr(M, fmt):
    dt = np.float64 if fmt == "fp64" else np.float32
    q, r = np.linalg.qr(fl(M, fmt).astype(dt), mode="reduced")
    return q.astype(np.float64), r.astype(np.float64)


def _eigh(M, fmt):
    dt = np.float64 if fmt == "fp64" else np.float32
    w, v = np.linalg.eigh((0.5 * (M + M.T)).astype(dt))
    return w.astype(np.float64), v.astype(np.float64)


def _mm(a, b, fmt):
    if fmt == "fp64":
        return a @ b
    return fl((fl(a, fmt).astype(np.float32) @ fl(b, fmt).astype(np.float32)).astype(np.float64), fmt)


# ----------------------------------------------------------------- Cholesky fragments
def res_fac_chol(A, L, Z, eta_r: float, fmt: str = "fp64"):
    """Fragment 2.1.  Returns (L+, L-, ||R||_F)."""
    c, m = Z.shape[1], L.shape[1]
    F = np.hstack([Z, _mm(A, Z, fmt), L])
    U, T = _qr(F, fmt)
    P = np.zeros((2 * c + m, 2 * c + m))
    P[:c, c:2 * c] = np.eye(c)
    P[c:2 * c, :c] = np.eye(c)
    P[2 * c:, 2 * c:] = np.eye(m)
    H = _mm(_mm(T, P, fmt), T.T, fmt)
    lam, Q = _eigh(H, fmt)
    normR = float(np.linalg.norm(lam))
    thr = eta_r * float(np.max(np.abs(lam))) if lam.size else 0.0
    jp = lam >= thr
    jm = lam <= -thr
    Lp = _mm(U, Q[:, jp], fmt) * np.sqrt(lam[jp])[None, :]
    Lm = _mm(U, Q[:, jm], fmt) * np.sqrt(-lam[jm])[None, :]
    return fl(Lp, fmt), fl(Lm, fmt), normR


def sol_upt_chol(Z, Zp, Zm, eta_s: float, fmt: str = "fp64"):
    """Fragment 2.2 (with projection onto the PSD cone)."""
    G = np.hstack([Z, Zp, Zm])
    V, Gam = _qr(G, fmt)
    J = np.concatenate([np.ones(Z.shape[1] + Zp.shape[1]), -np.ones(Zm.shape[1])])
    K = _mm(Gam * J[None, :], Gam.T, fmt)
    sig, Th = _eigh(K, fmt)
    thr = eta_s * float(np.max(np.abs(sig)))
    keep = sig >= thr
    return fl(_mm(V, Th[:, keep], fmt) * np.sqrt(sig[keep])[None, :], fmt)


# -------------------------------------------------------------------- LDL^T fragments
def res_fac_ldlt(A, L, S, Z, Y, eta_r: float, fmt: str = "fp64"):
    """Fragment 2.3.  ``S`` and ``Y`` are matrices.  Returns (L^D, s^D (1-D), ||R||_F)."""
    c, m = Z.shape[1], L.shape[1]
    F = np.hstack([Z, _mm(A, Z, fmt), L])
    U, T = _qr(F, fmt)
    N = np.zeros((2 * c + m, 2 * c + m))
    N[:c, c:2 * c] = Y
    N[c:2 * c, :c] = Y
    N[2 * c:, 2 * c:] = S
    H = _mm(_mm(T, N, fmt), T.T, fmt)
    lam, Q = _eigh(H, fmt)
    normR = float(np.linalg.norm(lam))
    thr = eta_r * float(np.max(np.abs(lam))) if lam.size else 0.0
    keep = np.abs(lam) >= thr
    return fl(_mm(U, Q[:, keep], fmt), fmt), fl(lam[keep], fmt), normR


def sol_upt_ldlt(Z, Y, Zd, Yd, eta_s: float, fmt: str = "fp64", psd: bool = True):
    """Fragment 2.4.  Returns (Z_{i+1}, Y_{i+1}) with Y diagonal (matrix)."""
    G = np.hstack([Z, Zd])
    Ups = sla.block_diag(Y, Yd)
    V, Gam = _qr(G, fmt)
    K = _mm(_mm(Gam, Ups, fmt), Gam.T, fmt)
    sig, Th = _eigh(K, fmt)
    thr = eta_s * float(np.max(np.abs(sig)))
    keep = sig >= thr if psd else np.abs(sig) >= thr
    return fl(_mm(V, Th[:, keep], fmt), fmt), np.diag(fl(sig[keep], fmt))


# ------------------------------------------------------------------------ IR driver
@dataclass
class IRInfo:
    status: str = "OK"             # OK, NOT_CONVERGED, STAGNATED
    res_hist: list = field(default_factory=list)
    newton_total: int = 0          # varsigma: Newton iterations over all solver calls
    newton_max: int = 0            # alpha: largest count in one call
    inversions: int = 0            # inverses actually computed (cache-fit)
    refinements: int = 0           # correction solves performed
    rank: int = 0
    mus: list = field(default_factory=list)
    u_s_final: str = ""            # solver precision of the last stage (escalation)
    escalations: int = 0

    @property
    def res(self) -> float:
        return self.res_hist[-1] if self.res_hist else float("nan")


def _norm_ldlt(Z, Y):
    """||Z Y Z^T||_F through the trace identity ||ZYZ^T||_F^2 = tr((Z^T Z Y)^2)."""
    G = Z.T @ Z @ Y
    return math.sqrt(max(float(np.trace(G @ G)), 0.0))


def _prep_S(L, S):
    """Diagonalise S once: S = Q_s diag(s) Q_s^T, L <- L Q_s (exact orthogonal change)."""
    m = L.shape[1]
    if S is None:
        return np.asarray(L, np.float64), np.ones(m), True
    S = np.asarray(S, np.float64)
    if S.ndim == 1:
        return np.asarray(L, np.float64), S.copy(), bool(np.all(S >= 0))
    s, Qs = np.linalg.eigh(0.5 * (S + S.T))
    return np.asarray(L, np.float64) @ Qs, s, bool(np.all(s >= 0))


def stagnated(res_hist, theta: float = 0.9) -> bool:
    """The early stop of eq (4.2): with theta_i = res_i / res_{i-1}, refinement is stopped once
    theta_i > theta for two consecutive steps, i.e. the last two ratios of ``res_hist`` (the
    residuals res_0, res_1, ... of the iterates so far) both exceed ``theta``."""
    h = list(res_hist)
    if len(h) < 3:
        return False
    return h[-1] > theta * h[-2] and h[-2] > theta * h[-3]


def _pow2_exponent(x: float) -> int:
    """e with 2^(e-1) <= x < 2^e (x > 0)."""
    return math.frexp(x)[1]


def _next_up(fmt: str) -> str:
    """The next solver precision up in unit roundoff (Table 1.1): bf16, fp16, fp32, fp64."""
    return {"bf16": "fp16", "fp16": "fp32", "fp32": "fp64"}.get(fmt, "fp64")


def ir_ldlt(A, L, S=None, prec=("fp32", "fp64", "fp64", "fp64"), tol: float = 1e-13,
            i_max: int = 50, k_max: int = 50, rho: float = 0.1, eta_r: float = 1e-4,
            eta_s: float | None = None, psd: bool | None = None, theta: float = 0.9,
            refine: bool = True, scaling: str = "frobenius", Z0=None, d0=None,
            escalate: bool = False, adaptive: bool = False, omega: float = 0.1,
            solver: str = "newton", adi_shifts: int = 0, adi_max: int = 100):
    """Alg 2.2 with Alg 3.2 as the solver (``solver="adi"``: the LDL^T low-rank ADI solver of
    ``oracle.adi`` on its cached shifted inverses instead).  ``prec`` = (u_s, u, u_r, u_c).  With
    ``refine=False`` only the first solve is made and its residual evaluated (plain
    sign-function Newton).  ``Z0``, ``d0``: start the refinement from X_0 = Z0 diag(d0) Z0^T
    instead of a first solve (the first line of Alg 2.2 accepts any starting factor); the
    inverse sequence is then formed only if a correction is needed.  ``escalate``: a stage
    that stagnates (eq 4.2), runs out of steps or overflows at u_s continues at the next
    precision up (Table 1.1 order, not beyond u), from the current iterate when it is valid.
    ``adaptive``: inexact inner solves with tolerances tied to the refinement (the direction
    the Conclusions point to): each correction solve truncates at max(u_s, eta_r / 10)
    relative (the residual factor is itself truncated at eta_r, so a more accurate correction
    buys nothing), and the update after a step with residual res_i keeps
    sigma >= max(eta_s, omega res_i) max|sigma| (directions that small only change the next
    residual by about omega res_i, far below the contraction of a refinement step).  Because
    that holds only for directions the next correction fixes, a step that contracts the
    residual by less than half (res_i > res_{i-1} / 2) switches both inexact thresholds off
    for the rest of the refinement.
    Returns (Z, d, info) with X ~ Z diag(d) Z^T."""
    us, u, ur, uc = prec
    A = np.asarray(A, np.float64)
    L, s, psd_auto = _prep_S(L, S)
    psd = psd_auto if psd is None else psd
    if eta_s is None:
        eta_s = 10.0 * unit_roundoff(u)
    Sm = np.diag(s)
    info = IRInfo()
    info.u_s_final = us
    info.escalations = 0
    normA = float(np.linalg.norm(A, "fro"))
    normW = _norm_ldlt(L, Sm)
    seq = None
    steps_left = i_max

    def make_sequence(us_):
        if solver == "adi":
            sq = adi_sequence(A, us_, adi_shifts)
            info.inversions += sq.J + 1
            info.mus = list(sq.shifts)
        else:
            sq = a_sequence(A, us_, k_max, scaling_kind=scaling)
            info.inversions += sq.K
            info.mus = list(sq.mus)
        return sq

    def inner(us_, sq, G, sv, psd_, tol_in):
        """One solve at u_s on the sequence; returns (Z, Y, inner iteration count)."""
        if solver == "adi":
            Zi, di, ai = lr_adi_ldlt(A, G, sv, us_, sq, psd_, rho, tol_in or 0.0, adi_max)
            return Zi, np.diag(di), ai.steps
        Zi, Yi, _, _ = sign_newton_ldlt(A, fl_scaled(G, us_, axis=0), sv, us_, psd=psd_,
                                        rho=rho, seq=sq, trunc_tol=tol_in)
        return Zi, Yi, sq.K

    if Z0 is not None:
        Z, Y = fl(np.asarray(Z0, np.float64), u), fl(np.diag(np.asarray(d0, np.float64)), u)
        fresh = False
    else:
        Z = Y = None
        fresh = True
    while True:
        status = "OK"
        try:
            if fresh:
                seq = make_sequence(us)
                Z, Y, its = inner(us, seq, L, s if solver == "adi" else Sm, psd, None)
                Z, Y = fl(Z, u), fl(Y, u)
                info.newton_total += its
                info.newton_max = max(info.newton_max, its)
            hist = []
            budget = steps_left
            inexact = adaptive
            for i in range(1, budget + 1):
                Ld, sd, normR = res_fac_ldlt(A, L, Sm, Z, Y, eta_r, ur)
                den = normW + 2.0 * _norm_ldlt(Z, Y) * normA
                # W = 0 and X = 0: the exact solution, R = 0 (eq 4.1 read as 0, not 0/0)
                res = normR / den if den > 0.0 else (0.0 if normR == 0.0 else math.inf)
                info.res_hist.append(res)
                hist.append(res)
                if inexact and len(hist) >= 2 and hist[-1] > 0.5 * hist[-2]:
                    inexact = False
                if not np.isfinite(res):
                    raise NonFiniteError("non-finite residual")
                if res <= tol:
                    break
                if not refine:
                    status = "NOT_CONVERGED"
                    break
                if stagnated(hist, theta):
                    status = "STAGNATED"
                    break
                if i == budget:
                    status = "NOT_CONVERGED"
                    break
                if seq is None:
                    seq = make_sequence(us)
                # scale the correction's right-hand side by a power of two (linearity)
                e = _pow2_exponent(float(np.max(np.abs(sd))))
                sd_s = fl(np.ldexp(sd, -e), us)
                Zd, Yd, its = inner(us, seq, Ld, sd_s, False, eta_r / 10.0 if inexact else None)
                Zd, Yd = fl(Zd, u), np.ldexp(fl(Yd, u), e)
                info.newton_total += its
                info.newton_max = max(info.newton_max, its)
                info.refinements += 1
                steps_left -= 1
                eta_i = max(eta_s, omega * res) if inexact else eta_s
                Z, Y = sol_upt_ldlt(Z, Y, Zd, Yd, eta_i, uc, psd)
        except NonFiniteError:
            status = "NONFINITE"
        except NotStableError:
            status = "NOT_STABLE"
        except np.linalg.LinAlgError:
            status = "SINGULAR"
        info.status = status
        if not (escalate and refine and status != "OK"
                and unit_roundoff(us) > unit_roundoff(u)):
            break
        valid = status in ("STAGNATED", "NOT_CONVERGED") and Z is not None
        us = _next_up(us)
        info.u_s_final = us
        info.escalations += 1
        seq = None
        steps_left = max(1, steps_left)
        fresh = not valid
    if Z is None:
        Z, Y = np.zeros((A.shape[0], 0)), np.zeros((0, 0))
    info.rank = Z.shape[1]
    d = np.diag(Y).copy() if Y.ndim == 2 else Y
    return Z, d, info


def ir_chol(A, L, prec=("fp32", "fp64", "fp64", "fp64"), tol: float = 1e-13,
            i_max: int = 50, k_max: int = 50, rho: float = 0.1, eta_r: float = 1e-4,
            eta_s: float | None = None, theta: float = 0.9, refine: bool = True):
    """Alg 2.1 with Alg 3.1 as the solver (the two correction equations share the inverse
    sequence).  Returns (Z, info) with X ~ Z Z^T."""
    us, u, ur, uc = prec
    A = np.asarray(A, np.float64)
    L = np.asarray(L, np.float64)
    if eta_s is None:
        eta_s = 10.0 * unit_roundoff(u)
    info = IRInfo()
    seq = a_sequence(A, us, k_max)
    info.inversions = seq.K
    info.mus = list(seq.mus)
    Z, _, _ = sign_newton_chol(A, L, us, rho=rho, seq=seq)
    Z = fl(Z, u)
    info.newton_total = info.newton_max = seq.K
    normA = float(np.linalg.norm(A, "fro"))
    G = L.T @ L
    normW = math.sqrt(float(np.trace(G @ G)))
    for i in range(1, i_max + 1):
        Lp, Lm, normR = res_fac_chol(A, L, Z, eta_r, ur)
        Gz = Z.T @ Z
        den = normW + 2.0 * math.sqrt(float(np.trace(Gz @ Gz))) * normA
        res = normR / den if den > 0.0 else (0.0 if normR == 0.0 else math.inf)
        info.res_hist.append(res)
        if res <= tol:
            break
        if not refine:
            info.status = "NOT_CONVERGED"
            break
        if stagnated(info.res_hist, theta):
            info.status = "STAGNATED"
            break
        if i == i_max:
            info.status = "NOT_CONVERGED"
            break
        big = max(float(np.max(np.abs(Lp))) if Lp.size else 0.0,
                  float(np.max(np.abs(Lm))) if Lm.size else 0.0)
        e = _pow2_exponent(big) if big > 0 else 0
        outs = []
        for Lx in (Lp, Lm):
            if Lx.shape[1] == 0:
                outs.append(np.zeros((A.shape[0], 0)))
                continue
            Zx, _, _ = sign_newton_chol(A, fl_scaled(np.ldexp(Lx, -e), us, axis=0), us, rho=rho, seq=seq)
            outs.append(np.ldexp(fl(Zx, u), e))
        info.newton_total += seq.K
        info.refinements += 1
        Z = sol_upt_chol(Z, outs[0], outs[1], eta_s, uc)
    info.rank = Z.shape[1]
    return Z, info
