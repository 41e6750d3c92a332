"""Low-rank ADI as a second inner solver of the refinement (test infrastructure).

Section 3 states that the precision settings of the refinement carry over when the inner
solver is another low-rank method, naming the low-rank ADI method, and the Conclusions
leave that combination as an open direction.  This module is that inner solver in the LDL^T
form, written from the published method; nothing here is from the paper beyond that
statement.

* ``lr_adi_ldlt``   -- residual-factor LR-ADI with real shifts in LDL^T form (Penzl 2000;
  Benner, Li and Penzl 2008; Lang, Mena and Saak 2015): with W_0 = G,
      V_j = (A + p_j I)^{-1} W_{j-1},   W_j = W_{j-1} - 2 p_j V_j,
      Z_j = [Z_{j-1}, V_j],             D_j = blkdiag(D_{j-1}, -2 p_j S),
  for A X + X A^T + G S G^T = 0 with every p_j < 0.  The residual of X_j = Z_j D_j Z_j^T is
  exactly W_j S W_j^T, so its norm comes from an m x m Gram matrix.  The J shifts are used
  cyclically; the products run at the solver precision on the cached inverses
  (A + p_j I)^{-1}, and Z is truncated by RankTruncLdlt whenever it has more than rho n
  columns, as in the Newton solver.
* ``wachspress_shifts`` -- the optimal real shifts for a spectrum in [-b, -a] (Wachspress
  1962): p_i = -b dn((2i - 1) K / (2J), k), k = sqrt(1 - (a/b)^2), K = K(k), and the number
  of shifts J = ceil(K ln(4/eps) / (pi K')) (K' = K(a/b)) that brings the ADI error
  function max |prod (x - |p_i|) / (x + |p_i|)| over [a, b] below eps.
* ``spectral_interval`` -- b = rho(A) and a = 1 / rho(A^{-1}) by power iteration (24 steps
  from x_0 = ones / sqrt(n); the estimate is the geometric mean of the growth factors
  ||M x_t|| of the last 12 steps), with A^{-1} at max(u_s, fp32).
* ``adi_sequence``  -- interval, shifts and the cached shifted inverses at u_s.

Readings (the paper gives none of these):
* shifts for a reduction of sqrt(u_s) per cycle (two cycles reach u_s); ``shifts``
  overrides J;
* the solve stops when ||W_j S W_j^T||_F <= max(10 u_s, tol_inner) ||G S G^T||_F, where
  tol_inner is the adaptive inner tolerance of the refinement (0 when off), or after
  ``max_steps`` steps;
* the interval inverse is formed at binary32 for the fp16 / bf16 solvers (their inverse is
  too inaccurate for the smallest eigenvalue at kappa ~ 1e3).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.special as ss

from .precision import fl, matmul, unit_roundoff
from .signnewton import NonFiniteError, inverse_at, rank_trunc_ldlt

RHO_ITERS = 24


def power_rho(M, iters: int = RHO_ITERS) -> float:
    """Spectral-radius estimate: x_0 = ones/sqrt(n), x_t = M x_{t-1} / ||M x_{t-1}||; the
    geometric mean of ||M x_{t-1}|| over the last iters - iters // 2 steps."""
    n = M.shape[0]
    x = np.full(n, 1.0 / math.sqrt(n))
    half = iters // 2
    logs = []
    for t in range(iters):
        y = M @ x
        nr = float(np.linalg.norm(y))
        x = y / nr if nr > 0.0 else y
        if t >= half:
            logs.append(math.log(nr))
    return math.exp(sum(logs) / len(logs))


def interval_fmt(us: str) -> str:
    return "fp64" if us == "fp64" else "fp32"


def spectral_interval(A, us: str):
    """(a, b) with -spec(A) inside [a, b] as estimated by power iteration."""
    b = power_rho(A)
    a = 1.0 / power_rho(inverse_at(A, interval_fmt(us)))
    if not (np.isfinite(a) and np.isfinite(b) and a > 0.0 and b > 0.0):
        raise NonFiniteError("spectral interval estimate out of range")
    return min(a, b), b


def shift_count(a: float, b: float, eps: float) -> int:
    if a >= b:
        return 1
    kp = a / b
    K = float(ss.ellipkm1(kp * kp))          # K(k), parameter m = k^2 = 1 - kp^2
    Kp = float(ss.ellipk(kp * kp))           # K(k')
    return max(1, math.ceil(K * math.log(4.0 / eps) / (math.pi * Kp)))


def wachspress_shifts(a: float, b: float, J: int) -> np.ndarray:
    """The J optimal real ADI shifts for [a, b] (negative numbers)."""
    if a >= b:
        return -np.full(J, b)
    kp = a / b
    m = 1.0 - kp * kp
    K = float(ss.ellipkm1(kp * kp))
    u = (2.0 * np.arange(1, J + 1) - 1.0) * K / (2.0 * J)
    _, _, dn, _ = ss.ellipj(u, m)
    return -b * np.asarray(dn, np.float64)


def adi_error_function(x, shifts):
    """max-norm ADI error function r(x) = prod |(x - |p|) / (x + |p|)| at the points x > 0."""
    x = np.asarray(x, np.float64)[:, None]
    q = np.abs(np.asarray(shifts, np.float64))[None, :]
    return np.prod(np.abs((x - q) / (x + q)), axis=1)


@dataclass
class ADISequence:
    fmt: str
    a: float
    b: float
    shifts: list = field(default_factory=list)
    inverses: list = field(default_factory=list)

    @property
    def J(self) -> int:
        return len(self.shifts)


def adi_sequence(A, us: str, shifts: int = 0) -> ADISequence:
    """Interval estimate, Wachspress shifts and the shifted inverses (A + p_j I)^{-1} at
    u_s (J + 1 inversions counting the interval's)."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    a, b = spectral_interval(A, us)
    J = shifts if shifts > 0 else shift_count(a, b, math.sqrt(unit_roundoff(us)))
    ps = wachspress_shifts(a, b, J)
    seq = ADISequence(fmt=us, a=a, b=b, shifts=[float(p) for p in ps])
    for p in ps:
        C = inverse_at(A + p * np.eye(n), us)
        if not np.all(np.isfinite(C)):
            raise NonFiniteError("non-finite shifted inverse")
        seq.inverses.append(C)
    return seq


@dataclass
class ADIInfo:
    steps: int = 0
    res_hist: list = field(default_factory=list)   # ||W_j S W_j^T||_F / ||G S G^T||_F
    truncations: int = 0


def _wnorm(W, s) -> float:
    G = W.T @ W
    return math.sqrt(max(float(np.sum(np.outer(s, s) * G * G)), 0.0))


def lr_adi_ldlt(A, G, s, fmt: str, seq: ADISequence, psd: bool, rho: float = 0.1,
                tol_inner: float = 0.0, max_steps: int = 100, trans: bool = False):
    """LR-ADI for A X + X A^T + G diag(s) G^T = 0 (A^T X + X A + ... with ``trans``) on the
    cached shifted inverses.  Returns (Z, d, info) with X ~ Z diag(d) Z^T."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    s = np.asarray(s, np.float64)
    W = np.array(G, np.float64)
    cap = math.floor(rho * n)
    tol = max(10.0 * unit_roundoff(fmt), tol_inner)
    Z = np.zeros((n, 0))
    Y = np.zeros((0, 0))
    info = ADIInfo()
    nrm0 = _wnorm(W, s)
    if W.shape[1] == 0 or nrm0 == 0.0:
        return Z, np.zeros(0), info
    J = seq.J
    for t in range(max_steps):
        p = seq.shifts[t % J]
        C = seq.inverses[t % J]
        V = matmul(C.T if trans else C, W, fmt)
        W = W - 2.0 * p * V
        Z = np.hstack([Z, V])
        Y = np.diag(np.concatenate([np.diag(Y), fl(-2.0 * p * s, fmt)]))
        if Z.shape[1] > cap:
            Z, Y = rank_trunc_ldlt(Z, Y, fmt, psd, tol_inner if tol_inner > 0 else None)
            info.truncations += 1
        info.steps = t + 1
        r = _wnorm(W, s) / nrm0
        info.res_hist.append(r)
        if not np.isfinite(r):
            raise NonFiniteError("non-finite ADI residual")
        if r <= tol:
            break
    return Z, np.diag(Y).copy(), info
