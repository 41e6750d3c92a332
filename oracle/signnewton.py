"""Scaled sign-function Newton iteration for AX + XA^T + W = 0 (test infrastructure).

Follows Section 3 of the paper:

* ``dense_iteration``  -- eq (3.1): A_k = (mu A_{k-1} + mu^{-1} A_{k-1}^{-1})/2 and
  W_k = (mu W_{k-1} + mu^{-1} A_{k-1}^{-1} W_{k-1} A_{k-1}^{-T})/2; A_k -> -I, W_k -> 2X.
* ``a_sequence``       -- the A-iteration alone with Frobenius scaling
  mu = sqrt(||A^{-1}||_F / ||A||_F) (or, as alternatives Section 3 lists, the
  determinantal |det A|^{-1/n}, the 2-norm sqrt(||A^{-1}||_2 / ||A||_2) or the spectral
  sqrt(rho(A^{-1}) / rho(A)) scaling; ``scaling_mu``), scaling switched off for good once
  delta_k = ||A_k - A_{k-1}||_F / ||A_k||_F < 1e-2, and the stopping rule (3.4):
  ||A_k + I||_1 <= tau_N = 10 sqrt(n u), or (scaling already off and
  delta_k > delta_{k-1}/2), then two more iterations counting the one that met the test
  (that is, one further Newton step; this reading reproduces every iteration count of
  Table 4.1 for the fp64 and fp32 solvers, while one step more than that overshoots
  each of them by one).  Because the
  stop depends on A alone, the whole sequence of inverses and scalings can be computed
  once and replayed by every solver call (the cache-fit variant of Section 3.4).
* ``sign_newton_chol`` -- Alg 3.1, factored Cholesky form eq (3.2) with RankTruncChol
  (rank-revealing QR of Z^T, ||S||_2 <= sqrt(u) ||Z||_2).
* ``sign_newton_ldlt`` -- Alg 3.2, factored LDL^T form eq (3.3) with RankTruncLdlt
  (thin QR, spectral decomposition of R Y R^T, keep eigenvalues above u ||Lambda||_1).

Precision model: ``fmt`` is the solver precision u_s.  For fp64 everything is plain
float64; for fp32 the dense kernels run in binary32 LAPACK/BLAS; for fp16 and bf16 values
are stored rounded to the format after every matrix-level operation, products accumulate
in binary32, and the inverse is computed by Gauss-Jordan elimination with partial pivoting
in which every stored intermediate is rounded (the elementwise "chop" model the paper used).
Before each inversion A_k is scaled by a power of two so its largest entry lies in [1/2, 1)
(exact in binary arithmetic) to keep fp16 in range, and every other value held at fp16 /
bf16 (iterates A_k, factors Z, the diagonal Y, QR and spectral factors, product operands)
is stored the same way, as a power of two times a value of the format (``fl_scaled``,
per column for tall factors and for Y, whose diagonal entries are separate scalars), so
that no stored value overflows x_max of Table 1.1.
Inside the solver "u" means u_s.

The A-iteration and the factor iteration are computed one after the other rather than
interleaved as printed in Alg 3.1/3.2; nothing in the factor iteration feeds back into
A_k or the stopping test, so the results are identical.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .precision import fl, fl_scaled, matmul, unit_roundoff


class NotStableError(RuntimeError):
    """The A-iteration did not reach its stopping test within k_max steps."""


class NonFiniteError(RuntimeError):
    """An inverse or iterate became non-finite (overflow at the solver precision)."""


# ----------------------------------------------------------------------------- kernels
def _lapack_dtype(fmt):
    return np.float64 if fmt == "fp64" else np.float32


def gauss_jordan_inverse(A, fmt: str) -> np.ndarray:
    """Inverse by Gauss-Jordan elimination with partial pivoting (ties to the lowest row
    index); every stored value is rounded to ``fmt`` after each elimination step."""
    n = A.shape[0]
    M = fl(np.array(A, np.float64), fmt)
    X = np.eye(n)
    for k in range(n):
        p = k + int(np.argmax(np.abs(M[k:, k])))
        if M[p, k] == 0.0:
            raise np.linalg.LinAlgError("singular matrix")
        if p != k:
            M[[k, p]] = M[[p, k]]
            X[[k, p]] = X[[p, k]]
        piv = M[k, k]
        M[k] = fl(M[k] / piv, fmt)
        X[k] = fl(X[k] / piv, fmt)
        f = M[:, k].copy()
        f[k] = 0.0
        M = fl(M - np.outer(f, M[k]), fmt)
        X = fl(X - np.outer(f, X[k]), fmt)
    return X


def inverse_at(A, fmt: str) -> np.ndarray:
    """A^{-1} at precision ``fmt`` with a power-of-two prescaling of A."""
    A = np.asarray(A, np.float64)
    amax = float(np.max(np.abs(A)))
    if not np.isfinite(amax):
        raise NonFiniteError("non-finite iterate")
    e = math.frexp(amax)[1] if amax > 0 else 0          # 2^(e-1) <= amax < 2^e
    As = np.ldexp(A, -e)                                 # exact
    if fmt == "fp64":
        inv_s = np.linalg.inv(As)
    elif fmt == "fp32":
        inv_s = np.linalg.inv(As.astype(np.float32)).astype(np.float64)
    else:
        inv_s = gauss_jordan_inverse(As, fmt)
    return np.ldexp(inv_s, -e)                          # (2^-e A)^{-1} = 2^e A^{-1}


def thin_qr(M, fmt: str):
    """Householder thin QR (LAPACK) at precision ``fmt``."""
    dt = _lapack_dtype(fmt)
    q, r = np.linalg.qr(fl_scaled(M, fmt, axis=0).astype(dt), mode="reduced")
    return fl_scaled(q.astype(np.float64), fmt), fl_scaled(r.astype(np.float64), fmt)


def sym_eig(M, fmt: str):
    """Symmetric spectral decomposition (LAPACK) at precision ``fmt``; ascending."""
    dt = _lapack_dtype(fmt)
    Ms = fl_scaled(0.5 * (M + M.T), fmt)
    if not np.all(np.isfinite(Ms)):
        raise NonFiniteError("non-finite matrix in the spectral decomposition")
    # eigh of 2^-e Ms (exact scaling) so that the binary32 LAPACK call sees values in range
    e = int(np.frexp(np.max(np.abs(Ms)))[1]) if Ms.size and np.any(Ms) else 0
    w, v = np.linalg.eigh(np.ldexp(Ms, -e).astype(dt))
    w = np.ldexp(w.astype(np.float64), e)
    # eigenvalues are separate scalars: each keeps its own power-of-two scale
    return fl_scaled(w[None, :], fmt, axis=0)[0], fl_scaled(v.astype(np.float64), fmt)


# --------------------------------------------------------------------- dense iteration
def dense_iteration(A, W, mus):
    """eq (3.1) with prescribed scalings ``mus`` in float64; returns lists [A_k], [W_k]
    for k = 0..len(mus)."""
    Ak = np.asarray(A, np.float64)
    Wk = np.asarray(W, np.float64)
    As, Ws = [Ak], [Wk]
    for mu in mus:
        Ai = np.linalg.inv(Ak)
        Ak, Wk = 0.5 * (mu * Ak + Ai / mu), 0.5 * (mu * Wk + (Ai @ Wk @ Ai.T) / mu)
        As.append(Ak)
        Ws.append(Wk)
    return As, Ws


# ----------------------------------------------------------------------- A-iteration
@dataclass
class ASequence:
    """Inverses A_0^{-1} .. A_{K-1}^{-1}, scalings mu_0 .. mu_{K-1} and diagnostics."""
    fmt: str
    inverses: list = field(default_factory=list)
    mus: list = field(default_factory=list)
    deltas: list = field(default_factory=list)
    onenorms: list = field(default_factory=list)
    A_last: np.ndarray | None = None

    @property
    def K(self) -> int:
        return len(self.inverses)


SCALINGS = ("frobenius", "det", "2norm", "spectral", "combined")


def scaling_mu(Ak, Ainv, kind: str = "frobenius") -> float:
    """The scaling parameter mu of a Newton step (Section 3, the list of scalings after eq
    (3.1)): Frobenius sqrt(||A^-1||_F / ||A||_F); determinantal |det A|^(-1/n) (from the LU
    factorisation's log-determinant); 2-norm sqrt(||A^-1||_2 / ||A||_2) (singular values);
    spectral sqrt(rho(A^-1) / rho(A)) (eigenvalues).  All in float64 from the computed
    A_k and inverse."""
    n = Ak.shape[0]
    if kind == "frobenius":
        return math.sqrt(np.linalg.norm(Ainv, "fro") / np.linalg.norm(Ak, "fro"))
    if kind == "det":
        _sign, logdet = np.linalg.slogdet(Ak)
        return math.exp(-logdet / n)
    if kind == "2norm":
        return math.sqrt(np.linalg.norm(Ainv, 2) / np.linalg.norm(Ak, 2))
    if kind == "spectral":
        rho = float(np.max(np.abs(np.linalg.eigvals(Ak))))
        rho_inv = float(np.max(np.abs(np.linalg.eigvals(Ainv))))
        return math.sqrt(rho_inv / rho)
    raise ValueError(f"unknown scaling {kind}")


def a_sequence(A, fmt: str = "fp64", k_max: int = 50, delta_off: float = 1e-2,
               tau_N: float | None = None, scaling_kind: str = "frobenius") -> ASequence:
    """Scaled Newton A-iteration with the stopping rule (3.4) and the Section 4 policy."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    u = unit_roundoff(fmt)
    tau = 10.0 * math.sqrt(n * u) if tau_N is None else tau_N
    I = np.eye(n)
    seq = ASequence(fmt=fmt)
    Ak = fl_scaled(A, fmt)
    scaling = True
    countdown = None
    delta_prev = None
    for _k in range(1, k_max + 1):
        try:
            Ainv = inverse_at(Ak, fmt)
        except np.linalg.LinAlgError as exc:
            raise np.linalg.LinAlgError(f"singular A_k at k={_k}") from exc
        if not np.all(np.isfinite(Ainv)):
            raise NonFiniteError(f"non-finite inverse at k={_k}")
        # combined Frobenius + determinantal scaling (the combination Section 4 reports trying,
        # which the paper does not spell out; read here as the determinantal scaling for the
        # first step, where the eigenvalues are furthest from +-1, then the Frobenius scaling)
        kind = scaling_kind
        if scaling_kind == "combined":
            kind = "det" if _k == 1 else "frobenius"
        mu = scaling_mu(Ak, Ainv, kind) if scaling else 1.0
        if not (np.isfinite(mu) and mu > 0.0):
            raise NonFiniteError(f"scaling parameter out of range at k={_k}")
        Anew = fl_scaled(0.5 * (mu * Ak + Ainv / mu), fmt)
        delta = float(np.linalg.norm(Anew - Ak, "fro") / np.linalg.norm(Anew, "fro"))
        onenorm = float(np.linalg.norm(Anew + I, 1))
        seq.inverses.append(Ainv)
        seq.mus.append(mu)
        seq.deltas.append(delta)
        seq.onenorms.append(onenorm)
        Ak = Anew
        if countdown is not None:
            countdown -= 1
            if countdown == 0:
                break
        elif onenorm <= tau or (not scaling and delta_prev is not None
                                and delta > delta_prev / 2.0):
            countdown = 1
        if scaling and delta < delta_off:
            scaling = False
        delta_prev = delta
    else:
        if countdown is None or countdown > 0:
            seq.A_last = Ak
            raise NotStableError(f"A-iteration did not converge in k_max={k_max} steps")
    seq.A_last = Ak
    return seq


# ------------------------------------------------------------------- truncations
def rank_trunc_chol(Z, fmt: str) -> np.ndarray:
    """RankTruncChol: rank-revealing QR Z^T P = Q [T C; 0 S] with the smallest leading
    block such that ||S||_2 <= sqrt(u) ||Z||_2; returns P [T C]^T."""
    u = unit_roundoff(fmt)
    dt = _lapack_dtype(fmt)
    Zt = fl_scaled(Z, fmt, axis=0).T.astype(dt)
    _, R, perm = sla.qr(Zt, mode="economic", pivoting=True)
    R = R.astype(np.float64)
    c = R.shape[0]
    normZ = np.linalg.norm(R, 2)
    thr = math.sqrt(u) * normZ
    # ||R[r:, r:]||_2 is non-increasing in r: find the smallest r that meets the bound
    lo, hi = 0, c
    while lo < hi:
        mid = (lo + hi) // 2
        tail = R[mid:, mid:]
        if tail.size == 0 or np.linalg.norm(tail, 2) <= thr:
            hi = mid
        else:
            lo = mid + 1
    r = max(lo, 1)
    Znew = np.zeros((Z.shape[0], r))
    Znew[perm, :] = R[:r, :].T
    return fl_scaled(Znew, fmt, axis=0)


def rank_trunc_ldlt(Z, Y, fmt: str, psd: bool, tol: float | None = None):
    """RankTruncLdlt: Z = QR, R Y R^T = V Lambda V^T, keep lambda_i > u ||Lambda||_1
    (|lambda_i| for an indefinite problem, signs kept); returns (Q V, Lambda).  ``tol``
    replaces u by max(u, tol) (an inexact solve, used by adaptive refinement)."""
    u = unit_roundoff(fmt) if tol is None else max(unit_roundoff(fmt), tol)
    Q, R = thin_qr(Z, fmt)
    M = matmul(matmul(R, Y, fmt), R.T, fmt)
    lam, V = sym_eig(M, fmt)
    if not np.all(np.isfinite(lam)):
        raise NonFiniteError("non-finite eigenvalue in RankTruncLdlt")
    thr = u * float(np.max(np.abs(lam)))          # 1-norm of a diagonal matrix
    keep = lam > thr if psd else np.abs(lam) > thr
    return matmul(Q, V[:, keep], fmt), np.diag(lam[keep])


# --------------------------------------------------------------------- solvers
@dataclass
class SolverInfo:
    K: int
    mus: list
    columns: list          # column count of Z after each step (after any truncation)
    truncations: int


def sign_newton_chol(A, L, fmt: str = "fp64", rho: float = 0.1, k_max: int = 50,
                     seq: ASequence | None = None):
    """Alg 3.1.  Returns (Z, seq, info) with X ~ Z Z^T."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    if seq is None:
        seq = a_sequence(A, fmt, k_max)
    cap = math.floor(rho * n)
    Z = fl_scaled(L, fmt, axis=0)
    cols, ntr = [], 0
    for Ainv, mu in zip(seq.inverses, seq.mus):
        AZ = matmul(Ainv, Z, fmt)
        Z = fl_scaled(np.hstack([math.sqrt(mu / 2.0) * Z, AZ / math.sqrt(2.0 * mu)]), fmt,
                      axis=0)
        if Z.shape[1] > cap:
            Z = rank_trunc_chol(Z, fmt)
            ntr += 1
        cols.append(Z.shape[1])
    Z = fl_scaled(Z / math.sqrt(2.0), fmt, axis=0)
    return Z, seq, SolverInfo(seq.K, list(seq.mus), cols, ntr)


def sign_newton_ldlt(A, L, S, fmt: str = "fp64", psd: bool = True, rho: float = 0.1,
                     k_max: int = 50, seq: ASequence | None = None,
                     trunc_tol: float | None = None):
    """Alg 3.2.  ``S`` is m x m (or a 1-D diagonal).  Returns (Z, Y, seq, info) with
    X ~ Z Y Z^T.  ``trunc_tol``: RankTruncLdlt threshold max(u, trunc_tol) instead of u."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    if seq is None:
        seq = a_sequence(A, fmt, k_max)
    cap = math.floor(rho * n)
    Z = fl_scaled(L, fmt, axis=0)
    S = np.asarray(S, np.float64)
    Y = fl_scaled(np.diag(S) if S.ndim == 1 else S, fmt, axis=0)
    cols, ntr = [], 0
    for Ainv, mu in zip(seq.inverses, seq.mus):
        Z = np.hstack([Z, matmul(Ainv, Z, fmt)])
        Y = fl_scaled(0.5 * sla.block_diag(mu * Y, Y / mu), fmt, axis=0)
        if Z.shape[1] > cap:
            Z, Y = rank_trunc_ldlt(Z, Y, fmt, psd, trunc_tol)
            ntr += 1
        cols.append(Z.shape[1])
    Y = fl_scaled(Y / 2.0, fmt, axis=0)
    return Z, Y, seq, SolverInfo(seq.K, list(seq.mus), cols, ntr)


def kron_y_structure(mus, S) -> np.ndarray:
    """Y_K before the final halving and without truncation: the Kronecker product
    diag(mu_{K-1}/2, 1/(2 mu_{K-1})) (x) ... (x) diag(mu_0/2, 1/(2 mu_0)) (x) S."""
    S = np.asarray(S, np.float64)
    Y = np.diag(S) if S.ndim == 1 else S
    for mu in mus:
        Y = np.kron(np.diag([mu / 2.0, 1.0 / (2.0 * mu)]), Y)
    return Y
