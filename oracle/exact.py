"""Exact solution of AX + XA^T + W = 0 by plain definitions (test infrastructure).

* ``kron_solve``     -- the n^2 x n^2 Kronecker system M vec(X) = -vec(W),
                        M = I (x) A + A (x) I (eq 2.1), solved by dense LU.  n <= ~70.
* ``bartels_stewart``-- Bartels & Stewart (1972): complex Schur form A = U T U^H (LAPACK,
                        via SciPy), C = U^H W U, then the column recurrence
                        (T + conj(t_jj) I) y_j = -c_j - sum_{k>j} conj(t_jk) y_k, j = n..1,
                        and X = U Y U^H (real part, symmetrised).
* ``schur_solve``    -- the same recurrence on a known real upper-triangular Schur form
                        A = Q T Q^T (no Schur decomposition needed).
* ``diag_closed_form`` -- diagonal A: X_ij = -W_ij / (a_i + a_j).
* ``shift_closed_form``-- A = -alpha I: X = W / (2 alpha).

W is passed either dense or as (L, S) with W = L S L^T (S = None means I; a 1-D S is a
diagonal).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def form_w(L, S=None) -> np.ndarray:
    """W = L S L^T (S None -> identity, 1-D S -> diag(S))."""
    L = np.asarray(L, np.float64)
    if S is None:
        return L @ L.T
    S = np.asarray(S, np.float64)
    if S.ndim == 1:
        return (L * S[None, :]) @ L.T
    return L @ S @ L.T


def kron_solve(A, W) -> np.ndarray:
    """Solve (I (x) A + A (x) I) vec(X) = -vec(W) with column-major vec (eq 2.1)."""
    A = np.asarray(A, np.float64)
    W = np.asarray(W, np.float64)
    n = A.shape[0]
    I = np.eye(n)
    M = np.kron(I, A) + np.kron(A, I)
    w = -W.reshape(-1, order="F")
    x = np.linalg.solve(M, w)
    return x.reshape(n, n, order="F")


def _triangular_recurrence(T, C, conj: bool):
    """Solve T Y + Y T^H + C = 0 (T upper triangular) column by column from the last:
    (T + conj(t_jj) I) y_j = -c_j - sum_{k>j} conj(t_jk) y_k."""
    n = T.shape[0]
    dtype = np.result_type(T.dtype, C.dtype)
    Y = np.zeros((n, n), dtype=dtype)
    Th = np.conj(T) if conj else T
    I = np.eye(n, dtype=dtype)
    for j in range(n - 1, -1, -1):
        rhs = -C[:, j].copy()
        if j + 1 < n:
            rhs -= Y[:, j + 1:] @ Th[j, j + 1:]
        Y[:, j] = sla.solve_triangular(T + Th[j, j] * I, rhs, lower=False)
    return Y


def _triangular_sylvester(T, C):
    """Solve T Y + Y T^H + C = 0 for upper triangular complex T with LAPACK's ztrsyl, which
    runs the same back-substitution as ``_triangular_recurrence`` in blocked compiled code
    (T Y + Y B = scale * (-C) with B = T^H, i.e. trana = 'N', tranb = 'C')."""
    Y, scale, info = sla.lapack.ztrsyl(T, T, -C, trana="N", tranb="C", isgn=1)
    if info < 0:
        raise ValueError(f"ztrsyl argument {-info} invalid")
    return Y / scale


def bartels_stewart(A, W, recurrence: bool | None = None) -> np.ndarray:
    """Bartels-Stewart on the complex Schur form of A (general real A).  The triangular
    equation is solved column by column (``_triangular_recurrence``) for n <= 512, and by
    LAPACK's ztrsyl (the same back-substitution) above that or with recurrence=False."""
    A = np.asarray(A, np.float64)
    W = np.asarray(W, np.float64)
    T, U = sla.schur(A, output="complex")
    C = U.conj().T @ W @ U
    if recurrence is None:
        recurrence = A.shape[0] <= 512
    Y = _triangular_recurrence(T, C, conj=True) if recurrence else _triangular_sylvester(T, C)
    X = (U @ Y @ U.conj().T).real
    return 0.5 * (X + X.T)


def schur_solve(Q, T, W) -> np.ndarray:
    """Solve with a known real Schur form A = Q T Q^T, T upper triangular (real spectrum)."""
    Q = np.asarray(Q, np.float64)
    T = np.asarray(T, np.float64)
    C = Q.T @ np.asarray(W, np.float64) @ Q
    Y = _triangular_recurrence(T, C, conj=False)
    X = Q @ Y @ Q.T
    return 0.5 * (X + X.T)


def diag_closed_form(a_diag, W) -> np.ndarray:
    """A = diag(a): X_ij = -W_ij / (a_i + a_j)."""
    a = np.asarray(a_diag, np.float64)
    return -np.asarray(W, np.float64) / (a[:, None] + a[None, :])


def shift_closed_form(alpha: float, W) -> np.ndarray:
    """A = -alpha I: X = W / (2 alpha)."""
    return np.asarray(W, np.float64) / (2.0 * alpha)
