"""Gradients of the quadratic loss tr(C X C^T) of the Lyapunov solution (test infrastructure).

X solves A X + X A^T + W = 0 with W = L S L^T.  For a loss l(X) with G = dl/dX symmetric,
the adjoint Y solves A^T Y + Y A + G = 0 and the first-order change of l is
<Y, dA X + X dA^T + dW>, so that dl/dA = 2 Y X, dl/dW = Y, dl/dL = 2 Y L S and, for a
diagonal S, dl/dS_i = (L^T Y L)_ii.  For l = tr(C X C^T): G = C^T C and dl/dC = 2 C X.
Every solution here is the exact one (Bartels-Stewart on the complex Schur form); nothing is
shared with the GPU library.
"""
from __future__ import annotations

import numpy as np

from . import exact


def trace_loss(A, L, S, C) -> float:
    """tr(C X C^T) with X the exact solution for W = L S L^T (S None: identity)."""
    X = exact.bartels_stewart(A, exact.form_w(L, S))
    C = np.asarray(C, np.float64)
    return float(np.trace(C @ X @ C.T))


def trace_loss_grad(A, L, S, C):
    """(dA, dL, dS, dC) of tr(C X C^T) by the adjoint equation; dS is None when S is None."""
    A = np.asarray(A, np.float64)
    L = np.asarray(L, np.float64)
    C = np.asarray(C, np.float64)
    X = exact.bartels_stewart(A, exact.form_w(L, S))
    Y = exact.bartels_stewart(A.T, C.T @ C)
    dA = 2.0 * Y @ X
    s = np.ones(L.shape[1]) if S is None else np.asarray(S, np.float64)
    dL = 2.0 * Y @ L * s[None, :]
    dS = None if S is None else np.einsum("ij,ik,kj->j", L, Y, L)
    dC = 2.0 * C @ X
    return dA, dL, dS, dC
