"""Residuals of a factored approximate solution (test infrastructure).

R(Z)   = A Z Z^T + Z Z^T A^T + L L^T            (eq 2.2)
R(Z,Y) = A Z Y Z^T + Z Y Z^T A^T + L S L^T      (eq 2.17)
res    = ||R||_F / (||W||_F + 2 ||X_hat||_F ||A||_F)   (eq 4.1), all in float64, formed
densely.  Y (or D) may be a matrix or the diagonal as a 1-D array.  With W = 0 and X_hat = 0
the denominator vanishes together with R; that exact solution (X = 0 solves the equation with
W = 0) is given res = 0.
"""
from __future__ import annotations

import numpy as np

from .exact import form_w


def form_x(Z, Y=None) -> np.ndarray:
    """X_hat = Z Z^T or Z Y Z^T."""
    Z = np.asarray(Z, np.float64)
    if Y is None:
        return Z @ Z.T
    Y = np.asarray(Y, np.float64)
    if Y.ndim == 1:
        return (Z * Y[None, :]) @ Z.T
    return Z @ Y @ Z.T


def residual_matrix(A, L, S, Z, Y=None) -> np.ndarray:
    """R = A X + X A^T + W with X = Z Z^T or Z Y Z^T and W = L L^T or L S L^T."""
    A = np.asarray(A, np.float64)
    X = form_x(Z, Y)
    AX = A @ X
    return AX + AX.T + form_w(L, S)


def _ratio(num: float, den: float) -> float:
    if den == 0.0:
        return 0.0 if num == 0.0 else float("inf")
    return num / den


def relres(A, L, S, Z, Y=None) -> float:
    """Normwise relative residual of eq (4.1)."""
    A = np.asarray(A, np.float64)
    X = form_x(Z, Y)
    AX = A @ X
    W = form_w(L, S)
    R = AX + AX.T + W
    den = np.linalg.norm(W, "fro") + 2.0 * np.linalg.norm(X, "fro") * np.linalg.norm(A, "fro")
    return _ratio(float(np.linalg.norm(R, "fro")), float(den))


def relres_dense(A, W, X) -> float:
    """eq (4.1) for a dense X."""
    A = np.asarray(A, np.float64)
    X = np.asarray(X, np.float64)
    W = np.asarray(W, np.float64)
    AX = A @ X
    R = AX + AX.T + W
    den = np.linalg.norm(W, "fro") + 2.0 * np.linalg.norm(X, "fro") * np.linalg.norm(A, "fro")
    return _ratio(float(np.linalg.norm(R, "fro")), float(den))
