"""Seeded synthetic inputs for the low-rank Lyapunov equation AX + XA^T + W = 0.

This module builds test matrices only; it holds none of the solver's arithmetic and is
shared by the CPU oracle, the tests and the benchmark.  Every generator is driven by
``numpy.random.default_rng(seed)`` (PCG64) and returns float64 arrays.

Workloads (all synthetic; the paper's own experiments use MATLAB ``randn`` with an
unstated seed and the SLICOT collection, neither of which is reproduced here):

* ``random_shift``   -- A = G - alpha*I, G_ij ~ N(0, 1/n), alpha chosen so that the
  spectral abscissa of A is -0.5; L ~ N(0, 1).  A dense non-normal Hurwitz matrix.
* ``schur_family``   -- A = Q T Q^T with Q Haar orthogonal and T upper triangular,
  diag(T) = -logspace(lo, 0, n), strict upper entries N(0, (s/sqrt n)^2) with s = 0.1
  (s = 0.003 for the n = 4096 workload, see _cfg_large).  The Schur form is returned so
  the oracle can solve on it directly.
* ``paper_family``   -- the synthetic family of the paper's Section 4.1: symmetric A with a
  log-spaced spectrum from -1 to -10^q in the eigenbasis of the symmetric sine matrix,
  L ~ N(0, 1) with m = 3 columns.
* ``batch_family``   -- many independent random_shift instances of uneven n and m.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "haar_orthogonal", "random_shift", "schur_family", "paper_family", "sine_orthogonal",
    "indefinite_signs", "batch_family", "config", "CONFIGS",
]


def haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the signs of
    diag(R) folded into Q (Mezzadri, 2007)."""
    g = rng.standard_normal((n, n))
    q, r = np.linalg.qr(g)
    s = np.sign(np.diag(r))
    s[s == 0] = 1.0
    return q * s[None, :]


def random_shift(seed: int, n: int, m: int, abscissa: float = -0.5):
    """A = G - alpha I with G_ij ~ N(0, 1/n) and max Re(lambda(A)) = ``abscissa``;
    L is n x m with N(0, 1) entries.  Returns (A, L)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n)) / np.sqrt(n)
    alpha = float(np.max(np.linalg.eigvals(g).real)) - abscissa
    a = g - alpha * np.eye(n)
    l = rng.standard_normal((n, m))
    return a, l


def schur_family(seed: int, n: int, m: int, lo: float, upper_std_scale: float = 0.1):
    """A = Q T Q^T, Q Haar, T upper triangular with diag -logspace(lo, 0, n) and strict
    upper part N(0, (upper_std_scale/sqrt(n))^2).  Returns (A, L, Q, T)."""
    rng = np.random.default_rng(seed)
    q = haar_orthogonal(rng, n)
    t = np.triu(rng.standard_normal((n, n)) * (upper_std_scale / np.sqrt(n)), 1)
    t[np.diag_indices(n)] = -np.logspace(lo, 0.0, n)
    a = q @ t @ q.T
    l = rng.standard_normal((n, m))
    return a, l, q, t


def indefinite_signs(seed: int, m: int) -> np.ndarray:
    """Random +-1 pattern of length m; if all signs agree the last one is flipped so the
    pattern is indefinite (for m >= 2)."""
    rng = np.random.default_rng(seed)
    s = np.where(rng.random(m) < 0.5, -1.0, 1.0)
    if m >= 2 and np.all(s == s[0]):
        s[-1] = -s[-1]
    return s


def sine_orthogonal(n: int) -> np.ndarray:
    """Symmetric orthogonal matrix V_ij = sqrt(2/(n+1)) sin(i j pi/(n+1)), i,j = 1..n
    (the eigenvector matrix of the second-difference matrix)."""
    i = np.arange(1, n + 1, dtype=np.float64)
    return np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(i, i) * np.pi / (n + 1))


def paper_family(n: int, q: float, m: int = 3, seed: int = 0):
    """Section 4.1 family: a symmetric negative definite A with condition number 10^q, its
    eigenvalues -1 .. -10^q spaced evenly in log scale and its eigenvectors the columns of
    the symmetric orthogonal sine matrix, so kappa_F of the Lyapunov operator is about 10^q;
    L has m independent N(0, 1) columns.  Returns (A, L)."""
    lam = -(10.0 ** np.linspace(0.0, q, n))       # spectrum of A
    basis = sine_orthogonal(n)                     # orthonormal eigenvectors (columns)
    a = (basis * lam[None, :]) @ basis.T           # sum_k lam_k v_k v_k^T
    a = 0.5 * (a + a.T)                            # exactly symmetric in floating point
    l = np.random.default_rng(seed).standard_normal((n, m))
    return a, l


def batch_family(seed: int = 4, count: int = 256, n_range=(64, 512), m_range=(1, 8),
                 instance_seed0: int = 40000):
    """``count`` random_shift instances with n ~ U{n_range}, m ~ U{m_range} drawn with
    ``seed``; instance i uses seed instance_seed0 + i.  Returns a list of (A, L)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    ms = rng.integers(m_range[0], m_range[1] + 1, size=count)
    return [random_shift(instance_seed0 + i, int(ns[i]), int(ms[i])) for i in range(count)]


# Named workloads.  Each entry: (builder, description).  The builders return a dict with
# keys A, L, S (None for W = L L^T, else a diagonal given as a 1-D array), plus extras.
def _cfg_small(seed=1, n=64, m=2):
    a, l = random_shift(seed, n, m)
    return {"A": a, "L": l, "S": None}


def _cfg_medium(seed=2, n=1024, m=4):
    a, l, q, t = schur_family(seed, n, m, lo=-2.0)
    return {"A": a, "L": l, "S": None, "Q": q, "T": t}


def _cfg_large(seed=3, n=4096, m=8, upper_std_scale=0.003):
    # With strict-upper std 0.1/sqrt(n) (the medium workload's scale) the triangular factor
    # at n = 4096 with diagonal down to 1e-3 has ||T^-1||_F ~ 1e82: the equation is not
    # numerically stable and no sign iteration converges.  0.003/sqrt(n) keeps ||T^-1||_F
    # within 1.2x of the normal matrix's, i.e. kappa ~ 1.2e3 as the workload intends.
    a, l, q, t = schur_family(seed, n, m, lo=-3.0, upper_std_scale=upper_std_scale)
    s = indefinite_signs(seed + 1000, m)
    return {"A": a, "L": l, "S": s, "Q": q, "T": t}


def _cfg_grad(seed=5, n=2048, m=4):
    a, l = random_shift(seed, n, m)
    c = np.random.default_rng(50).standard_normal((2, n))
    return {"A": a, "L": l, "S": None, "C": c}


CONFIGS = {
    "small": _cfg_small,      # n=64, m=2, W = L L^T
    "medium": _cfg_medium,    # n=1024, m=4, W = L L^T, Schur family kappa ~ 1e2
    "large": _cfg_large,      # n=4096, m=8, W = L S L^T indefinite, kappa ~ 1e3
    "grad": _cfg_grad,        # n=2048, m=4 with a 2 x n output matrix C
}


def config(name: str, **kw):
    """Build a named workload (see CONFIGS)."""
    return CONFIGS[name](**kw)
