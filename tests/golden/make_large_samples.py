"""Write large_x_samples.json: sampled entries of the exact solution of the n = 4096 workload
(lyapgen.config("large"), A = Q T Q^T with T upper triangular, W = L S L^T), computed by the
oracle's Schur-form solver (Bartels-Stewart recurrence on the known Schur form).  Only the
oracle and the seeded generator are used.

Usage (from the repository root; a few minutes on the host):  python tests/golden/make_large_samples.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lyapgen  # noqa: E402
from oracle import exact  # noqa: E402


def main():
    cfg = lyapgen.config("large")
    A, L, S, Q, T = cfg["A"], cfg["L"], cfg["S"], cfg["Q"], cfg["T"]
    W = exact.form_w(L, S)
    X = exact.schur_solve(Q, T, W)
    n = X.shape[0]
    rng = np.random.default_rng(4096)
    rows = rng.integers(0, n, size=192)
    cols = rng.integers(0, n, size=192)
    diag = rng.integers(0, n, size=32)
    big = np.argsort(-np.abs(X), axis=None)[:32]
    ii = np.concatenate([rows, diag, big // n]).astype(int)
    jj = np.concatenate([cols, diag, big % n]).astype(int)
    out = {
        "source": "oracle.exact.schur_solve on lyapgen.config('large') (n = 4096, m = 8, "
                  "W = L S L^T); entries of the exact X",
        "n": n,
        "fro": float(np.linalg.norm(X)),
        "trace": float(np.trace(X)),
        "i": ii.tolist(),
        "j": jj.tolist(),
        "x": [float(X[i, j]) for i, j in zip(ii, jj)],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large_x_samples.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    print("wrote", path, "fro", out["fro"])


if __name__ == "__main__":
    main()
