"""Write trajectory_n1024.json: the oracle's IR trajectory on the n = 1024 instance of the
large-workload construction (A = Q T Q^T, diag T = -logspace(-3, 0), strict upper part of
std 0.003/sqrt(n), W = L S L^T with S = diag(+-1), m = 8; seed 3) with an fp32 inner solver
(Alg 2.2, Section 4.1 parameters, fixed and adaptive tolerances): residual history, rank,
refinement and Newton counts, and the solution's Frobenius norm and trace from the exact
Schur-form solve.  Only the oracle and the seeded generator are used.

Usage (from the repository root; about a minute on the host):
    python tests/golden/make_trajectory_n1024.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lyapgen  # noqa: E402
from oracle import exact, refine  # noqa: E402


def main():
    n, m = 1024, 8
    A, L, Q, T = lyapgen.schur_family(3, n, m, lo=-3.0, upper_std_scale=0.003)
    S = lyapgen.indefinite_signs(1003, m)
    X = exact.schur_solve(Q, T, exact.form_w(L, S))
    out = {"source": "oracle.refine.ir_ldlt on lyapgen.schur_family(3, 1024, 8, lo=-3.0, "
                     "upper_std_scale=0.003), S = lyapgen.indefinite_signs(1003, 8); "
                     "X from oracle.exact.schur_solve",
           "n": n, "m": m, "x_fro": float(np.linalg.norm(X)), "x_trace": float(np.trace(X))}
    for key, kw in (("fp32", {}), ("fp32_adaptive", {"adaptive": True}),
                    ("fp64", {"refine": False})):
        us = "fp64" if key == "fp64" else "fp32"
        Z, d, info = refine.ir_ldlt(A, L, S, prec=(us, "fp64", "fp64", "fp64"), **kw)
        Xh = (Z * d) @ Z.T
        out[key] = {"status": info.status, "res_hist": info.res_hist, "rank": info.rank,
                    "refinements": info.refinements, "newton_total": info.newton_total,
                    "inversions": info.inversions, "mus": info.mus,
                    "x_err": float(np.linalg.norm(Xh - X) / np.linalg.norm(X))}
        print(key, out[key]["status"], out[key]["rank"], out[key]["refinements"],
              ["%.2e" % r for r in info.res_hist], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "trajectory_n1024.json"),
              "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
