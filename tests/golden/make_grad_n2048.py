"""Write grad_n2048.json: the oracle's gradient of tr(C X C^T) on the n = 2048 gradient
workload (lyapgen.config("grad"): A, L from the random-shift family, m = 4, W = L L^T,
C 2 x n), by the adjoint equation with exact Bartels-Stewart solves
(oracle.adjoint.trace_loss_grad): the loss, the Frobenius norms of dA, dL, dC, sampled
entries of each, and four directional derivatives <dA, E_k> + <dL, F_k> along seeded
unit-Frobenius directions, each beside the central difference of the oracle's exact loss
(step 1e-6) along the same direction.  Only the oracle and the seeded generator are used.

Usage (from the repository root; about 20 minutes on the host, most of it in LAPACK's
triangular Sylvester solver, ten solves of order 2048 run five at a time):
    python tests/golden/make_grad_n2048.py
"""
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lyapgen  # noqa: E402
from oracle import adjoint  # noqa: E402


def directions(n, m, k=4, seed=2048):
    """Seeded unit-Frobenius direction pairs (E_k for A, F_k for L)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        E = rng.standard_normal((n, n))
        F = rng.standard_normal((n, m))
        s = np.sqrt(np.linalg.norm(E) ** 2 + np.linalg.norm(F) ** 2)
        out.append((E / s, F / s))
    return out


H = 1e-6


def _shifted_loss(args):
    k, sign = args
    cfg = lyapgen.config("grad")
    A, L, C = cfg["A"], cfg["L"], cfg["C"]
    E, F = directions(*L.shape)[k]
    return adjoint.trace_loss(A + sign * H * E, L + sign * H * F, None, C)


def main():
    cfg = lyapgen.config("grad")
    A, L, C = cfg["A"], cfg["L"], cfg["C"]
    n, m = L.shape
    jobs = [(k, s) for k in range(4) for s in (1.0, -1.0)]
    with ProcessPoolExecutor(max_workers=5) as ex:
        shifted = ex.map(_shifted_loss, jobs)
        loss = adjoint.trace_loss(A, L, None, C)
        dA, dL, _, dC = adjoint.trace_loss_grad(A, L, None, C)
        shifted = list(shifted)
    rng = np.random.default_rng(2049)
    ia, ja = rng.integers(0, n, 256), rng.integers(0, n, 256)
    il, jl = rng.integers(0, n, 128), rng.integers(0, m, 128)
    jc = rng.integers(0, n, 64)
    h = H
    dd, fd = [], []
    for k, (E, F) in enumerate(directions(n, m)):
        dd.append(float(np.sum(dA * E) + np.sum(dL * F)))
        fd.append((shifted[2 * k] - shifted[2 * k + 1]) / (2 * h))
        print("direction", dd[-1], fd[-1], flush=True)
    out = {
        "source": "oracle.adjoint.trace_loss_grad / trace_loss on lyapgen.config('grad') "
                  "(n = 2048, m = 4, W = L L^T); directions from directions(n, m) in this file",
        "n": n, "m": m, "loss": loss,
        "dA_fro": float(np.linalg.norm(dA)), "dL_fro": float(np.linalg.norm(dL)),
        "dC_fro": float(np.linalg.norm(dC)),
        "dA_i": ia.tolist(), "dA_j": ja.tolist(), "dA_val": dA[ia, ja].tolist(),
        "dL_i": il.tolist(), "dL_j": jl.tolist(), "dL_val": dL[il, jl].tolist(),
        "dC_j": jc.tolist(), "dC_val": dC[:, jc].tolist(),
        "fd_step": h, "directional": dd, "central_difference": fd,
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_n2048.json"),
              "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
