"""Gradient parity at the n = 2048 gradient workload: the autograd gradient of tr(C X C^T)
(forward IR solve, adjoint IR solve replaying the inverses, factored products) against the
oracle's exact adjoint gradient (tests/golden/grad_n2048.json, written by
make_grad_n2048.py from oracle.adjoint only): loss, norms, sampled entries and four
directional derivatives, at 1e-9 relative, with fp32 and fp16 inner solvers.  The oracle's
directional derivatives are themselves pinned against central differences of its exact loss
(tests/test_oracle_adjoint.py)."""
import json
import os

import numpy as np
import pytest
import torch

import lyapgen

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "grad_n2048.json")


@pytest.fixture(scope="module")
def lyap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_02126_amd as m
    return m


def _directions(n, m, k=4, seed=2048):
    # the same seeded unit-Frobenius directions as tests/golden/make_grad_n2048.py
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        E = rng.standard_normal((n, n))
        F = rng.standard_normal((n, m))
        s = np.sqrt(np.linalg.norm(E) ** 2 + np.linalg.norm(F) ** 2)
        out.append((E / s, F / s))
    return out


@pytest.mark.parametrize("us", ["fp64", "fp32", "fp16"])
def test_gradient_n2048_matches_oracle(lyap, us):
    g = json.load(open(GOLD))
    cfg = lyapgen.config("grad")
    A, L, C = cfg["A"], cfg["L"], cfg["C"]
    n, m = L.shape
    print(f"gradient n=2048 {us}-inner IR vs oracle", flush=True)
    At = torch.from_numpy(A).cuda().requires_grad_(True)
    Lt = torch.from_numpy(L).cuda().requires_grad_(True)
    Ct = torch.from_numpy(C).cuda().requires_grad_(True)
    loss = lyap.lyapunov_trace_loss(At, Lt, None, Ct, (us, "fp64", "fp64", "fp64"))
    loss.backward()
    dA, dL, dC = At.grad.cpu().numpy(), Lt.grad.cpu().numpy(), Ct.grad.cpu().numpy()
    tol = 1e-9
    rel = abs(float(loss.detach()) - g["loss"]) / abs(g["loss"])
    print(f"  loss rel err {rel:.2e}", flush=True)
    assert rel <= tol
    for got, name in ((dA, "dA"), (dL, "dL"), (dC, "dC")):
        assert abs(np.linalg.norm(got) - g[f"{name}_fro"]) <= tol * g[f"{name}_fro"], name
    for got, ii, jj, want, scale in (
            (dA, g["dA_i"], g["dA_j"], g["dA_val"], g["dA_fro"]),
            (dL, g["dL_i"], g["dL_j"], g["dL_val"], g["dL_fro"])):
        d = np.asarray(got)[np.asarray(ii), np.asarray(jj)] - np.asarray(want)
        assert np.abs(d).max() <= tol * scale
    assert np.abs(dC[:, g["dC_j"]] - np.asarray(g["dC_val"])).max() <= tol * g["dC_fro"]
    scale = np.hypot(g["dA_fro"], g["dL_fro"])
    for (E, F), want in zip(_directions(n, m), g["directional"]):
        got = float(np.sum(dA * E) + np.sum(dL * F))
        print(f"  directional {got:.12e} oracle {want:.12e}", flush=True)
        assert abs(got - want) <= tol * scale
