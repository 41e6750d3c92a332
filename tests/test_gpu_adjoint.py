"""Adjoint solves and the differentiable loss tr(C X C^T) on the GPU, against the oracle's
exact adjoint gradients (small n) and against central finite differences of the GPU loss
(the n = 2048 gradient workload)."""
import numpy as np
import pytest
import torch

import lyapgen
from oracle import adjoint, exact

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lyap():
    import paper_2510_02126_amd as m
    return m


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_adjoint_solve_matches_oracle_and_replays_inverses(lyap):
    print("adjoint solve n=64", flush=True)
    cfg = lyapgen.config("small")
    A, L = cfg["A"], cfg["L"]
    C = np.random.default_rng(21).standard_normal((2, A.shape[0]))
    Ad = _cuda(A)
    _, _, inf_f = lyap.solve(Ad, _cuda(L), None, precisions=("fp64",) * 4)
    ZY, DY, inf_a = lyap.solve_adjoint(Ad, _cuda(C.T), None, precisions=("fp64",) * 4)
    assert inf_a["status"] == "OK" and inf_a["res"] <= 1e-13
    assert inf_f["inversions"] > 0 and inf_a["inversions"] == 0  # inverse sequence replayed
    Y = (ZY.cpu().numpy() * DY.cpu().numpy()) @ ZY.cpu().numpy().T
    Yo = exact.bartels_stewart(A.T, C.T @ C)
    assert np.linalg.norm(Y - Yo) <= 1e-11 * np.linalg.norm(Yo)
    # a different A (new tensor) computes its own sequence
    A2 = A - 0.1 * np.eye(A.shape[0])
    _, _, inf_b = lyap.solve_adjoint(_cuda(A2), _cuda(C.T), None, precisions=("fp64",) * 4)
    assert inf_b["inversions"] > 0 and inf_b["res"] <= 1e-13


_LOSS_TOL = {}


def _loss_tol(A, L, S, C, lo, res_stop=1e-13):
    """Bound on |loss - exact| / |loss| for a solve stopped at relative residual ``res_stop``
    (eq (4.1)): X_hat - X = L^{-1}(R) with ||R||_F = res (||W||_F + 2 ||A||_F ||X_hat||_F), so
    |tr(C (X_hat - X) C^T)| <= ||C^T C||_F ||L^{-1}||_2 ||R||_F.  ||L^{-1}||_2 by power
    iteration on L^{-T} L^{-1} (exact Bartels-Stewart solves), with a factor 2 of margin."""
    key = (A.shape, S is not None)
    if key not in _LOSS_TOL:
        W = exact.form_w(L, S)
        X = exact.bartels_stewart(A, W)
        V = np.random.default_rng(5).standard_normal(A.shape)
        V /= np.linalg.norm(V)
        s = 1.0
        for _ in range(12):
            Z = exact.bartels_stewart(A.T, exact.bartels_stewart(A, V))
            s = np.linalg.norm(Z)
            V = Z / s
        rnorm = res_stop * (np.linalg.norm(W) + 2.0 * np.linalg.norm(A) * np.linalg.norm(X))
        _LOSS_TOL[key] = 2.0 * np.linalg.norm(C.T @ C) * np.sqrt(s) * rnorm / abs(lo)
    return _LOSS_TOL[key]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("with_s", [False, True])
def test_trace_loss_gradients_match_oracle(lyap, prec, with_s):
    print(f"trace loss grad n=96 {prec} S={with_s}", flush=True)
    n, m = 96, 3
    A, L = lyapgen.random_shift(31, n, m)
    S = lyapgen.indefinite_signs(32, m) * 1.5 if with_s else None
    C = np.random.default_rng(33).standard_normal((2, n))
    At = _cuda(A).requires_grad_(True)
    Lt = _cuda(L).requires_grad_(True)
    St = _cuda(S).requires_grad_(True) if with_s else None
    Ct = _cuda(C).requires_grad_(True)
    loss = lyap.lyapunov_trace_loss(At, Lt, St, Ct, (prec, "fp64", "fp64", "fp64"))
    loss.backward()
    lo = adjoint.trace_loss(A, L, S, C)
    dA, dL, dS, dC = adjoint.trace_loss_grad(A, L, S, C)
    tol = _loss_tol(A, L, S, C, lo)
    print(f"  loss rel err {abs(float(loss.detach()) - lo) / abs(lo):.2e} (bound {tol:.2e})",
          flush=True)
    assert float(loss.detach()) == pytest.approx(lo, rel=tol)
    for got, want in ((At.grad, dA), (Lt.grad, dL), (Ct.grad, dC)) + (
            ((St.grad, dS),) if with_s else ()):
        g = got.cpu().numpy()
        assert np.linalg.norm(g - want) <= 1e-9 * np.linalg.norm(want)


@pytest.mark.parametrize("us", ["fp32", "fp16"])
def test_trace_loss_gradient_n2048_central_differences(lyap, us):
    print(f"trace loss grad n=2048 {us}-inner IR vs central differences", flush=True)
    cfg = lyapgen.config("grad")
    A, L, C = cfg["A"], cfg["L"], cfg["C"]
    prec = (us, "fp64", "fp64", "fp64")
    At = _cuda(A).requires_grad_(True)
    Lt = _cuda(L).requires_grad_(True)
    loss = lyap.lyapunov_trace_loss(At, Lt, None, _cuda(C), prec)
    loss.backward()
    gA, gL = At.grad.cpu().numpy(), Lt.grad.cpu().numpy()
    rng = np.random.default_rng(51)

    def f(a, l):  # central differences of the FP64 solve (step 1e-6)
        z, d, info = lyap.solve(_cuda(a), _cuda(l), None, precisions=("fp64",) * 4)
        assert info["res"] <= 1e-13
        return lyap.trace_loss(_cuda(C), z, d)

    h = 1e-6
    for _ in range(2):
        E = rng.standard_normal(A.shape) / np.sqrt(A.shape[0])
        fd = (f(A + h * E, L) - f(A - h * E, L)) / (2 * h)
        assert np.sum(gA * E) == pytest.approx(fd, rel=1e-5)
        E = rng.standard_normal(L.shape)
        fd = (f(A, L + h * E) - f(A, L - h * E)) / (2 * h)
        assert np.sum(gL * E) == pytest.approx(fd, rel=1e-5)
    assert np.isfinite(gA).all() and np.abs(gA).max() > 0
