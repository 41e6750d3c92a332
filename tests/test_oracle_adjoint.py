"""Pins of the oracle's adjoint gradients: central finite differences of the exact loss in
random directions (independent of the adjoint formula), and a planted mistake (the adjoint
solved with A instead of A^T) that must fail them."""
import numpy as np
import pytest

import lyapgen
from oracle import adjoint, exact


def _problem(n=10, m=3, k=2, seed=3, with_s=True):
    A, L = lyapgen.random_shift(seed, n, m)
    rng = np.random.default_rng(seed + 100)
    A = A + 0.3 * np.triu(rng.standard_normal((n, n)), 1)  # clearly non-normal
    S = lyapgen.indefinite_signs(seed + 7, m) * (1.0 + rng.random(m)) if with_s else None
    C = rng.standard_normal((k, n))
    return A, L, S, C


def _fd(fun, x, d, h):
    return (fun(x + h * d) - fun(x - h * d)) / (2.0 * h)


@pytest.mark.parametrize("with_s", [False, True])
def test_gradient_matches_central_differences(with_s):
    A, L, S, C = _problem(with_s=with_s)
    dA, dL, dS, dC = adjoint.trace_loss_grad(A, L, S, C)
    rng = np.random.default_rng(11)
    h = 1e-6
    for _ in range(3):
        E = rng.standard_normal(A.shape)
        fd = _fd(lambda x: adjoint.trace_loss(x, L, S, C), A, E, h)
        assert np.sum(dA * E) == pytest.approx(fd, rel=1e-6, abs=1e-9)
        E = rng.standard_normal(L.shape)
        fd = _fd(lambda x: adjoint.trace_loss(A, x, S, C), L, E, h)
        assert np.sum(dL * E) == pytest.approx(fd, rel=1e-6, abs=1e-9)
        E = rng.standard_normal(C.shape)
        fd = _fd(lambda x: adjoint.trace_loss(A, L, S, x), C, E, h)
        assert np.sum(dC * E) == pytest.approx(fd, rel=1e-6, abs=1e-9)
        if with_s:
            E = rng.standard_normal(S.shape)
            fd = _fd(lambda x: adjoint.trace_loss(A, L, x, C), S, E, h)
            assert np.sum(dS * E) == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_planted_untransposed_adjoint_fails():
    A, L, S, C = _problem()
    X = exact.bartels_stewart(A, exact.form_w(L, S))
    Y_wrong = exact.bartels_stewart(A, C.T @ C)  # mistake: A instead of A^T
    dA_wrong = 2.0 * Y_wrong @ X
    E = np.random.default_rng(5).standard_normal(A.shape)
    fd = _fd(lambda x: adjoint.trace_loss(x, L, S, C), A, E, 1e-6)
    assert abs(np.sum(dA_wrong * E) - fd) > 1e-3 * abs(fd)


def test_loss_is_quadratic_form_of_solution():
    # tr(C X C^T) = sum over rows c of c^T X c, and X is the exact Lyapunov solution
    A, L, S, C = _problem(with_s=False)
    X = exact.kron_solve(A, exact.form_w(L, None))
    assert adjoint.trace_loss(A, L, None, C) == pytest.approx(
        sum(c @ X @ c for c in C), rel=1e-12)


def test_gradient_golden_n2048_matches_central_differences():
    # tests/golden/grad_n2048.json holds the oracle's adjoint gradient at the n = 2048
    # gradient workload and central differences (step 1e-6) of its exact loss along four
    # unit-Frobenius directions; they agree to the differences' error budget, normwise
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "grad_n2048.json")))
    scale = np.hypot(g["dA_fro"], g["dL_fro"])
    for dd, fd in zip(g["directional"], g["central_difference"]):
        assert abs(dd - fd) <= 1e-8 * scale
    assert g["n"] == 2048 and g["fd_step"] == 1e-6
