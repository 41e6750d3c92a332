"""Degenerate and extreme inputs through the C ABI: the order-1 and order-2 equations, n not
a multiple of any tile, a zero right-hand side (X = 0 exactly), zero entries in S, sizes
outside the library's range (m > n, n > 4096), and both inner solvers where they apply."""
import numpy as np
import pytest
import torch

import lyapgen
from oracle import exact as E
from oracle import residual as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lyap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_02126_amd as m
    return m


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("solver", [0, 1])
@pytest.mark.parametrize("us", ["fp64", "fp32", "fp16", "bf16"])
def test_order_one_and_two(lyap, us, solver):
    print(f"n=1,2 us={us} solver={solver}", flush=True)
    # n = 1 (m <= n): -3 x - 3 x + 4 s = 0 with s = -1 gives x = -2/3
    Z, D, info = lyap.solve(_cuda(np.array([[-3.0]])), _cuda(np.array([[2.0]])),
                            _cuda(np.array([-1.0])), precisions=(us, "fp64", "fp64", "fp64"),
                            solver=solver)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    assert info["status"] == "OK"
    assert float(((Z * D) @ Z.T)[0, 0]) == pytest.approx(-2.0 / 3.0, rel=1e-13)
    A = np.array([[-1.0, 0.3], [0.0, -2.0]])
    L = np.array([[1.0], [0.5]])
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=(us, "fp64", "fp64", "fp64"),
                            solver=solver)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    assert info["status"] == "OK"
    np.testing.assert_allclose((Z * D) @ Z.T, E.kron_solve(A, L @ L.T), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("solver", [0, 1])
def test_zero_right_hand_side(lyap, solver):
    A, _ = lyapgen.random_shift(1, 37, 2)
    print(f"W = 0 n=37 solver={solver}", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(np.zeros((37, 2))), None,
                            precisions=("fp16", "fp64", "fp64", "fp64"), solver=solver)
    assert info["status"] == "OK" and info["rank"] == 0 and info["res"] == 0.0


def test_zero_entries_in_s(lyap):
    A, L = lyapgen.random_shift(5, 70, 4)
    s = np.array([1.0, 0.0, -1.0, 0.0])
    X = E.kron_solve(A, (L * s) @ L.T)
    print("S with zero entries n=70", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), _cuda(s), precisions=("fp32", "fp64", "fp64", "fp64"))
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert np.linalg.norm((Z * D) @ Z.T - X) <= 1e-11 * np.linalg.norm(X)


def test_sizes_outside_the_range_are_rejected(lyap):
    A, L = lyapgen.random_shift(1, 8, 2)
    Lw = np.random.default_rng(0).standard_normal((8, 12))  # m > n
    with pytest.raises(lyap.LyapError) as e:
        lyap.solve(_cuda(A), _cuda(Lw), None, precisions=("fp64",) * 4)
    assert e.value.status == "BADARG"
    with pytest.raises(lyap.LyapError) as e:
        lyap.workspace_size(4097, 2, "fp64")
    assert e.value.status == "BADARG"
