"""lyap_solve_static, the allocation-free variant of lyap_solve (fixed device scratch),
through the C ABI: the same factors as lyap_solve on two calls in a row, the second smaller,
and problems beyond the scratch rejected before any device work."""
import ctypes

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


@pytest.mark.parametrize("us", ["fp64", "fp16"])
def test_static_matches_solve_on_two_calls(lyap, us):
    prec = (us, "fp64", "fp64", "fp64")
    for n, m in ((200, 6), (64, 2)):  # the second call is smaller
        A, L = lyapgen.random_shift(30 + n, n, m)
        print(f"static solve n={n} m={m} us={us}", flush=True)
        Zs, Ds, info_s = lyap.solve_static(_cuda(A), _cuda(L), None, precisions=prec)
        Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec)
        assert info_s["status"] == info["status"] == "OK"
        assert info_s["rank"] == info["rank"]
        # the same kernels on the same inputs: identical factors
        assert torch.equal(Zs, Z) and torch.equal(Ds, D)
        Zn, Dn = Zs.cpu().numpy(), Ds.cpu().numpy()
        assert R.relres(A, L, None, Zn, Dn) <= 1e-13
        X = E.bartels_stewart(A, L @ L.T)
        assert np.linalg.norm((Zn * Dn) @ Zn.T - X) <= 1e-11 * np.linalg.norm(X)
        assert info_s["kern_calls"] == [0, 0, 0, 0]


def test_static_rejects_problems_beyond_its_scratch(lyap):
    n = 384
    A, L = lyapgen.random_shift(5, n, 4)
    assert lyap.workspace_size(n, 4, "fp64") > 64 << 20
    with pytest.raises(lyap.LyapError) as e:
        lyap.solve_static(_cuda(A), _cuda(L), None, precisions=("fp64",) * 4)
    assert e.value.status == "TOO_LARGE"
    # fewer cached inverses make it fit
    assert lyap.workspace_size(n, 4, "fp16", k_max=12) <= 64 << 20
    Z, D, info = lyap.solve_static(_cuda(A), _cuda(L), None, precisions=("fp16", "fp64", "fp64", "fp64"),
                                   k_max=12)
    assert info["status"] == "OK" and info["res"] <= 1e-13
