"""Parity on the remaining named workloads, at their full sizes.

* n = 1024, m = 4, W = L L^T, A = Q T Q^T with diag(T) = -logspace(-2, 0)
  (lyapgen.config("medium")): the FP64 sign-function Newton solve, fp32-inner IR in the
  LDL^T form and in the Cholesky form (Alg 2.1).  Checked: the relative residual of eq
  (4.1), recomputed on the host by the oracle, <= 1e-13; X against the oracle's exact
  Schur-form solution.  Tolerance 1e-9 in norm: X_hat - X = L^{-1}(R), ||L^{-1}||_2 about
  1 / (2 * 0.01) = 50 for this spectrum, ||A||_F about 11, so a residual of 1e-13 allows a
  relative forward error of about 50 * 1e-13 * (2 * 11 + ||W||_F / ||X||_F), a few 1e-10.
* 256 independent equations, n uniform in [64, 512], m uniform in [1, 8]
  (lyapgen.batch_family), fp16-inner IR through the batched entry point: every instance
  reaches res <= 1e-13; eight sampled instances have their residual recomputed on the host,
  and four are compared with the exact solution (Bartels-Stewart) to 1e-10."""
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


@pytest.fixture(scope="module")
def medium():
    cfg = lyapgen.config("medium")
    X = E.schur_solve(cfg["Q"], cfg["T"], cfg["L"] @ cfg["L"].T)
    return cfg, X


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("prec,form", [(("fp64",) * 4, 0), (("fp32", "fp64", "fp64", "fp64"), 0),
                                       (("fp32", "fp64", "fp64", "fp64"), 1)],
                         ids=["fp64_sign_newton", "ir_fp32_ldlt", "ir_fp32_chol"])
def test_medium_workload(lyap, medium, prec, form):
    cfg, X = medium
    A, L = cfg["A"], cfg["L"]
    print(f"medium workload n=1024 m=4 precisions={prec} form={form}", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec, form=form)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    res = R.relres(A, L, None, Z, D)
    err = np.linalg.norm((Z * D) @ Z.T - X) / np.linalg.norm(X)
    print(f"  status={info['status']} res host={res:.2e} lib={info['res']:.2e} "
          f"rank={info['rank']} refinements={info['refinements']} err={err:.2e}", flush=True)
    assert info["status"] == "OK"
    assert res <= 1e-13
    assert info["res"] == pytest.approx(res, rel=0.05, abs=1e-16)
    assert err <= 1e-9
    if form == 1:
        assert np.all(D == 1.0)
    else:
        assert np.all(D > 0)  # W = L L^T: X is positive semidefinite


def test_batched_256_fp16(lyap):
    print("batched 256 instances n in [64, 512] m in [1, 8] fp16 inner", flush=True)
    batch = lyapgen.batch_family()
    As = [_cuda(a) for a, _ in batch]
    Ls = [_cuda(l) for _, l in batch]
    out = lyap.solve_batched(As, Ls, None, precisions=("fp16", "fp64", "fp64", "fp64"))
    res = [o[2]["res"] for o in out]
    print(f"  max res {max(res):.2e}", flush=True)
    assert all(o[2]["status"] == "OK" for o in out)
    assert max(res) <= 1e-13
    rng = np.random.default_rng(256)
    for k, i in enumerate(rng.choice(len(batch), size=8, replace=False)):
        a, l = batch[i]
        Z, D = out[i][0].cpu().numpy(), out[i][1].cpu().numpy()
        r = R.relres(a, l, None, Z, D)
        assert r <= 1e-13 and out[i][2]["res"] == pytest.approx(r, rel=0.05, abs=1e-16), i
        if k < 4:
            X = E.bartels_stewart(a, l @ l.T)
            assert np.linalg.norm((Z * D) @ Z.T - X) <= 1e-10 * np.linalg.norm(X), i
