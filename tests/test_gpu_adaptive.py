"""Adaptive inexact inner tolerances (lyap_options.adaptive) on the GPU against the oracle's
same rule: each correction truncated at max(u_s, eta_r / 10), each update at
max(eta_s, omega res_i).  Both reach tau_I; the factor is not larger than with the fixed
thresholds of Alg 3.2 / Fragment 2.4.  With an fp32 inner solver the refinement counts agree
within one.  With fp16 they are parity unpinned: the oracle rounds every stored value to
fp16 (the paper's elementwise model) while the GPU keeps the inversion's working copy and
every sum in binary32, so its corrections are more accurate and it never needs more
refinements than the oracle."""
import numpy as np
import pytest
import torch

import lyapgen
from oracle import exact as E
from oracle import refine as IR
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


@pytest.mark.parametrize("us", ["fp32", "fp16"])
def test_adaptive_matches_oracle(lyap, us):
    A, L, Q, T = lyapgen.schur_family(3, 300, 4, lo=-3.0, upper_std_scale=0.003)
    X = E.schur_solve(Q, T, L @ L.T)
    prec = (us, "fp64", "fp64", "fp64")
    print(f"adaptive n=300 {us}", flush=True)
    Zf, Df, fixed = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec, adaptive=1)
    _, _, io = IR.ir_ldlt(A, L, None, prec=prec, adaptive=True)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    res = R.relres(A, L, None, Z, D)
    err = np.linalg.norm((Z * D) @ Z.T - X) / np.linalg.norm(X)
    print(f"  gpu {info['status']} res={res:.2e} err={err:.2e} rank={info['rank']} (fixed "
          f"{fixed['rank']}) refinements={info['refinements']}; oracle rank={io.rank} "
          f"refinements={io.refinements}", flush=True)
    assert info["status"] == "OK" and res <= 1e-13
    assert err <= 1e-10
    if us == "fp32":
        assert abs(info["refinements"] - io.refinements) <= 1
    else:
        assert info["refinements"] <= io.refinements
    assert info["rank"] <= 1.05 * fixed["rank"] + 2


@pytest.mark.parametrize("k", [5, 14, 24])
@pytest.mark.parametrize("opts", [{}, {"adaptive": 1}])
def test_fp16_solves_of_batch_instances_report_their_true_residual(lyap, k, opts):
    # Regression: the factor of an fp16 solve was marked orthonormal after a truncation with
    # binary32 rotations (orthonormal to ~1e-6 only); the residual factorisation then took it
    # as an exact orthonormal block and over-reported res (7e-13 against a true 1e-15), so
    # refinement stagnated.  The library's res must match the host's recomputation.
    A, L = lyapgen.batch_family()[k]
    print(f"batch instance {k} n={A.shape[0]} m={L.shape[1]} fp16 {opts}", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp16", "fp64", "fp64", "fp64"),
                            **opts)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    host = R.relres(A, L, None, Z, D)
    print(f"  {info['status']} res lib={info['res']:.2e} host={host:.2e} "
          f"hist={[f'{r:.1e}' for r in info['res_hist']]}", flush=True)
    assert info["status"] == "OK" and host <= 1e-13
    assert info["res"] == pytest.approx(host, rel=0.05, abs=2e-16)
    # the returned factor of an FP64-updated solve is orthonormal to working precision
    if info["refinements"] > 0:
        assert np.abs(Z.T @ Z - np.eye(Z.shape[1])).max() <= 1e-12
