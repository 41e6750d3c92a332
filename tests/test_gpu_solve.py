"""End-to-end parity of the GPU solver (C ABI lyap_solve) with the CPU oracle.

Acceptance (on the CPU, in float64, from the returned factors):
  * relative residual of eq (4.1) <= 1e-13 for the FP64 sign-function Newton solve and for
    mixed-precision IR;
  * ||Z diag(D) Z^T - X||_F / ||X||_F <= 10 kappa_hat res (X from the Kronecker system or
    Bartels-Stewart), with the sign of D matching the definiteness of W;
  * the FP64 solve reproduces the oracle's Newton count K and scalings mu_k.
Factors themselves are not compared entrywise (Z is defined up to an orthogonal change of
basis within eigenvalue clusters and column signs)."""
import numpy as np
import pytest
import torch

import lyapgen
from oracle import exact as E
from oracle import refine as IR
from oracle import residual as R
from oracle import signnewton as SN

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lyap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_02126_amd as m
    return m


def _cuda(x):
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(lyap, A, L, S, us, **kw):
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), _cuda(S),
                            precisions=(us, "fp64", "fp64", "fp64"), **kw)
    return Z.cpu().numpy(), D.cpu().numpy(), info


def _check(A, L, S, Z, D, X, res_tol=1e-13, err_factor=None):
    res = R.relres(A, L, S, Z, D)
    Xh = (Z * D) @ Z.T
    err = np.linalg.norm(Xh - X) / np.linalg.norm(X)
    return res, err


@pytest.mark.parametrize("us", ["fp64", "fp32", "fp16", "bf16", "fp16x2"])
def test_small_all_precisions(lyap, us):
    cfg = lyapgen.config("small")
    A, L = cfg["A"], cfg["L"]
    print(f"solve small n=64 us={us}", flush=True)
    X = E.kron_solve(A, L @ L.T)
    Z, D, info = _run(lyap, A, L, None, us)
    res, err = _check(A, L, None, Z, D, X)
    print(f"  status={info['status']} res={res:.2e} gpu_res={info['res']:.2e} err={err:.2e} "
          f"rank={info['rank']} iters={info['newton_total']}({info['newton_max']}) "
          f"refinements={info['refinements']}", flush=True)
    assert info["status"] == "OK"
    assert res <= 1e-13
    assert err <= 1e-11
    assert np.all(D > 0)                       # W = L L^T: PSD solution
    assert info["res"] == pytest.approx(res, rel=0.05, abs=1e-16)
    if us == "fp64":
        assert info["refinements"] == 0


def test_fp64_newton_sequence_matches_oracle(lyap):
    cfg = lyapgen.config("small")
    A, L = cfg["A"], cfg["L"]
    seq = SN.a_sequence(A, "fp64")
    Z, D, info = _run(lyap, A, L, None, "fp64")
    assert info["inversions"] == seq.K
    assert np.allclose(info["mus"], seq.mus, rtol=1e-10, atol=0)


def test_paper_family_newton_counts(lyap):
    # Table 4.1 FP64 solver counts on the Section 4.1 family, n = 100
    want = [4, 5, 5, 6, 6, 7, 7, 7]
    qs = [0.11394335230683679, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5]
    got = []
    for q in qs:
        A, L = lyapgen.paper_family(100, q)
        print(f"paper family n=100 q={q:.2f}", flush=True)
        _, _, info = _run(lyap, A, L, None, "fp64", refine=False)
        got.append(info["inversions"])
    assert got == want


def test_indefinite_rhs(lyap):
    A, L = lyapgen.random_shift(2, 96, 4)
    s = np.array([1.0, -1.0, -1.0, 1.0])
    X = E.kron_solve(A, E.form_w(L, s)) if A.shape[0] <= 64 else E.bartels_stewart(A, E.form_w(L, s))
    for us in ("fp64", "fp16"):
        print(f"indefinite n=96 us={us}", flush=True)
        Z, D, info = _run(lyap, A, L, s, us)
        res, err = _check(A, L, s, Z, D, X)
        print(f"  status={info['status']} res={res:.2e} err={err:.2e} rank={info['rank']}", flush=True)
        assert info["status"] == "OK" and res <= 1e-13 and err <= 1e-11
        assert np.any(D < 0) and np.any(D > 0)


@pytest.mark.parametrize("us", ["fp64", "fp32"])
def test_medium_ragged(lyap, us):
    # n = 300 (not a multiple of any tile), Schur family with a known Schur form
    A, L, Q, T = lyapgen.schur_family(7, 300, 3, lo=-2.0)
    X = E.schur_solve(Q, T, L @ L.T)
    print(f"medium n=300 us={us}", flush=True)
    Z, D, info = _run(lyap, A, L, None, us)
    res, err = _check(A, L, None, Z, D, X)
    print(f"  status={info['status']} res={res:.2e} err={err:.2e} rank={info['rank']} "
          f"K={info['inversions']} refinements={info['refinements']}", flush=True)
    assert info["status"] == "OK" and res <= 1e-13
    assert err <= 1e-9


def test_matches_oracle_ir_rank_and_iterations_fp32(lyap):
    # same algorithm on both sides: the residual histories agree to within an order of
    # magnitude and the refinement counts match
    A, L = lyapgen.random_shift(1, 64, 2)
    Zo, do, io = IR.ir_ldlt(A, L, None, prec=("fp32", "fp64", "fp64", "fp64"))
    Z, D, info = _run(lyap, A, L, None, "fp32")
    print(f"oracle refinements {io.refinements} gpu {info['refinements']}; "
          f"res oracle {io.res_hist} gpu {info['res_hist']}", flush=True)
    assert info["inversions"] == io.inversions
    assert abs(info["refinements"] - io.refinements) <= 1


def test_not_stable_and_singular(lyap):
    A = -np.eye(32)
    A[5, 5] = 0.3   # eigenvalue in the right half-plane
    L = np.ones((32, 1))
    Z, D, info = _run(lyap, A, L, None, "fp64", raise_on_error=False)
    assert info["status"] == "NOT_STABLE"
    A2 = -np.eye(32)
    A2[3, 3] = 0.0
    with pytest.raises(lyap.LyapError) as e:
        _run(lyap, A2, L, None, "fp64")
    assert e.value.status == "SINGULAR"


def test_repeat_is_deterministic(lyap):
    cfg = lyapgen.config("small")
    A, L = cfg["A"], cfg["L"]
    a = _run(lyap, A, L, None, "fp16")
    b = _run(lyap, A, L, None, "fp16")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("us", ["fp16x2"])
def test_split_solver_matches_oracle(lyap, us):
    # u_s = fp16x2 (split binary16 operands, unit roundoff 2^-22): the GPU and the oracle take
    # the same number of Newton steps and refinements (within one) on a graded problem
    A, L, Q, T = lyapgen.schur_family(7, 160, 3, lo=-2.0)
    X = E.schur_solve(Q, T, L @ L.T)
    Zo, do, io = IR.ir_ldlt(A, L, None, prec=(us, "fp64", "fp64", "fp64"))
    print(f"split solver n=160 (oracle: K={io.inversions} refinements={io.refinements})", flush=True)
    Z, D, info = _run(lyap, A, L, None, us)
    res, err = _check(A, L, None, Z, D, X)
    print(f"  gpu: status={info['status']} res={res:.2e} err={err:.2e} K={info['inversions']} "
          f"refinements={info['refinements']} rank={info['rank']} (oracle rank {io.rank})",
          flush=True)
    assert info["status"] == "OK" and res <= 1e-13 and err <= 1e-9
    assert abs(info["inversions"] - io.inversions) <= 1
    assert abs(info["refinements"] - io.refinements) <= 1
