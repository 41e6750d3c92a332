"""The low-rank ADI inner solver (opt.solver = 1) through the C ABI against the oracle's
LR-ADI: the shifts (same power-iteration interval and Wachspress formula, computed
independently), the step count and the solution of a plain FP64 ADI solve; refinement with
ADI at reduced solver precisions; the adjoint replay of the shifted inverses; the butterfly
inversion of the shifted matrices; an indefinite S."""
import numpy as np
import pytest
import torch

import lyapgen
from oracle import adi as AD
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
    return None if x is None else torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = {
    "shift64": lambda: lyapgen.random_shift(1, 64, 2),
    "schur300": lambda: lyapgen.schur_family(7, 300, 3, lo=-2.0)[:2],
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_fp64_adi_solve_matches_oracle(lyap, case):
    A, L = CASES[case]()
    n, m = L.shape
    seq = AD.adi_sequence(A, "fp64")
    Zo, do, ai = AD.lr_adi_ldlt(A, L, np.ones(m), "fp64", seq, psd=True)
    print(f"ADI fp64 {case}: oracle J={seq.J} steps={ai.steps} a={seq.a:.6g} b={seq.b:.6g}",
          flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp64",) * 4, solver=1,
                            refine=0)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    J = len(info["mus"])
    print(f"  gpu J={J} steps={info['newton_total']} res={info['res']:.2e} "
          f"rank={info['rank']} (oracle {Zo.shape[1]})", flush=True)
    assert J == seq.J
    np.testing.assert_allclose(info["mus"][:J], seq.shifts, rtol=1e-8)
    assert abs(info["newton_total"] - ai.steps) <= 1
    assert info["inversions"] == J + 1
    assert info["res"] <= 1e-13
    Xo = (Zo * do) @ Zo.T
    assert _rel((Z * D) @ Z.T, Xo) <= 1e-11
    if n <= 64:
        assert _rel((Z * D) @ Z.T, E.kron_solve(A, L @ L.T)) <= 1e-11


@pytest.mark.parametrize("us", ["fp32", "fp16"])
def test_refinement_with_adi_matches_oracle(lyap, us):
    n = 300 if us == "fp32" else 160
    A, L, Q, T = lyapgen.schur_family(7, n, 3, lo=-2.0)
    X = E.schur_solve(Q, T, L @ L.T)
    prec = (us, "fp64", "fp64", "fp64")
    _, _, io = IR.ir_ldlt(A, L, None, prec=prec, solver="adi")
    print(f"IR+ADI {us} n={n}: oracle {io.status} ref={io.refinements} "
          f"iters={io.newton_total}({io.newton_max}) rank={io.rank} J={len(io.mus)}", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec, solver=1)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    print(f"  gpu {info['status']} res={info['res']:.2e} ref={info['refinements']} "
          f"iters={info['newton_total']}({info['newton_max']}) rank={info['rank']} "
          f"J={len(info['mus'])}", flush=True)
    assert io.status == "OK" and info["status"] == "OK"
    assert info["res"] <= 1e-13
    assert R.relres(A, L, None, Z, D) <= 1e-13
    assert _rel((Z * D) @ Z.T, X) <= 1e-9
    # same interval and shift formula; the interval inverse is binary32 on both sides, and
    # for this non-normal A (||A^-1||_2 far above rho(A^-1)) two correct binary32 inverses
    # differ by about kappa(A) u_32 ~ 1e-2 relative, which the power iteration passes on
    assert len(info["mus"]) == len(io.mus)
    np.testing.assert_allclose(info["mus"], io.mus, rtol=2e-2)
    if us == "fp32":
        assert abs(info["refinements"] - io.refinements) <= 1
    else:
        # the oracle rounds every stored fp16 value (chop model); the kernels keep the
        # products' binary32 sums, so they need at most as many corrections
        assert info["refinements"] <= io.refinements + 1


def test_adi_adjoint_replays_the_shifted_inverses(lyap):
    A, L = CASES["shift64"]()
    C = np.random.default_rng(4).standard_normal((2, A.shape[0]))
    Ad = _cuda(A)
    prec = ("fp32", "fp64", "fp64", "fp64")
    print("ADI adjoint replay n=64 fp32", flush=True)
    _, _, i1 = lyap.solve(Ad, _cuda(L), None, precisions=prec, solver=1)
    Y, DY, i2 = lyap.solve_adjoint(Ad, _cuda(C.T), None, precisions=prec, solver=1)
    Y, DY = Y.cpu().numpy(), DY.cpu().numpy()
    assert i1["status"] == i2["status"] == "OK"
    assert i2["cache_reused"] and i2["inversions"] == 0
    Yx = E.kron_solve(A.T, C.T @ C)
    assert _rel((Y * DY) @ Y.T, Yx) <= 1e-11


def test_adi_with_butterfly_inversions(lyap):
    A, L, Q, T = lyapgen.schur_family(7, 300, 3, lo=-2.0)
    X = E.schur_solve(Q, T, L @ L.T)
    print("ADI + butterfly n=300 fp32", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp32", "fp64", "fp64", "fp64"),
                            solver=1, pivoting=1)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    print(f"  {info['status']} res={info['res']:.2e} rbt={info['rbt_steps']} "
          f"fallbacks={info['rbt_fallbacks']} J={len(info['mus'])}", flush=True)
    assert info["status"] == "OK" and info["res"] <= 1e-13
    # the J shifted inverses and the spectral-interval inverse
    assert info["rbt_steps"] == len(info["mus"]) + 1 and info["rbt_fallbacks"] == 0
    assert _rel((Z * D) @ Z.T, X) <= 1e-9


@pytest.mark.parametrize("us", ["fp64", "fp32"])
def test_adi_indefinite_s(lyap, us):
    A, L = lyapgen.random_shift(4, 48, 3)
    s = np.array([1.0, -1.0, 2.0])
    W = (L * s) @ L.T
    X = E.kron_solve(A, W)
    print(f"ADI indefinite S n=48 {us}", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), _cuda(s), precisions=(us, "fp64", "fp64", "fp64"),
                            solver=1)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert _rel((Z * D) @ Z.T, X) <= 1e-10
    assert np.any(D < 0)


def test_adi_metric_workload_n1024(lyap):
    cfg = lyapgen.config("medium")
    A, L = cfg["A"], cfg["L"]
    print("ADI fp32 inner n=1024", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp32", "fp64", "fp64", "fp64"),
                            solver=1)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    print(f"  {info['status']} res={info['res']:.2e} ref={info['refinements']} "
          f"iters={info['newton_total']}({info['newton_max']}) rank={info['rank']} "
          f"J={len(info['mus'])} inv={info['inversions']}", flush=True)
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert R.relres(A, L, None, Z, D) <= 1e-13


def test_adi_cholesky_form(lyap):
    # Alg 2.1 with the ADI solver: the two correction equations (L+ and L-) each run ADI
    A, L = CASES["shift64"]()
    X = E.kron_solve(A, L @ L.T)
    print("ADI Cholesky form n=64 fp32", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp32", "fp64", "fp64", "fp64"),
                            solver=1, form=1)
    Z = Z.cpu().numpy()
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert _rel(Z @ Z.T, X) <= 1e-11


def test_adi_shift_count_override_and_step_cap(lyap):
    A, L = CASES["schur300"]()
    prec = ("fp32", "fp64", "fp64", "fp64")
    print("ADI J=4 and adi_max=3 n=300 fp32", flush=True)
    _, _, base = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec, solver=1)
    # four shifts (oracle shifts for J = 4 on the same interval; binary32 interval inverse)
    seq = AD.adi_sequence(A, "fp32", shifts=4)
    Z, D, i4 = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec, solver=1, adi_shifts=4)
    assert len(i4["mus"]) == 4 and i4["inversions"] == 5
    np.testing.assert_allclose(i4["mus"], seq.shifts, rtol=2e-2)
    assert i4["status"] == "OK" and i4["res"] <= 1e-13
    # three ADI steps per solve use only the three largest of the 13 shifts, so the
    # corrections barely touch the small eigenvalues' components: the refinement stops by
    # eq (4.2) with a valid factor
    Z, D, i3 = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec, solver=1, adi_max=3,
                          raise_on_error=False)
    print(f"  base ref={base['refinements']} J=4 ref={i4['refinements']} "
          f"adi_max=3 {i3['status']} ref={i3['refinements']} hist={i3['res_hist']}", flush=True)
    assert i3["newton_max"] <= 3
    assert i3["status"] in ("STAGNATED", "NOT_CONVERGED") and i3["res"] > 1e-13
    assert torch.isfinite(Z).all() and torch.isfinite(D).all()
    # one cycle of shifts and two more steps per solve: inexact corrections that still
    # contract, so the refinement converges (with more steps than the full inner solve)
    J = len(base["mus"])
    _, _, ic = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec, solver=1, adi_max=J + 2)
    print(f"  adi_max={J + 2}: {ic['status']} ref={ic['refinements']} res={ic['res']:.1e}",
          flush=True)
    assert ic["status"] == "OK" and ic["res"] <= 1e-13
    assert ic["newton_max"] <= J + 2 and ic["refinements"] >= base["refinements"]


def test_adi_escalation_rescues_bf16(lyap):
    A, L = lyapgen.paper_family(60, 6.0, seed=3)
    print("ADI escalate bf16 paper family n=60 q=6", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("bf16", "fp64", "fp64", "fp64"),
                            solver=1, escalate=1)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    print(f"  {info['status']} u_s_final={info['u_s_final']} escalations={info['escalations']} "
          f"res={info['res']:.1e}", flush=True)
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert R.relres(A, L, None, Z, D) <= 1e-13


def test_adi_through_the_other_entry_points(lyap):
    # batched, allocation-free, warm-started refinement and a fresh adjoint solve, each with
    # the ADI inner solver, against exact solutions
    prec = ("fp32", "fp64", "fp64", "fp64")
    batch = lyapgen.batch_family(count=6, seed=77)
    print("ADI batched 6 instances", flush=True)
    out = lyap.solve_batched([_cuda(a) for a, _ in batch], [_cuda(l) for _, l in batch], None,
                             precisions=prec, solver=1)
    for (a, l), (Z, D, info) in zip(batch, out):
        assert info["status"] == "OK" and info["res"] <= 1e-13
        assert R.relres(a, l, None, Z.cpu().numpy(), D.cpu().numpy()) <= 1e-13
    A, L = CASES["shift64"]()
    X = E.kron_solve(A, L @ L.T)
    print("ADI static n=64", flush=True)
    Z, D, info = lyap.solve_static(_cuda(A), _cuda(L), None, precisions=prec, solver=1)
    Zs, Ds = Z.cpu().numpy(), D.cpu().numpy()
    assert info["status"] == "OK" and _rel((Zs * Ds) @ Zs.T, X) <= 1e-11
    print("ADI refine from a perturbed factor n=64", flush=True)
    Zp = Zs + 1e-6 * np.random.default_rng(3).standard_normal(Zs.shape)
    Z, D, info = lyap.refine(_cuda(A), _cuda(L), None, _cuda(Zp), _cuda(Ds), precisions=prec,
                             solver=1)
    Z, D = Z.cpu().numpy(), D.cpu().numpy()
    assert info["status"] == "OK" and info["refinements"] >= 1
    assert _rel((Z * D) @ Z.T, X) <= 1e-11
    print("ADI fresh adjoint n=64", flush=True)
    C = np.random.default_rng(9).standard_normal((2, 64))
    Y, DY, info = lyap.solve_adjoint(_cuda(A), _cuda(C.T), None, precisions=prec, solver=1,
                                     reuse=0)
    Y, DY = Y.cpu().numpy(), DY.cpu().numpy()
    assert info["status"] == "OK" and not info["cache_reused"] and info["inversions"] > 0
    assert _rel((Y * DY) @ Y.T, E.kron_solve(A.T, C.T @ C)) <= 1e-11
