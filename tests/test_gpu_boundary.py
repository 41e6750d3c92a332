"""The C-ABI calls beyond the basic solve, through the library on the GPU: a caller-owned
workspace (lyap_workspace_size), a full symmetric S, warm-started refinement (lyap_refine),
inverse-sequence replay keyed by the content of A, precision escalation, working precision
u = fp32 (Table 3.1's u = fp32 rows), the alternative Newton scalings of Section 3, the
scaled (power-of-two) storage of reduced-precision operands, and every failure status
forced through normal, fault-free runs."""
import math

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


def _np(*ts):
    return [t.cpu().numpy() for t in ts]


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _small():
    cfg = lyapgen.config("small")
    return cfg["A"], cfg["L"]


# ------------------------------------------------------------------------- workspace
def test_caller_workspace_gives_identical_factors(lyap):
    A, L = _small()
    n, m = L.shape
    print("caller workspace n=64 fp16", flush=True)
    nbytes = lyap.workspace_size(n, m, "fp16")
    assert nbytes > 8 * n * n
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    Z1, D1, i1 = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp16", "fp64", "fp64", "fp64"))
    Z2, D2, i2 = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp16", "fp64", "fp64", "fp64"),
                            ws=ws)
    assert i1["status"] == i2["status"] == "OK"
    assert torch.equal(Z1, Z2) and torch.equal(D1, D2)
    # too small, or misaligned: rejected before any device work
    with pytest.raises(lyap.LyapError) as e:
        lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp16", "fp64", "fp64", "fp64"),
                   ws=ws[: nbytes - 4096])
    assert e.value.status == "WORKSPACE"
    with pytest.raises(lyap.LyapError) as e:
        lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp16", "fp64", "fp64", "fp64"),
                   ws=ws[8:])
    assert e.value.status == "WORKSPACE"


def test_workspace_size_grows_with_k_max_and_escalation(lyap):
    a = lyap.workspace_size(512, 4, "fp16")
    b = lyap.workspace_size(512, 4, "fp16", k_max=10)
    c = lyap.workspace_size(512, 4, "fp16", escalate=1)
    assert b < a < c
    # 40 fewer cached fp16 inverses of 512 x 512
    assert a - b >= 40 * 512 * 512 * 2


# --------------------------------------------------------------------------- full S
@pytest.mark.parametrize("us", ["fp64", "fp16"])
def test_full_symmetric_s(lyap, us):
    A, L = lyapgen.random_shift(4, 64, 3)
    rng = np.random.default_rng(11)
    B = rng.standard_normal((3, 3))
    S = B + B.T
    W = L @ S @ L.T
    X = E.kron_solve(A, W)
    print(f"full S n=64 m=3 us={us}", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), _cuda(S), precisions=(us, "fp64", "fp64", "fp64"))
    Z, D = _np(Z, D)
    Xh = (Z * D) @ Z.T
    print(f"  status={info['status']} res={info['res']:.2e} err={_rel(Xh, X):.2e}", flush=True)
    assert info["status"] == "OK"
    assert R.relres_dense(A, W, Xh) <= 1e-13
    assert _rel(Xh, X) <= 1e-11


# ------------------------------------------------------------------------ warm start
def _exact_factor(A, W):
    X = E.bartels_stewart(A, W)
    w, V = np.linalg.eigh(0.5 * (X + X.T))
    keep = np.abs(w) > 1e-15 * np.abs(w).max()
    return V[:, keep], w[keep], X


def test_refine_from_the_solution_does_nothing(lyap):
    A, L = lyapgen.random_shift(2, 48, 3)
    Z0, d0, X = _exact_factor(A, L @ L.T)
    print("refine from exact n=48", flush=True)
    Z, D, info = lyap.refine(_cuda(A), _cuda(L), None, _cuda(Z0), _cuda(d0),
                             precisions=("fp16", "fp64", "fp64", "fp64"))
    assert info["status"] == "OK" and info["refinements"] == 0 and info["inversions"] == 0
    assert info["res"] <= 1e-13


def test_refine_from_a_perturbed_solution_matches_oracle(lyap):
    A, L = lyapgen.random_shift(2, 48, 3)
    Z0, d0, X = _exact_factor(A, L @ L.T)
    Zp = Z0 + 1e-5 * np.random.default_rng(1).standard_normal(Z0.shape)
    _, _, io = IR.ir_ldlt(A, L, None, prec=("fp32", "fp64", "fp64", "fp64"), Z0=Zp, d0=d0)
    print("refine from perturbed n=48 fp32", flush=True)
    Z, D, info = lyap.refine(_cuda(A), _cuda(L), None, _cuda(Zp), _cuda(d0),
                             precisions=("fp32", "fp64", "fp64", "fp64"))
    Z, D = _np(Z, D)
    print(f"  gpu res {info['res_hist']} oracle {io.res_hist}", flush=True)
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert info["inversions"] == io.inversions
    assert abs(info["refinements"] - io.refinements) <= 1
    assert _rel((Z * D) @ Z.T, X) <= 1e-10


def test_refine_after_solve_replays_the_inverse_sequence(lyap):
    A, L = lyapgen.random_shift(2, 48, 3)
    ws = torch.empty(lyap.workspace_size(48, 3, "fp32"), dtype=torch.uint8, device="cuda")
    Ad, Ld = _cuda(A), _cuda(L)
    print("solve + refine in one workspace n=48", flush=True)
    Z1, D1, i1 = lyap.solve(Ad, Ld, None, precisions=("fp32", "fp64", "fp64", "fp64"), tol=1e-9,
                            ws=ws)
    assert i1["status"] == "OK" and i1["inversions"] > 0
    Z2, D2, i2 = lyap.refine(Ad, Ld, None, Z1, D1, precisions=("fp32", "fp64", "fp64", "fp64"),
                             ws=ws)
    assert i2["status"] == "OK" and i2["res"] <= 1e-13
    if i2["refinements"] > 0:
        assert i2["cache_reused"] and i2["inversions"] == 0


# ------------------------------------------------------- replay keyed by content of A
def test_adjoint_replay_follows_the_contents_of_a(lyap):
    A, L = _small()
    C = np.random.default_rng(21).standard_normal((2, A.shape[0]))
    Ad = _cuda(A)
    print("adjoint replay keyed by content", flush=True)
    lyap.solve(Ad, _cuda(L), None, precisions=("fp32", "fp64", "fp64", "fp64"))
    # same contents in another tensor: replayed
    _, _, i1 = lyap.solve_adjoint(Ad.clone(), _cuda(C.T), None,
                                  precisions=("fp32", "fp64", "fp64", "fp64"))
    assert i1["cache_reused"] and i1["inversions"] == 0 and i1["status"] == "OK"
    # the same tensor edited in place (Frobenius norm kept: a swap of two entries): recomputed
    lyap.solve(Ad, _cuda(L), None, precisions=("fp32", "fp64", "fp64", "fp64"))
    a, b = Ad[0, 1].item(), Ad[1, 0].item()
    Ad[0, 1], Ad[1, 0] = b, a
    _, _, i2 = lyap.solve_adjoint(Ad, _cuda(C.T), None,
                                  precisions=("fp32", "fp64", "fp64", "fp64"))
    assert not i2["cache_reused"] and i2["inversions"] > 0 and i2["status"] == "OK"
    Y = E.bartels_stewart(Ad.cpu().numpy().T, C.T @ C)
    assert i2["res"] <= 1e-13 and np.isfinite(Y).all()
    # a forward solve never replays by default
    _, _, i3 = lyap.solve(Ad, _cuda(L), None, precisions=("fp32", "fp64", "fp64", "fp64"))
    assert not i3["cache_reused"] and i3["inversions"] > 0


# ------------------------------------------------------------------------ escalation
def test_escalation_rescues_bf16(lyap):
    A, L = lyapgen.paper_family(60, 6.0, seed=3)
    print("escalate bf16 paper family n=60 q=6", flush=True)
    _, _, plain = lyap.solve(_cuda(A), _cuda(L), None,
                             precisions=("bf16", "fp64", "fp64", "fp64"), raise_on_error=False)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("bf16", "fp64", "fp64", "fp64"),
                            escalate=1, raise_on_error=False)
    print(f"  plain {plain['status']} {plain['res']:.2e}; escalated {info['status']} "
          f"{info['res']:.2e} u_s_final={info['u_s_final']} escalations={info['escalations']}",
          flush=True)
    assert plain["status"] != "OK"
    assert info["status"] == "OK" and info["escalations"] >= 1
    assert info["u_s_final"] in ("fp16", "fp32", "fp64")
    Z, D = _np(Z, D)
    assert R.relres(A, L, None, Z, D) <= 1e-13
    _, _, io = IR.ir_ldlt(A, L, None, prec=("bf16", "fp64", "fp64", "fp64"), escalate=True)
    assert io.status == "OK"


# ------------------------------------------------------------- working precision fp32
@pytest.mark.parametrize("prec", [("fp32", "fp32", "fp32", "fp32"), ("fp16", "fp32", "fp32", "fp32"),
                                  ("fp32", "fp32", "fp64", "fp64")])
def test_working_precision_fp32(lyap, prec):
    A, L = lyapgen.random_shift(3, 64, 2)
    X = E.kron_solve(A, L @ L.T)
    print(f"u=fp32 n=64 prec={prec}", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=prec, tol=1e-7)
    Z, D = _np(Z, D)
    res = R.relres(A, L, None, Z, D)
    err = _rel((Z * D) @ Z.T, X)
    _, _, io = IR.ir_ldlt(A, L, None, prec=prec, tol=1e-7)
    print(f"  status={info['status']} res={res:.2e} err={err:.2e} refinements="
          f"{info['refinements']} (oracle {io.refinements}, res {io.res_hist})", flush=True)
    assert info["status"] == "OK" and res <= 1e-7
    assert np.array_equal(Z.astype(np.float32).astype(np.float64), Z)
    assert np.array_equal(D.astype(np.float32).astype(np.float64), D)
    assert err <= 1e3 * 2.0 ** -24
    assert abs(info["refinements"] - io.refinements) <= 1


def test_working_precision_fp32_stagnates(lyap):
    A, L = lyapgen.random_shift(3, 64, 2)
    print("u=fp32 tol=1e-13 -> STAGNATED", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp32",) * 4, tol=1e-13,
                            raise_on_error=False)
    assert info["status"] == "STAGNATED"
    assert 1e-10 < info["res"] < 1e-6 and Z.shape[1] > 0


# --------------------------------------------------------------------------- scalings
@pytest.mark.parametrize("kind,code", [("det", 1), ("2norm", 2), ("spectral", 3),
                                       ("combined", 4)])
def test_alternative_scalings(lyap, kind, code):
    A, L = _small()
    X = E.kron_solve(A, L @ L.T)
    seq = SN.a_sequence(A, "fp64", scaling_kind=kind)
    print(f"scaling {kind} n=64", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp64",) * 4, scaling=code)
    Z, D = _np(Z, D)
    print(f"  mus gpu {info['mus']} oracle {seq.mus}", flush=True)
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert _rel((Z * D) @ Z.T, X) <= 1e-11
    # determinantal: from the pivots, exact up to rounding; the others are power-iteration
    # estimates of norms / spectral radii
    exact = kind in ("det", "combined")
    tol = 1e-9 if exact else 0.05
    assert info["mus"][0] == pytest.approx(seq.mus[0], rel=tol)
    assert abs(info["inversions"] - seq.K) <= (0 if exact else 1)
    if kind == "combined":
        # determinantal first, then the Frobenius scaling of the iterates it produced
        assert np.allclose(info["mus"][:seq.K], seq.mus, rtol=1e-8)


def test_determinantal_scaling_of_scaled_identity(lyap):
    A = -3.0 * np.eye(40)
    L = np.random.default_rng(2).standard_normal((40, 2))
    for us in ("fp64", "fp32", "fp16"):
        _, _, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=(us, "fp64", "fp64", "fp64"),
                                scaling=1)
        assert info["status"] == "OK"
        assert info["mus"][0] == pytest.approx(1.0 / 3.0, rel=1e-6)


# -------------------------------------------------- scaled storage of reduced precisions
@pytest.mark.parametrize("us", ["fp16", "bf16"])
def test_reduced_precision_solve_is_scale_invariant(lyap, us):
    # A <- 2^-20 A makes max|A_k^-1| ~ 1e6 (beyond fp16's 65504) and L <- 2^8 L makes the
    # factor's entries ~ 1e3: without power-of-two scaled casts the cached inverse and the
    # product operands would overflow.  X scales as 2^(20 + 16) X.
    A, L = _small()
    c, g = 2.0 ** -20, 2.0 ** 8
    X = E.kron_solve(A, L @ L.T)
    print(f"scale invariance {us}", flush=True)
    Z, D, info = lyap.solve(_cuda(c * A), _cuda(g * L), None,
                            precisions=(us, "fp64", "fp64", "fp64"))
    Z, D = _np(Z, D)
    Xs = (Z * D) @ Z.T * (c / g ** 2)
    print(f"  status={info['status']} res={info['res']:.2e} err={_rel(Xs, X):.2e}", flush=True)
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert _rel(Xs, X) <= 1e-11
    Z1, D1, _ = lyap.solve(_cuda(A), _cuda(L), None, precisions=(us, "fp64", "fp64", "fp64"))
    Z1, D1 = _np(Z1, D1)
    assert _rel(Xs, (Z1 * D1) @ Z1.T) <= 1e-11


# ----------------------------------------------------------- forced failure statuses
def test_status_stagnated_with_zero_tolerance(lyap):
    A, L = _small()
    print("tol=0 -> STAGNATED", flush=True)
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp32", "fp64", "fp64", "fp64"),
                            tol=0.0, raise_on_error=False)
    h = info["res_hist"]
    print(f"  {info['status']} {h}", flush=True)
    assert info["status"] == "STAGNATED"
    assert h[-1] > 0.9 * h[-2] and h[-2] > 0.9 * h[-3]
    assert Z.shape[1] > 0 and info["res"] <= 1e-14
    _, _, io = IR.ir_ldlt(A, L, None, prec=("fp32", "fp64", "fp64", "fp64"), tol=0.0)
    assert io.status == "STAGNATED"


def test_status_not_converged_with_one_step(lyap):
    A, L = _small()
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp16", "fp64", "fp64", "fp64"),
                            i_max=1, raise_on_error=False)
    assert info["status"] == "NOT_CONVERGED" and info["refinements"] == 0
    assert info["res"] > 1e-13 and Z.shape[1] > 0


def test_status_capacity(lyap):
    A, L = _small()
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp64",) * 4, z_cap=3,
                            raise_on_error=False)
    assert info["status"] == "CAPACITY" and info["rank"] > 3


def test_status_nonfinite_and_badarg(lyap):
    n = 64
    L = np.random.default_rng(3).standard_normal((n, 2))
    # finite A whose inverse's squared Frobenius norm overflows binary64
    A = -(2.0 ** -600) * np.eye(n)
    _, _, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=("fp64",) * 4,
                            raise_on_error=False)
    assert info["status"] == "NONFINITE"
    A2, _ = _small()
    A2 = A2.copy()
    A2[3, 7] = np.nan
    with pytest.raises(lyap.LyapError) as e:
        lyap.solve(_cuda(A2), _cuda(L), None, precisions=("fp64",) * 4)
    assert e.value.status == "BADARG"
    with pytest.raises(lyap.LyapError) as e:  # u_s finer than u
        lyap.solve(_cuda(_small()[0]), _cuda(L), None, precisions=("fp64", "fp32", "fp32", "fp32"))
    assert e.value.status == "BADARG"


# ----------------------------------------------------------- random butterfly pivoting
@pytest.mark.parametrize("us", ["fp64", "fp32", "fp16"])
def test_butterfly_pivoting_solve(lyap, us):
    # opt.pivoting = 1: the pivoted inversions go through the random butterfly
    # transformation (probe-checked); the solve reaches the same accuracy and the FP64
    # Newton count is unchanged
    A, L, Q, T = lyapgen.schur_family(7, 300, 3, lo=-2.0)
    X = E.schur_solve(Q, T, L @ L.T)
    print(f"butterfly pivoting n=300 {us}", flush=True)
    _, _, ref = lyap.solve(_cuda(A), _cuda(L), None, precisions=(us, "fp64", "fp64", "fp64"))
    Z, D, info = lyap.solve(_cuda(A), _cuda(L), None, precisions=(us, "fp64", "fp64", "fp64"),
                            pivoting=1)
    Z, D = _np(Z, D)
    print(f"  {info['status']} res={info['res']:.2e} rbt={info['rbt_steps']} "
          f"fallbacks={info['rbt_fallbacks']} K={info['inversions']} (pivoted K={ref['inversions']})",
          flush=True)
    assert info["status"] == "OK" and info["res"] <= 1e-13
    assert info["rbt_steps"] >= 1 and info["rbt_fallbacks"] == 0
    assert _rel((Z * D) @ Z.T, X) <= 1e-9
    if us == "fp64":
        assert info["inversions"] == ref["inversions"]
    # n % 4 != 0: partial pivoting throughout
    A2, L2 = lyapgen.random_shift(8, 65, 2)
    _, _, i2 = lyap.solve(_cuda(A2), _cuda(L2), None, precisions=(us, "fp64", "fp64", "fp64"),
                          pivoting=1)
    assert i2["status"] == "OK" and i2["rbt_steps"] == 0
