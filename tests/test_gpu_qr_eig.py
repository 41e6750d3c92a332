"""GPU tests of the thin QR and the symmetric spectral decomposition, through the C ABI.

References: backward error F - U T and orthogonality of U (any correct thin QR satisfies
them); LAPACK eigenvalues and the reconstruction H - V diag(w) V^T for the eigensolver."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lyap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_02126_amd as m
    return m


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("n,p", [(5, 3), (64, 64), (300, 33), (1000, 96), (4096, 150), (777, 65)])
def test_qr_full_rank(lyap, n, p):
    print(f"qr n={n} p={p}", flush=True)
    rng = np.random.default_rng(n + p)
    F = rng.standard_normal((n, p)) * np.logspace(0, -6, p)[None, :]
    U, T = (x.cpu().numpy() for x in lyap.qr(_cuda(F)))
    u = 2.0 ** -53
    assert np.linalg.norm(U @ T - F) <= 50 * u * np.sqrt(n * p) * np.linalg.norm(F)
    assert np.linalg.norm(U.T @ U - np.eye(p)) <= 50 * u * np.sqrt(n * p)
    assert np.allclose(np.tril(T, -1), 0.0)


@pytest.mark.parametrize("n,c,q", [(1000, 300, 400), (2048, 512, 512), (4096, 96, 33),
                                   (500, 40, 1)])
def test_qr_orthonormal_lead(lyap, n, c, q):
    # F = [Z, Y] with Z orthonormal and Y partly in the span of Z (the structure of a
    # truncated factor extended by A^{-1} Z): lyap_qr_lead keeps Z as the first columns of U
    # and I as the leading block of T; U T = F and U^T U = I to working precision, and T^T T
    # equals that of the plain Householder QR (both are F^T F).
    print(f"qr with orthonormal lead n={n} c={c} q={q}", flush=True)
    rng = np.random.default_rng(n + c + q)
    Z, _ = np.linalg.qr(rng.standard_normal((n, c)))
    Y = rng.standard_normal((n, q)) * np.logspace(0, -8, q)[None, :]
    k = min(q, c) // 2
    Y[:, :k] = Z[:, :k] @ rng.standard_normal((k, k)) + 1e-12 * rng.standard_normal((n, k))
    F = np.hstack([Z, Y])
    U, T = (x.cpu().numpy() for x in lyap.qr(_cuda(F), lead=c))
    u = 2.0 ** -53
    p = c + q
    assert np.array_equal(U[:, :c], Z)
    assert np.array_equal(T[:c, :c], np.eye(c))
    assert np.allclose(np.tril(T, -1), 0.0)
    assert np.linalg.norm(U @ T - F) <= 50 * u * np.sqrt(n * p) * np.linalg.norm(F)
    assert np.linalg.norm(U.T @ U - np.eye(p)) <= 50 * u * np.sqrt(n * p)
    U0, T0 = (x.cpu().numpy() for x in lyap.qr(_cuda(F)))
    G = F.T @ F
    assert np.linalg.norm(T.T @ T - T0.T @ T0) <= 100 * u * np.sqrt(n * p) * np.linalg.norm(G)


@pytest.mark.parametrize("n,c,q", [(512, 300, 400), (1000, 968, 500), (256, 256, 100),
                                   (300, 40, 400), (4096, 3900, 3900)])
def test_qr_orthonormal_lead_wide(lyap, n, c, q):
    # more columns than rows (c + q > n): U = [Z, Q2] is Z completed to an orthonormal basis
    # of the whole space and T = U^T F, whose first c columns are [I; 0]; U T = F and
    # U^T U = I to working precision
    print(f"qr with orthonormal lead, wide: n={n} c={c} q={q}", flush=True)
    rng = np.random.default_rng(n + 3 * c + q)
    Z, _ = np.linalg.qr(rng.standard_normal((n, c)))
    Y = rng.standard_normal((n, q)) * np.logspace(0, -8, q)[None, :]
    F = np.hstack([Z, Y])
    U, T = (x.cpu().numpy() for x in lyap.qr(_cuda(F), lead=c))
    u = 2.0 ** -53
    p = c + q
    assert U.shape == (n, n) and T.shape == (n, p)
    assert np.array_equal(U[:, :c], Z)
    assert np.array_equal(T[:, :c], np.eye(n, c))
    assert np.linalg.norm(U @ T - F) <= 50 * u * np.sqrt(n * p) * np.linalg.norm(F)
    assert np.linalg.norm(U.T @ U - np.eye(n)) <= 50 * u * n


def test_qr_rank_deficient(lyap):
    # F = [Z, A Z, L]-like: the middle block is (nearly) in the span of the others
    print("qr rank-deficient n=2048 p=136", flush=True)
    rng = np.random.default_rng(1)
    n, c, m = 2048, 64, 8
    Z = np.linalg.qr(rng.standard_normal((n, c)))[0]
    L = rng.standard_normal((n, m))
    B = Z @ rng.standard_normal((c, c)) + L @ rng.standard_normal((m, c)) \
        + 1e-12 * rng.standard_normal((n, c))
    F = np.hstack([Z, B, L])
    U, T = (x.cpu().numpy() for x in lyap.qr(_cuda(F)))
    u = 2.0 ** -53
    assert np.linalg.norm(U @ T - F) <= 100 * u * np.sqrt(n) * np.linalg.norm(F)
    assert np.linalg.norm(U.T @ U - np.eye(F.shape[1])) <= 1e-12


@pytest.mark.parametrize("p", [1, 5, 32, 37, 100, 256, 518, 2100, 4096])
def test_syev_indefinite(lyap, p):
    # graded indefinite spectra as in the truncations (2100: ragged, 66 blocks of 32 with
    # padding; 4096: the largest size the entry point takes)
    print(f"syev p={p}", flush=True)
    rng = np.random.default_rng(p)
    Q = np.linalg.qr(rng.standard_normal((p, p)))[0]
    lam = rng.standard_normal(p) * np.logspace(0, -10, p)
    H = (Q * lam) @ Q.T
    H = 0.5 * (H + H.T)
    w, V = (x.cpu().numpy() for x in lyap.syev(_cuda(H)))
    u = 2.0 ** -53
    ref = np.linalg.eigvalsh(H)
    ref = ref[np.argsort(-np.abs(ref), kind="stable")]
    nrm = np.linalg.norm(H)
    assert np.max(np.abs(w - ref)) <= 100 * u * p * nrm
    assert np.all(np.diff(np.abs(w)) <= 0)
    # Jacobi accumulates the block rotations into V: allow 1000 u p (about 6e-11 at p = 518)
    assert np.linalg.norm(V.T @ V - np.eye(p)) <= 1000 * u * p
    assert np.linalg.norm((V * w) @ V.T - H) <= 100 * u * p * nrm


def test_syev_rejects_oversize(lyap):
    print("syev p=4097 (rejected)", flush=True)
    with pytest.raises(lyap.LyapError) as e:
        lyap.syev(torch.zeros((4097, 4097), dtype=torch.float64, device="cuda"))
    assert e.value.status == "BADARG"


def test_syev_clustered_and_zero(lyap):
    print("syev clustered p=96", flush=True)
    rng = np.random.default_rng(7)
    p = 96
    Q = np.linalg.qr(rng.standard_normal((p, p)))[0]
    lam = np.concatenate([np.full(30, 2.0), np.full(30, -2.0), np.zeros(20), rng.standard_normal(16)])
    H = (Q * lam) @ Q.T
    H = 0.5 * (H + H.T)
    w, V = (x.cpu().numpy() for x in lyap.syev(_cuda(H)))
    assert np.linalg.norm((V * w) @ V.T - H) <= 1e-12 * np.linalg.norm(H)
    assert np.linalg.norm(V.T @ V - np.eye(p)) <= 1e-12
