"""GPU unit tests of the matrix-core product and the inversion, called through the C ABI.

References: float64 NumPy products of the operands rounded to the solver precision, and
LAPACK inverses.  Shapes span several tiles plus ragged tails."""
import numpy as np
import pytest
import torch

import lyapgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lyap():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_02126_amd as m
    return m


def _round(x, dtype):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype == "fp32":
        return t.float().double().numpy()
    if dtype == "fp16":
        return t.float().half().double().numpy()
    if dtype == "bf16":
        return t.float().bfloat16().double().numpy()
    return x


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("M,N,K,ta,tb", [
    (16, 16, 4, False, False), (67, 45, 33, False, False), (130, 70, 129, True, False),
    (64, 200, 90, False, True), (33, 17, 65, True, True), (512, 384, 300, False, False),
    (64, 32, 4096, True, False),   # split-K path
    # split-K on the tall-skinny shapes of the solvers' products; K = 4100 leaves the last
    # k-chunk empty
    (2000, 50, 3000, False, True), (300, 20, 4100, True, False), (4096, 130, 4096, False, False),
])
def test_gemm_f64(lyap, M, N, K, ta, tb):
    print(f"gemm_f64 M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(M * 7 + N)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    ref = 1.5 * ((A.T if ta else A) @ (B.T if tb else B)) - 0.5 * C0
    C = _cuda(C0)
    lyap.gemm(_cuda(A), _cuda(B), C, alpha=1.5, beta=-0.5, transa=ta, transb=tb)
    got = C.cpu().numpy()
    scale = np.abs(A).max() * np.abs(B).max() * K
    assert np.abs(got - ref).max() <= 1e-14 * scale


@pytest.mark.parametrize("M,N,K,ta,tb", [(67, 45, 33, False, False), (128, 96, 160, True, False),
                                         (50, 130, 70, False, True), (300, 260, 1000, False, False),
                                         (2000, 50, 3000, False, False),
                                         (300, 20, 4100, True, True)])
def test_gemm_split_fp16(lyap, M, N, K, ta, tb):
    # split binary16 operands (hi + 2^-11 lo): each operand is carried to 2^-22, the three
    # products are summed in binary32
    print(f"gemm_fp16x2 M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(K + 1)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    opA = (lambda X: X.T) if ta else (lambda X: X)
    opB = (lambda X: X.T) if tb else (lambda X: X)
    got = lyap.gemm(_cuda(A), _cuda(B), transa=ta, transb=tb, dtype="fp16x2").cpu().numpy()
    absprod = np.abs(opA(A)) @ np.abs(opB(B))
    err = np.abs(got - opA(A) @ opB(B))
    assert np.all(err <= (3 * 2.0 ** -22 + 4 * K * 2.0 ** -24) * absprod)
    g16 = lyap.gemm(_cuda(A), _cuda(B), transa=ta, transb=tb, dtype="fp16").cpu().numpy()
    assert np.median(err / absprod) * 100 < np.median(np.abs(g16 - opA(A) @ opB(B)) / absprod)


@pytest.mark.parametrize("dtype", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("M,N,K,ta,tb", [(67, 45, 33, False, False), (128, 96, 160, True, False),
                                         (50, 130, 70, False, True),
                                         # 128 x 128 tiles (>= 48 of them), ragged M, N, K
                                         (1000, 900, 200, False, False),
                                         (1000, 900, 200, True, False),
                                         (1000, 900, 200, False, True),
                                         (1000, 900, 200, True, True),
                                         # few tiles and a long k-loop: K split over
                                         # workgroups (K = 4100 leaves the last chunk empty)
                                         (1000, 40, 3000, False, False),
                                         (1000, 40, 3000, True, True),
                                         (300, 20, 4100, False, False),
                                         (4096, 130, 4096, False, False)])
def test_gemm_reduced(lyap, dtype, M, N, K, ta, tb):
    print(f"gemm_{dtype} M={M} N={N} K={K} ta={ta} tb={tb}", flush=True)
    rng = np.random.default_rng(K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    B = rng.standard_normal((N, K) if tb else (K, N))
    u_op = {"fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}[dtype]
    u32 = 2.0 ** -24
    opA = lambda X: X.T if ta else X
    opB = lambda X: X.T if tb else X
    # (1) operands already representable in the format: only the binary32 accumulation
    #     (in the matrix cores' own summation order) separates the result from the exact one
    Ar, Br = _round(A, dtype), _round(B, dtype)
    got = lyap.gemm(_cuda(Ar), _cuda(Br), transa=ta, transb=tb, dtype=dtype).cpu().numpy()
    absprod = np.abs(opA(Ar)) @ np.abs(opB(Br))
    ratio = float(np.max(np.abs(got - opA(Ar) @ opB(Br)) / (K * u32 * absprod + 1e-300)))
    print(f"  accumulation error / (K u32 |A||B|) = {ratio:.3f}", flush=True)
    assert ratio <= 4.0
    # (2) general operands: rounding each operand to the format costs at most u_op each
    got = lyap.gemm(_cuda(A), _cuda(B), transa=ta, transb=tb, dtype=dtype).cpu().numpy()
    absprod = np.abs(opA(A)) @ np.abs(opB(B))
    err = np.abs(got - opA(A) @ opB(B))
    assert np.all(err <= (2.01 * u_op + 4 * K * u32) * absprod + 1e-300)


@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp16", "bf16", "fp16x2"])
def test_split_k_products_are_deterministic(lyap, dtype):
    # the split-K partial products are summed in a fixed order: repeated calls agree bit for bit
    print(f"gemm split-K determinism {dtype} 2000 x 50 x 3000", flush=True)
    rng = np.random.default_rng(11)
    A, B = _cuda(rng.standard_normal((2000, 3000))), _cuda(rng.standard_normal((3000, 50)))
    first = lyap.gemm(A, B, dtype=dtype).cpu().numpy()
    for _ in range(2):
        assert np.array_equal(lyap.gemm(A, B, dtype=dtype).cpu().numpy(), first)


@pytest.mark.parametrize("n", [1, 7, 37, 200, 1000])
@pytest.mark.parametrize("dtype", ["fp64", "fp32", "fp16", "bf16", "fp16x2"])
def test_inverse_accuracy(lyap, n, dtype):
    print(f"inverse {dtype} n={n}", flush=True)
    A, _ = lyapgen.random_shift(100 + n, n, 1)
    X = lyap.inverse(_cuda(A), dtype).cpu().numpy()
    Xr = np.linalg.inv(A)
    kappa = np.linalg.cond(A, 1)
    u = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8,
         "fp16x2": 2.0 ** -22}[dtype]
    err = np.linalg.norm(X - Xr, 1) / np.linalg.norm(Xr, 1)
    assert err <= 20 * n ** 0.5 * kappa * u, err
    res = np.linalg.norm(A @ X - np.eye(n), 1)
    assert res <= 20 * n ** 0.5 * kappa * u + 1e-300


def test_inverse_needs_pivoting_and_large(lyap):
    # a permutation-like matrix: zero diagonal, so unpivoted elimination would break down
    n = 4096
    rng = np.random.default_rng(5)
    perm = rng.permutation(n)
    A = np.zeros((n, n))
    A[np.arange(n), perm] = 1.0 + rng.random(n)
    A += 1e-3 * rng.standard_normal((n, n)) / np.sqrt(n)
    print("inverse fp64 n=4096 permutation-like", flush=True)
    X = lyap.inverse(_cuda(A), "fp64").cpu().numpy()
    assert np.linalg.norm(A @ X - np.eye(n), 1) <= 1e-10
    print("inverse fp32 n=4096 permutation-like", flush=True)
    X32 = lyap.inverse(_cuda(A), "fp32").cpu().numpy()
    assert np.linalg.norm(A @ X32 - np.eye(n), 1) <= 1e-3


def test_inverse_singular_reports(lyap):
    A = np.diag([1.0, 2.0, 0.0, 3.0])
    with pytest.raises(lyap.LyapError) as e:
        lyap.inverse(_cuda(A), "fp64")
    assert e.value.status == "SINGULAR"


def test_inverse_deterministic(lyap):
    A, _ = lyapgen.random_shift(3, 300, 1)
    a = lyap.inverse(_cuda(A), "fp16").cpu().numpy()
    b = lyap.inverse(_cuda(A), "fp16").cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [1, 63, 64, 65, 777, 4096])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_inverse_diag_dominant_unpivoted(lyap, n, dtype):
    # ||A + I||_1 < 1 makes A strictly column diagonally dominant: partial pivoting picks the
    # diagonal at every step, so the solver's unpivoted route computes the same elimination
    # (the two differ only by the blocking of the update products)
    print(f"inverse unpivoted {dtype} n={n}", flush=True)
    rng = np.random.default_rng(9 + n)
    E = rng.standard_normal((n, n))
    E *= 0.5 / np.abs(E).sum(axis=0, keepdims=True)
    A = -np.eye(n) + E
    Xp = lyap.inverse(_cuda(A), dtype, pivot=True).cpu().numpy()
    Xn = lyap.inverse(_cuda(A), dtype, pivot=False).cpu().numpy()
    u = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}[dtype]
    kappa = np.linalg.cond(A, 1)
    tol = 20 * n ** 0.5 * kappa * u
    for X in (Xp, Xn):
        assert np.linalg.norm(A @ X - np.eye(n), 1) <= tol
    assert np.linalg.norm(Xn - Xp, 1) / np.linalg.norm(Xp, 1) <= tol


@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_inverse_unpivoted_repeatable(lyap, dtype):
    # every workgroup of the unpivoted panel update reads only the panel entries it writes
    # itself, so repeated inversions agree bit for bit whatever ran before them
    print(f"inverse unpivoted repeatability {dtype}", flush=True)
    rng = np.random.default_rng(31)
    mats = []
    for n in (131, 777, 2048):
        E = rng.standard_normal((n, n))
        E *= 0.9 / np.abs(E).sum(axis=0, keepdims=True)
        mats.append(_cuda(-np.eye(n) + E))
    first = [lyap.inverse(M, dtype, pivot=False) for M in mats]
    for rep in range(6):
        for k in ((rep + 1) % 3, rep % 3, (rep + 2) % 3):
            X = lyap.inverse(mats[k], dtype, pivot=False)
            assert torch.equal(X, first[k]), (rep, k)


def test_inverse_unpivoted_zero_pivot_reports(lyap):
    A = np.array([[0.0, 1.0], [1.0, 0.0]])
    with pytest.raises(lyap.LyapError) as e:
        lyap.inverse(_cuda(A), "fp64", pivot=False)
    assert e.value.status == "SINGULAR"
    X = lyap.inverse(_cuda(A), "fp64", pivot=True).cpu().numpy()
    assert np.array_equal(X, A)


@pytest.mark.parametrize("n", [4, 200, 1000, 4096])
@pytest.mark.parametrize("dtype", ["fp64", "fp32"])
def test_inverse_random_butterfly(lyap, n, dtype):
    # A^{-1} = V (U^T A V)^{-1} U^T with random depth-2 butterflies and no pivoting: as
    # accurate as the pivoted inversion on the same matrix
    print(f"inverse rbt {dtype} n={n}", flush=True)
    A, _ = lyapgen.random_shift(100 + n, n, 1)
    X = lyap.inverse(_cuda(A), dtype, pivot="rbt").cpu().numpy()
    Xp = lyap.inverse(_cuda(A), dtype, pivot=True).cpu().numpy()
    u = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24}[dtype]
    kappa = np.linalg.cond(A, 1)
    res = np.linalg.norm(A @ X - np.eye(n), 1)
    resp = np.linalg.norm(A @ Xp - np.eye(n), 1)
    print(f"  ||AX - I||_1 rbt {res:.2e} pivoted {resp:.2e}", flush=True)
    assert res <= 20 * n ** 0.5 * kappa * u
    assert res <= 10 * resp + 10 * n * u
    # the same seeded transformation every call
    assert torch.equal(lyap.inverse(_cuda(A), dtype, pivot="rbt"), _cuda(X))
    with pytest.raises(lyap.LyapError):
        lyap.inverse(_cuda(A[:3, :3] - 3 * np.eye(3)), dtype, pivot="rbt")  # n % 4 != 0
