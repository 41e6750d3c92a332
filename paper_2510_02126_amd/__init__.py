"""MI355X (gfx950) solver for low-rank Lyapunov equations A X + X A^T + W = 0.

Python entry points over the C ABI of liblyap.so (include/lyap.h).  Tensors must be CUDA
(HIP) float64 tensors on the same device; they are passed by pointer together with the
current stream.  All arithmetic runs in the library's HIP kernels.

    solve(A, L, S=None, precisions=("fp16", "fp64", "fp64", "fp64"), tol=1e-13, ...)
        -> (Z, D, info) with X ~ Z diag(D) Z^T     (Alg 2.2 with Alg 3.2 as the solver)
    refine(A, L, S, Z0, D0, ...)      -- the same refinement started from X_0 = Z0 diag(D0) Z0^T
    workspace_size(n, m, u_s, **opts) -- bytes of the device workspace a solve needs
    (every solve accepts ``ws=``, a uint8 CUDA tensor of at least that size; the call then
     allocates no device memory)
    solve_batched(As, Ls, Ss=None, ...) -- independent equations of uneven sizes, concurrently
    solve_adjoint(A, L, S=None, ...)  -- A^T Y + Y A + L S L^T = 0, replaying the inverses
    lyapunov_trace_loss(A, L, S, C)   -- tr(C X C^T), differentiable (adjoint backward)
    inverse(A, dtype, pivot) -- inversion at a solver precision (Gauss-Jordan)
    gemm(A, B, ...)          -- matrix-core product
    qr(F) -> (U, T)          -- thin QR of a tall matrix
    syev(H) -> (w, V)        -- symmetric spectral decomposition
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import DTYPES, Info, LyapError, Options, Precisions

__all__ = ["solve", "solve_static", "refine", "workspace_size", "solve_batched", "solve_adjoint", "trace_loss", "trace_loss_grad", "LyapunovTraceLoss",
           "lyapunov_trace_loss", "inverse", "gemm", "qr", "syev", "LyapError", "version"]


def _dev(*ts):
    dev = None
    for t in ts:
        if t is None:
            continue
        if not t.is_cuda:
            raise ValueError("tensors must be on a GPU device")
        if t.dtype != torch.float64:
            raise ValueError("tensors must be float64")
        if dev is None:
            dev = t.device.index if t.device.index is not None else torch.cuda.current_device()
    return dev


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _rowmajor(t):
    """(tensor, leading dimension) for a row-major view with unit column stride."""
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        t = t.contiguous()
    return t, t.stride(0)


def version() -> str:
    return _lib.lib().lyap_version().decode()


def inverse(A: torch.Tensor, dtype: str = "fp64", pivot=True) -> torch.Tensor:
    """A^{-1} at solver precision ``dtype``: pivot True (partial pivoting), False (none) or
    "rbt" (random butterfly transformation, no pivoting)."""
    dev = _dev(A)
    n = A.shape[0]
    A, lda = _rowmajor(A)
    out = torch.empty((n, n), dtype=torch.float64, device=A.device)
    pv = 2 if pivot == "rbt" else int(bool(pivot))
    code = _lib.lib().lyap_inverse(_lib.handle(dev), _stream(dev), DTYPES[dtype], pv,
                                   n, _ptr(A), lda, _ptr(out), n)
    _lib.check(code, "lyap_inverse")
    return out


def gemm(A, B, C=None, alpha=1.0, beta=0.0, transa=False, transb=False, dtype="fp64"):
    dev = _dev(A, B, C)
    A, lda = _rowmajor(A)
    B, ldb = _rowmajor(B)
    M = A.shape[1] if transa else A.shape[0]
    K = A.shape[0] if transa else A.shape[1]
    N = B.shape[0] if transb else B.shape[1]
    if C is None:
        C = torch.zeros((M, N), dtype=torch.float64, device=A.device)
        beta = 0.0
    if C.stride(1) != 1:
        raise ValueError("C must have unit column stride")
    code = _lib.lib().lyap_gemm(_lib.handle(dev), _stream(dev), DTYPES[dtype], int(transa),
                                int(transb), M, N, K, float(alpha), _ptr(A), lda, _ptr(B), ldb,
                                float(beta), _ptr(C), C.stride(0))
    _lib.check(code, "lyap_gemm")
    return C


def qr(F: torch.Tensor, lead: int = 0):
    """Thin QR F = U T (library kernels).  ``lead`` > 0 states that the first ``lead``
    columns of F are orthonormal (lyap_qr_lead)."""
    dev = _dev(F)
    F, ldf = _rowmajor(F)
    n, p = F.shape
    k = min(n, p)
    U = torch.empty((n, k), dtype=torch.float64, device=F.device)
    T = torch.empty((k, p), dtype=torch.float64, device=F.device)
    if lead > 0:
        code = _lib.lib().lyap_qr_lead(_lib.handle(dev), _stream(dev), n, p, int(lead), _ptr(F),
                                       ldf, _ptr(U), k, _ptr(T), p)
        _lib.check(code, "lyap_qr_lead")
        return U, T
    code = _lib.lib().lyap_qr(_lib.handle(dev), _stream(dev), n, p, _ptr(F), ldf, _ptr(U), k,
                              _ptr(T), p)
    _lib.check(code, "lyap_qr")
    return U, T


def syev(H: torch.Tensor):
    dev = _dev(H)
    H, ldh = _rowmajor(H)
    p = H.shape[0]
    w = torch.empty(p, dtype=torch.float64, device=H.device)
    V = torch.empty((p, p), dtype=torch.float64, device=H.device)
    code = _lib.lib().lyap_syev(_lib.handle(dev), _stream(dev), p, _ptr(H), ldh, _ptr(w),
                                _ptr(V), p)
    _lib.check(code, "lyap_syev")
    return w, V


def jacobi_schedule(nb: int):
    """The block-pair schedule of the Jacobi sweeps (host only): ``pairs`` (nb, nb/2, 2) with
    pairs[t, k] the blocks of pair k in round t, and ``bmap`` (nb, nb) with
    bmap[t, b] = 2 k + h for block b at half h of pair k of round t."""
    import numpy as np

    pairs = np.zeros(max(nb, 0) * max(nb, 0), dtype=np.int32)
    bmap = np.zeros(max(nb, 0) * max(nb, 0), dtype=np.int32)
    code = _lib.lib().lyap_jacobi_schedule(int(nb), pairs.ctypes.data, bmap.ctypes.data)
    _lib.check(code, "lyap_jacobi_schedule")
    return pairs.reshape(nb, nb // 2, 2), bmap.reshape(nb, nb)


def _options(tol, refine, opts):
    o = _lib.default_options()
    o.tol = tol
    o.refine = int(bool(refine))
    for k, v in opts.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _s_args(S):
    """(tensor, lds): lds = 0 for a vector of diagonal entries, the row stride for an m x m S."""
    if S is None:
        return None, 0
    if S.dim() == 1:
        return S.contiguous(), 0
    S, lds = _rowmajor(S)
    return S, lds


def _ws_args(ws):
    if ws is None:
        return ctypes.c_void_p(0), 0
    if not ws.is_cuda or ws.dtype != torch.uint8:
        raise ValueError("ws must be a uint8 CUDA tensor")
    return ctypes.c_void_p(ws.data_ptr()), ws.numel()


def workspace_size(n, m, u_s="fp64", **opts) -> int:
    """Bytes of device workspace a solve of order n with m columns in L needs
    (lyap_workspace_size); ``opts`` are lyap_options fields (k_max, form, escalate, ...)."""
    o = _options(1e-13, True, opts)
    out = ctypes.c_size_t(0)
    _lib.check(_lib.lib().lyap_workspace_size(int(n), int(m), DTYPES[u_s], ctypes.byref(o),
                                              ctypes.byref(out)), "lyap_workspace_size")
    return out.value


def _solve(fn_name, A, L, S, precisions, tol, refine, z_cap, raise_on_error, opts, ws=None,
           Z0=None, D0=None):
    dev = _dev(A, L, S, Z0, D0)
    n = A.shape[0]
    m = L.shape[1]
    A, lda = _rowmajor(A)
    L, ldl = _rowmajor(L)
    S, lds = _s_args(S)
    if z_cap is None:
        z_cap = n  # the rank of X never exceeds n
    Z = torch.zeros((n, z_cap), dtype=torch.float64, device=A.device)
    Dv = torch.zeros(z_cap, dtype=torch.float64, device=A.device)
    o = _options(tol, refine, opts)
    prec = Precisions(*[DTYPES[p] for p in precisions])
    rank = ctypes.c_int(0)
    info = Info()
    wsp, wsb = _ws_args(ws)
    fn = getattr(_lib.lib(), fn_name)
    if fn_name == "lyap_refine":
        Z0, ldz0 = _rowmajor(Z0) if Z0.shape[1] > 0 else (Z0, max(1, Z0.shape[1]))
        D0 = D0.contiguous()
        code = fn(_lib.handle(dev), _stream(dev), n, m, _ptr(A), lda, _ptr(L), ldl, _ptr(S), lds,
                  prec, ctypes.byref(o), _ptr(Z0), ldz0, _ptr(D0), Z0.shape[1], _ptr(Z), z_cap,
                  z_cap, _ptr(Dv), ctypes.byref(rank), wsp, wsb, ctypes.byref(info))
    elif fn_name == "lyap_solve_static":
        code = fn(_lib.handle(dev), _stream(dev), n, m, _ptr(A), lda, _ptr(L), ldl, _ptr(S), lds,
                  prec, ctypes.byref(o), _ptr(Z), z_cap, z_cap, _ptr(Dv), ctypes.byref(rank),
                  ctypes.byref(info))
    else:
        code = fn(_lib.handle(dev), _stream(dev), n, m, _ptr(A), lda, _ptr(L), ldl, _ptr(S), lds,
                  prec, ctypes.byref(o), _ptr(Z), z_cap, z_cap, _ptr(Dv), ctypes.byref(rank),
                  wsp, wsb, ctypes.byref(info))
    d = info.as_dict()
    d["code"] = code
    if code != 0 and raise_on_error and code not in (1, 2):
        _lib.check(code, fn_name)
    r = rank.value
    return Z[:, :r], Dv[:r], d


def solve(A, L, S=None, precisions=("fp16", "fp64", "fp64", "fp64"), tol=1e-13, refine=True,
          z_cap=None, raise_on_error=True, ws=None, **opts):
    """Alg 2.2 (LDL^T-type mixed-precision IR) on the GPU for A X + X A^T + L S L^T = 0.
    S: None (S = I), a vector (the diagonal of S) or an m x m symmetric matrix.  Returns
    (Z, D, info) with X ~ Z diag(D) Z^T.  ``form=1`` (with S = None) runs the Cholesky type,
    Alg 2.1, and returns the Cholesky-type factor (X ~ Z Z^T, D = 1).  ``ws``: optional
    caller workspace (uint8 CUDA tensor of at least workspace_size(...) bytes)."""
    return _solve("lyap_solve", A, L, S, precisions, tol, refine, z_cap, raise_on_error, opts,
                  ws=ws)


def solve_static(A, L, S=None, precisions=("fp16", "fp64", "fp64", "fp64"), tol=1e-13,
                 refine=True, z_cap=None, raise_on_error=True, **opts):
    """lyap_solve in the library's fixed 64 MiB device scratch (lyap_solve_static): no
    device allocation inside the call; problems needing more workspace raise TOO_LARGE.
    Calls overlapping in time on one GPU must be serialised by the caller."""
    return _solve("lyap_solve_static", A, L, S, precisions, tol, refine, z_cap, raise_on_error,
                  opts)


def refine(A, L, S, Z0, D0, precisions=("fp16", "fp64", "fp64", "fp64"), tol=1e-13,
           z_cap=None, raise_on_error=True, ws=None, **opts):
    """Alg 2.1 / 2.2 started from X_0 = Z0 diag(D0) Z0^T (lyap_refine).  Returns (Z, D, info)."""
    return _solve("lyap_refine", A, L, S, precisions, tol, True, z_cap, raise_on_error, opts,
                  ws=ws, Z0=Z0, D0=D0)


def solve_batched(As, Ls, Ss=None, precisions=("fp16", "fp64", "fp64", "fp64"), tol=1e-13,
                  refine=True, z_caps=None, workers=0, raise_on_error=True, ws=None, **opts):
    """Independent equations A_i X_i + X_i A_i^T + L_i S_i L_i^T = 0 of uneven sizes solved
    concurrently (lyap_solve_batched).  Returns a list of (Z_i, D_i, info_i)."""
    count = len(As)
    if len(Ls) != count or (Ss is not None and len(Ss) != count):
        raise ValueError("As, Ls (and Ss) must have the same length")
    Ss = list(Ss) if Ss is not None else [None] * count
    dev = _dev(*As, *Ls, *[s for s in Ss if s is not None])
    As = [_rowmajor(a) for a in As]
    Ls = [_rowmajor(l) for l in Ls]
    Ss = [s.contiguous() if s is not None else None for s in Ss]
    ns = [a.shape[0] for a, _ in As]
    caps = list(z_caps) if z_caps is not None else ns
    device = As[0][0].device
    Zs = [torch.zeros((n, c), dtype=torch.float64, device=device) for n, c in zip(ns, caps)]
    Ds = [torch.zeros(c, dtype=torch.float64, device=device) for c in caps]
    IA = ctypes.c_int * count
    PA = ctypes.c_void_p * count
    o = _options(tol, refine, opts)
    prec = Precisions(*[DTYPES[p] for p in precisions])
    rank = IA()
    codes = IA()
    infos = (Info * count)()
    s_ptrs = PA(*[s.data_ptr() if s is not None else None for s in Ss])
    code = _lib.lib().lyap_solve_batched(
        _lib.handle(dev), _stream(dev), count, IA(*ns), IA(*[l.shape[1] for l, _ in Ls]),
        PA(*[a.data_ptr() for a, _ in As]), IA(*[ld for _, ld in As]),
        PA(*[l.data_ptr() for l, _ in Ls]), IA(*[ld for _, ld in Ls]),
        s_ptrs if any(s is not None for s in Ss) else None, prec, ctypes.byref(o),
        PA(*[z.data_ptr() for z in Zs]), IA(*caps), IA(*caps), PA(*[d.data_ptr() for d in Ds]),
        rank, infos, codes, int(workers), *_ws_args(ws))
    if code != 0 and raise_on_error and code not in (1, 2):
        _lib.check(code, "lyap_solve_batched")
    return [(Zs[i][:, :rank[i]], Ds[i][:rank[i]], infos[i].as_dict()) for i in range(count)]


def solve_adjoint(A, L, S=None, precisions=("fp16", "fp64", "fp64", "fp64"), tol=1e-13,
                  refine=True, z_cap=None, raise_on_error=True, ws=None, **opts):
    """The adjoint equation A^T Y + Y A + L S L^T = 0 (same method).  Replays the inverse
    sequence left in the workspace by an earlier solve on a matrix with the same contents
    (content fingerprint).  Returns (Z, D, info) with Y ~ Z diag(D) Z^T."""
    return _solve("lyap_solve_adjoint", A, L, S, precisions, tol, refine, z_cap, raise_on_error,
                  opts, ws=ws)


def trace_loss(C, Z, D):
    """tr(C X C^T) for X = Z diag(D) Z^T (library kernels; returns a Python float)."""
    dev = _dev(C, Z, D)
    C, ldc = _rowmajor(C)
    Z, ldz = _rowmajor(Z)
    D = D.contiguous()
    out = ctypes.c_double(0.0)
    code = _lib.lib().lyap_trace_loss(_lib.handle(dev), _stream(dev), Z.shape[0], C.shape[0],
                                      _ptr(C), ldc, Z.shape[1], _ptr(Z), ldz, _ptr(D),
                                      ctypes.byref(out))
    _lib.check(code, "lyap_trace_loss")
    return out.value


def trace_loss_grad(L, S, C, Z, D, ZY, DY, scale=1.0):
    """(dA, dL, dS, dC) of scale * tr(C X C^T) from the factors of X and of the adjoint
    solution Y (see lyap_trace_loss_grad in include/lyap.h); dS is None when S is None."""
    dev = _dev(L, S, C, Z, D, ZY, DY)
    L, ldl = _rowmajor(L)
    C, ldc = _rowmajor(C)
    Z, ldz = _rowmajor(Z)
    ZY, ldzy = _rowmajor(ZY)
    D, DY = D.contiguous(), DY.contiguous()
    if S is not None:
        S = S.contiguous()
    n, m = L.shape
    k = C.shape[0]
    opts = dict(dtype=torch.float64, device=L.device)
    dA = torch.empty((n, n), **opts)
    dL = torch.empty((n, m), **opts)
    dS = torch.empty(m, **opts) if S is not None else None
    dC = torch.empty((k, n), **opts)
    code = _lib.lib().lyap_trace_loss_grad(
        _lib.handle(dev), _stream(dev), n, m, k, _ptr(L), ldl, _ptr(S), _ptr(C), ldc,
        Z.shape[1], _ptr(Z), ldz, _ptr(D), ZY.shape[1], _ptr(ZY), ldzy, _ptr(DY),
        float(scale), _ptr(dA), n, _ptr(dL), m, _ptr(dS), _ptr(dC), n)
    _lib.check(code, "lyap_trace_loss_grad")
    return dA, dL, dS, dC


class LyapunovTraceLoss(torch.autograd.Function):
    """loss = tr(C X C^T) with A X + X A^T + L diag(S) L^T = 0, differentiable in A, L, S and C.

    The backward solves the adjoint equation A^T Y + Y A + C^T C = 0 with the same solver
    (replaying the forward's inverse sequence) and forms dA = 2 Y X, dL = 2 Y L diag(S),
    dS = diag(L^T Y L) and dC = 2 C X with the library's matrix-core products; Y and X stay
    factored except in the dense dA.  Usage:
    ``LyapunovTraceLoss.apply(A, L, S, C, precisions, tol)`` (S may be None: W = L L^T)."""

    @staticmethod
    def forward(ctx, A, L, S, C, precisions=("fp64", "fp64", "fp64", "fp64"), tol=1e-13):
        Z, D, info = solve(A, L, S, precisions=precisions, tol=tol)
        loss = trace_loss(C, Z, D)
        ctx.save_for_backward(A, L, C, Z, D, *([S] if S is not None else []))
        ctx.has_s = S is not None
        ctx.precisions, ctx.tol = precisions, tol
        ctx.info = info
        return torch.tensor(loss, dtype=A.dtype, device=A.device)

    @staticmethod
    def backward(ctx, g):
        saved = ctx.saved_tensors
        A, L, C, Z, D = saved[:5]
        S = saved[5] if ctx.has_s else None
        ZY, DY, info = solve_adjoint(A, C.t().contiguous(), None, precisions=ctx.precisions,
                                     tol=ctx.tol)
        ctx.adjoint_info = info
        dA, dL, dS, dC = trace_loss_grad(L, S, C, Z, D, ZY, DY, scale=float(g))
        return dA, dL, dS, dC, None, None


def lyapunov_trace_loss(A, L, S, C, precisions=("fp64", "fp64", "fp64", "fp64"), tol=1e-13):
    """tr(C X C^T) for the solution X of A X + X A^T + L diag(S) L^T = 0 (autograd-aware)."""
    return LyapunovTraceLoss.apply(A, L, S, C, precisions, tol)
