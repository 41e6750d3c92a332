"""ctypes binding of liblyap.so (argument marshalling only).

Every numerical step runs inside the HIP library; this module only turns torch tensors into
device pointers, sizes and the current HIP stream, and raises on a non-zero status.  The
library must have been built (``python -m paper_2510_02126_amd.build``); there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblyap.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "lyap.h")

DTYPES = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp16x2": 4}

STATUS = {
    0: "OK", 1: "NOT_CONVERGED", 2: "STAGNATED", 3: "NONFINITE", 4: "SINGULAR",
    5: "NOT_STABLE", 6: "CAPACITY", 7: "BADARG", 8: "HIP_ERROR", 9: "NO_MEMORY",
    10: "WORKSPACE", 11: "TOO_LARGE",
}


class LyapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class Precisions(ctypes.Structure):
    _fields_ = [("u_s", ctypes.c_int), ("u", ctypes.c_int), ("u_r", ctypes.c_int),
                ("u_c", ctypes.c_int)]


class Options(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("i_max", ctypes.c_int), ("k_max", ctypes.c_int),
                ("rho", ctypes.c_double), ("eta_r", ctypes.c_double), ("eta_s", ctypes.c_double),
                ("delta_off", ctypes.c_double), ("theta", ctypes.c_double),
                ("refine", ctypes.c_int), ("psd", ctypes.c_int), ("form", ctypes.c_int),
                ("scaling", ctypes.c_int), ("escalate", ctypes.c_int), ("reuse", ctypes.c_int),
                ("adaptive", ctypes.c_int), ("pivoting", ctypes.c_int),
                ("omega", ctypes.c_double), ("solver", ctypes.c_int),
                ("adi_shifts", ctypes.c_int), ("adi_max", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("res", ctypes.c_double), ("n_res", ctypes.c_int),
                ("res_hist", ctypes.c_double * 64), ("newton_total", ctypes.c_int),
                ("newton_max", ctypes.c_int), ("inversions", ctypes.c_int),
                ("refinements", ctypes.c_int), ("rank", ctypes.c_int), ("n_mu", ctypes.c_int),
                ("mus", ctypes.c_double * 64), ("onenorm", ctypes.c_double * 64),
                ("phase_ms", ctypes.c_double * 8), ("kern_ms", ctypes.c_double * 4),
                ("kern_work", ctypes.c_double * 4), ("kern_calls", ctypes.c_int * 4),
                ("u_s_final", ctypes.c_int), ("escalations", ctypes.c_int),
                ("cache_reused", ctypes.c_int), ("rbt_steps", ctypes.c_int),
                ("rbt_fallbacks", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {
            "status": STATUS.get(self.status, self.status),
            "res": self.res,
            "res_hist": list(self.res_hist[: self.n_res]),
            "newton_total": self.newton_total,
            "newton_max": self.newton_max,
            "inversions": self.inversions,
            "refinements": self.refinements,
            "rank": self.rank,
            "mus": list(self.mus[: self.n_mu]),
            "onenorm": list(self.onenorm[: self.n_mu]),
            "phase_ms": list(self.phase_ms),
            "kern_ms": list(self.kern_ms),
            "kern_work": list(self.kern_work),
            "kern_calls": list(self.kern_calls),
            "u_s_final": {v: k for k, v in DTYPES.items()}.get(self.u_s_final, self.u_s_final),
            "escalations": self.escalations,
            "cache_reused": bool(self.cache_reused),
            "rbt_steps": self.rbt_steps,
            "rbt_fallbacks": self.rbt_fallbacks,
        }


_LIB = None
_HANDLES: dict = {}

P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double

_SIGS = {
    "lyap_create": (I, [ctypes.POINTER(P), I]),
    "lyap_destroy": (I, [P]),
    "lyap_default_options": (None, [ctypes.POINTER(Options)]),
    "lyap_strerror": (ctypes.c_char_p, [I]),
    "lyap_version": (ctypes.c_char_p, []),
    "lyap_workspace_size": (I, [I, I, I, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]),
    "lyap_workspace_size_batched": (I, [I, P, P, I, ctypes.POINTER(Options), I,
                                        ctypes.POINTER(ctypes.c_size_t)]),
    "lyap_solve": (I, [P, P, I, I, P, I, P, I, P, I, Precisions, ctypes.POINTER(Options), P, I,
                       I, P, ctypes.POINTER(I), P, ctypes.c_size_t, ctypes.POINTER(Info)]),
    "lyap_solve_static": (I, [P, P, I, I, P, I, P, I, P, I, Precisions, ctypes.POINTER(Options),
                              P, I, I, P, ctypes.POINTER(I), ctypes.POINTER(Info)]),
    "lyap_refine": (I, [P, P, I, I, P, I, P, I, P, I, Precisions, ctypes.POINTER(Options), P, I,
                        P, I, P, I, I, P, ctypes.POINTER(I), P, ctypes.c_size_t,
                        ctypes.POINTER(Info)]),
    "lyap_solve_batched": (I, [P, P, I, P, P, P, P, P, P, P, Precisions, ctypes.POINTER(Options),
                               P, P, P, P, P, P, P, I, P, ctypes.c_size_t]),
    "lyap_trace_loss": (I, [P, P, I, I, P, I, I, P, I, P, ctypes.POINTER(D)]),
    "lyap_trace_loss_grad": (I, [P, P, I, I, I, P, I, P, P, I, I, P, I, P, I, P, I, P, D, P, I,
                                 P, I, P, P, I]),
    "lyap_solve_adjoint": (I, [P, P, I, I, P, I, P, I, P, I, Precisions, ctypes.POINTER(Options),
                               P, I, I, P, ctypes.POINTER(I), P, ctypes.c_size_t,
                               ctypes.POINTER(Info)]),
    "lyap_inverse": (I, [P, P, I, I, I, P, I, P, I]),
    "lyap_gemm": (I, [P, P, I, I, I, I, I, I, D, P, I, P, I, D, P, I]),
    "lyap_qr": (I, [P, P, I, I, P, I, P, I, P, I]),
    "lyap_qr_lead": (I, [P, P, I, I, I, P, I, P, I, P, I]),
    "lyap_syev": (I, [P, P, I, P, I, P, P, I]),
    "lyap_jacobi_schedule": (I, [I, P, P]),
}


def header_functions() -> list[str]:
    """Names of the functions declared in include/lyap.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lyap_[a-z_0-9]+)\s*\(", text)))


def lib():
    """Load liblyap.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2510_02126_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def check(code: int, what: str = ""):
    if code != 0:
        msg = lib().lyap_strerror(code).decode()
        raise LyapError(code, f"{what}: {msg}" if what else msg)


def handle(device: int):
    """Per-device library handle (created on first use, kept for the process)."""
    h = _HANDLES.get(device)
    if h is None:
        hp = P()
        check(lib().lyap_create(ctypes.byref(hp), device), "lyap_create")
        h = hp
        _HANDLES[device] = h
    return h


def default_options() -> Options:
    o = Options()
    lib().lyap_default_options(ctypes.byref(o))
    return o
