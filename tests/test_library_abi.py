"""The C-ABI library loads and exports every function include/lyap.h declares (no GPU)."""
import ctypes
import os

import pytest

from paper_2510_02126_amd import _lib


def test_library_built():
    assert os.path.exists(_lib.LIB_PATH), "run python -m paper_2510_02126_amd.build first"


def test_every_declared_symbol_is_exported():
    names = _lib.header_functions()
    assert "lyap_solve" in names and "lyap_inverse" in names
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    assert set(_lib.header_functions()) == set(_lib._SIGS)


def test_host_only_calls():
    L = _lib.lib()
    assert b"gfx950" in L.lyap_version()
    for code in range(10):
        assert len(L.lyap_strerror(code)) > 0
    o = _lib.default_options()
    assert o.tol == 1e-13 and o.i_max == 50 and o.k_max == 50
    assert o.rho == pytest.approx(0.1) and o.eta_r == pytest.approx(1e-4)
    assert o.theta == pytest.approx(0.9) and o.delta_off == pytest.approx(1e-2)
    # a NULL handle is rejected before any device work
    assert L.lyap_destroy(None) == 0
    assert L.lyap_inverse(None, None, 0, 1, 4, None, 4, None, 4) == 7


def test_struct_layouts_match_header(tmp_path):
    # compile a tiny host program against include/lyap.h and compare sizes and field offsets
    # with the ctypes structures of the binding
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = tmp_path / "layout.c"
    fields = {"lyap_info": [f for f, _ in _lib.Info._fields_],
              "lyap_options": [f for f, _ in _lib.Options._fields_],
              "lyap_precisions": [f for f, _ in _lib.Precisions._fields_]}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lyap.h"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'  printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(root, "include"), str(src), "-o",
                    str(exe)], check=True)
    out = dict(l.rsplit(" ", 1) for l in
               subprocess.run([str(exe)], check=True, capture_output=True, text=True)
               .stdout.split("\n") if l)
    for st, cls in (("lyap_info", _lib.Info), ("lyap_options", _lib.Options),
                    ("lyap_precisions", _lib.Precisions)):
        assert int(out[st]) == ctypes.sizeof(cls), st
        for f, _ in cls._fields_:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)


def test_workspace_size_is_host_only():
    # lyap_workspace_size needs no handle and no GPU
    L = _lib.lib()
    out = ctypes.c_size_t(0)
    o = _lib.default_options()
    assert L.lyap_workspace_size(4096, 8, 1, ctypes.byref(o), ctypes.byref(out)) == 0
    fp32 = out.value
    # k_max cached binary32 inverses of 4096 x 4096 are part of it
    assert fp32 > o.k_max * 4096 * 4096 * 4
    o.escalate = 1
    assert L.lyap_workspace_size(4096, 8, 1, ctypes.byref(o), ctypes.byref(out)) == 0
    assert out.value > fp32
    for bad in ((0, 1, 0), (4097, 8, 0), (16, 17, 0), (16, 2, 9)):
        assert L.lyap_workspace_size(*bad, None, ctypes.byref(out)) == 7
    ns = (ctypes.c_int * 3)(100, 512, 64)
    ms = (ctypes.c_int * 3)(1, 8, 2)
    assert L.lyap_workspace_size_batched(3, ns, ms, 2, None, 2, ctypes.byref(out)) == 0
    one = ctypes.c_size_t(0)
    assert L.lyap_workspace_size(512, 8, 2, None, ctypes.byref(one)) == 0
    assert out.value >= 2 * one.value
