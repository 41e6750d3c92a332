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
