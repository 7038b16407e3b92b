"""The C-ABI library loads and exports every symbol include/fr.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2105_08632_amd import fr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"^\s*(?:fr_status|const char\*|void|int)\s+\**(fr_\w+)\s*\(", txt, re.M))
    return names


def test_header_declares_the_hot_calls():
    names = _declared()
    for hot in ("fr_rhs", "fr_jacobian_blocks", "fr_jvp", "fr_apply_precond", "fr_newton_step"):
        assert hot in names, hot


def test_library_exports_every_declared_symbol():
    if not os.path.exists(fr.LIB_PATH):
        pytest.skip("libfr.so not built")
    L = ctypes.CDLL(fr.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(L, n)]
    assert not missing, missing


def test_create_rejects_bad_mesh_without_gpu_work():
    """Argument validation happens on the host before any device call."""
    if not os.path.exists(fr.LIB_PATH):
        pytest.skip("libfr.so not built")
    L = fr.lib()
    h = ctypes.c_void_p()
    m = fr._Mesh(5, 1, 1, None, None, 4, None, None, 4, None)
    ph = fr._Phys(0, 1, (ctypes.c_double * 3)(1, 0, 0), 1.4, 0, 0.7, 0, 0)
    rc = L.fr_ctx_create(ctypes.byref(m), ctypes.byref(ph), 0, None, ctypes.byref(h))
    assert rc == -1
    assert b"ndim" in L.fr_last_error(None)
