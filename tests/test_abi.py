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


def test_create_refuses_non_br1_without_gpu_work():
    """ldg_beta / ldg_penalty other than 0 are refused on the host (BR1 only)."""
    if not os.path.exists(fr.LIB_PATH):
        pytest.skip("libfr.so not built")
    import numpy as np
    from paper_2105_08632_amd import inputs as I
    L = fr.lib()
    m = I.quad_mesh(4, degree=2)
    keep = [np.ascontiguousarray(m.elem_type, dtype=np.int8), np.ascontiguousarray(m.xyz),
            np.ascontiguousarray(m.nbr, dtype=np.int64), np.ascontiguousarray(m.nbr_face, dtype=np.int8)]
    md = fr._Mesh(2, m.n_elem, 2, keep[0].ctypes.data, keep[1].ctypes.data, m.max_vert,
                  keep[2].ctypes.data, keep[3].ctypes.data, m.max_face, None)
    for beta, eta in ((0.5, 0.0), (0.0, 0.1)):
        ph = fr._Phys(2, 4, (ctypes.c_double * 3)(0, 0, 0), 1.4, 0.01, 0.72, beta, eta)
        h = ctypes.c_void_p()
        rc = L.fr_ctx_create(ctypes.byref(md), ctypes.byref(ph), 0, None, ctypes.byref(h))
        assert rc == -2
        assert b"BR1" in L.fr_last_error(None)


def test_create_refuses_ungrouped_mixed_mesh_without_gpu_work():
    """A mesh that mixes triangles and quadrilaterals must list them grouped
    by type; an interleaved order is refused on the host."""
    if not os.path.exists(fr.LIB_PATH):
        pytest.skip("libfr.so not built")
    import numpy as np
    from paper_2105_08632_amd import inputs as I
    L = fr.lib()
    m = I.mixed_mesh(4, 0.5, degree=1, seed=1)
    perm = np.argsort(np.arange(m.n_elem) % 2, kind="stable")       # interleave the two groups
    inv = np.empty_like(perm)
    inv[perm] = np.arange(m.n_elem)
    et = np.ascontiguousarray(m.elem_type[perm])
    assert np.any(np.diff(et.astype(int)) > 0) and np.any(np.diff(et.astype(int)) < 0)
    nbr = np.where(m.nbr[perm] >= 0, inv[np.maximum(m.nbr[perm], 0)], -1).astype(np.int64)
    keep = [et, np.ascontiguousarray(m.xyz[perm]), np.ascontiguousarray(nbr),
            np.ascontiguousarray(m.nbr_face[perm], dtype=np.int8), np.ascontiguousarray(I.tri_points(1))]
    md = fr._Mesh(2, m.n_elem, 1, keep[0].ctypes.data, keep[1].ctypes.data, m.max_vert,
                  keep[2].ctypes.data, keep[3].ctypes.data, m.max_face, keep[4].ctypes.data)
    ph = fr._Phys(1, 4, (ctypes.c_double * 3)(0, 0, 0), 1.4, 0.0, 0.72, 0.0, 0.0, 0)
    h = ctypes.c_void_p()
    rc = L.fr_ctx_create(ctypes.byref(md), ctypes.byref(ph), 0, None, ctypes.byref(h))
    assert rc == -1
    assert b"grouped by type" in L.fr_last_error(None)


def test_create_tetrahedra_need_their_points_without_gpu_work():
    """Tetrahedra without tet_sol_pts are refused on the host."""
    if not os.path.exists(fr.LIB_PATH):
        pytest.skip("libfr.so not built")
    import numpy as np
    from paper_2105_08632_amd import inputs as I
    L = fr.lib()
    m = I.tet_mesh(3, degree=2)
    keep = [np.ascontiguousarray(m.elem_type, dtype=np.int8), np.ascontiguousarray(m.xyz),
            np.ascontiguousarray(m.nbr, dtype=np.int64), np.ascontiguousarray(m.nbr_face, dtype=np.int8),
            np.ascontiguousarray(I.tri_points(2))]
    md = fr._Mesh(3, m.n_elem, 2, keep[0].ctypes.data, keep[1].ctypes.data, m.max_vert,
                  keep[2].ctypes.data, keep[3].ctypes.data, m.max_face, keep[4].ctypes.data, None)
    ph = fr._Phys(1, 5, (ctypes.c_double * 3)(0, 0, 0), 1.4, 0.0, 0.72, 0.0, 0.0, 0)
    h = ctypes.c_void_p()
    rc = L.fr_ctx_create(ctypes.byref(md), ctypes.byref(ph), 0, None, ctypes.byref(h))
    assert rc == -1
    assert b"tet_sol_pts" in L.fr_last_error(None)
