"""ctypes wrapper of the FP64 CPU oracle (fr_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the library's compute path.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fr_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain -O2, OpenMP over elements)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(_LIB)
            P = C.c_void_p
            d = C.c_double
            i64 = C.c_int64
            L.oracle_create.argtypes = [C.c_int, i64, P, C.c_int, P, C.c_int, P, P, C.c_int,
                                        C.c_int, C.c_int, P, d, d, d, d, d, C.c_int, P, P, C.POINTER(C.c_void_p)]
            L.oracle_create.restype = C.c_int
            L.oracle_destroy.argtypes = [P]
            L.oracle_ndof.argtypes = [P]
            L.oracle_ndof.restype = i64
            L.oracle_rhs.argtypes = [P, P, P]
            L.oracle_jvp.argtypes = [P, P, P, P]
            L.oracle_jac_block.argtypes = [P, P, i64, i64, P]
            L.oracle_jac_blocks.argtypes = [P, P, P, i64, P, i64]
            L.oracle_jac_full.argtypes = [P, P, P]
            L.oracle_elem_geom.argtypes = [P, i64, P, P, P, P, P]
            L.oracle_elem_geom.restype = C.c_int
            L.oracle_ref.argtypes = [P, C.c_int, P, P, P, P, P, P, P, P, P]
            L.oracle_ref.restype = C.c_int
            L.oracle_ref1d.argtypes = [C.c_int] + [P] * 7
            L.oracle_flux.argtypes = [C.c_int, C.c_int, C.c_int, P, d, d, d, P, P, P]
            L.oracle_common_flux.argtypes = [C.c_int, C.c_int, C.c_int, P, d, d, d, d, d, P, P, P, P, P, P]
            L.oracle_lu_solve.argtypes = [C.c_int, P, P, P]
            L.oracle_lu_solve.restype = C.c_int
            _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class Oracle:
    """FP64 reference for one mesh + physics (single polynomial degree)."""

    def __init__(self, mesh, phys, p: int, tri_pts: np.ndarray | None = None, tet_pts: np.ndarray | None = None):
        L = lib()
        self.mesh, self.phys, self.p = mesh, phys, p
        self._keep = []
        et = np.ascontiguousarray(mesh.elem_type, dtype=np.int8)
        xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        nbr = np.ascontiguousarray(mesh.nbr, dtype=np.int64)
        nbf = np.ascontiguousarray(mesh.nbr_face, dtype=np.int8)
        c = np.ascontiguousarray(np.asarray(phys.adv_vel, dtype=np.float64).reshape(3))
        tp = None if tri_pts is None else np.ascontiguousarray(tri_pts, dtype=np.float64)
        qp = None if tet_pts is None else np.ascontiguousarray(tet_pts, dtype=np.float64)
        self._keep += [et, xyz, nbr, nbf, c, tp, qp]
        h = C.c_void_p()
        rc = L.oracle_create(mesh.ndim, mesh.n_elem, _p(et), p, _p(xyz), mesh.max_vert, _p(nbr), _p(nbf),
                             mesh.max_face, phys.system, phys.nvars, _p(c), phys.gamma, phys.mu,
                             phys.prandtl, phys.beta, phys.eta, int(getattr(phys, "scheme", 0)),
                             None if tp is None else _p(tp), None if qp is None else _p(qp), C.byref(h))
        if rc != 0:
            raise RuntimeError(f"oracle_create failed ({rc})")
        self.h = h
        self.ndof = int(L.oracle_ndof(h))

    def __del__(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.oracle_destroy(self.h)
            self.h = None

    @staticmethod
    def _vec(U):
        return np.ascontiguousarray(np.asarray(U, dtype=np.float64).reshape(-1))

    def rhs(self, U) -> np.ndarray:
        U = self._vec(U)
        R = np.zeros_like(U)
        lib().oracle_rhs(self.h, _p(U), _p(R))
        return R

    def jvp(self, U, v) -> np.ndarray:
        U, v = self._vec(U), self._vec(v)
        out = np.zeros_like(U)
        lib().oracle_jvp(self.h, _p(U), _p(v), _p(out))
        return out

    def jac_block(self, U, n: int, k: int, bn: int, bk: int) -> np.ndarray:
        """dR_n/dU_k, [bn, bk] row-major."""
        U = self._vec(U)
        out = np.zeros((bn, bk))
        lib().oracle_jac_block(self.h, _p(U), n, k, _p(out))
        return out

    def jac_blocks(self, U, elems, b: int, nface: int) -> np.ndarray:
        """[len(elems), 1+nface, b, b]: self block then one per local face."""
        U = self._vec(U)
        el = np.ascontiguousarray(np.asarray(elems, dtype=np.int64))
        out = np.zeros((len(el), 1 + nface, b, b))
        lib().oracle_jac_blocks(self.h, _p(U), _p(el), len(el), _p(out), (1 + nface) * b * b)
        return out

    def jac_full(self, U) -> np.ndarray:
        U = self._vec(U)
        out = np.zeros((self.ndof, self.ndof))
        lib().oracle_jac_full(self.h, _p(U), _p(out))
        return out

    def elem_geom(self, e: int, ns: int, nf: int):
        nd = self.mesh.ndim
        detJ = np.zeros(ns)
        fx = np.zeros((nf, nd))
        N = np.zeros((nf, nd))
        pair = np.zeros(nf, dtype=np.int32)
        sx = np.zeros((ns, nd))
        lib().oracle_elem_geom(self.h, e, _p(detJ), _p(fx), _p(N), _p(pair), _p(sx))
        return dict(detJ=detJ, fx=fx, N=N, pair=pair, sx=sx)

    def ref(self, etype: int) -> dict:
        dims = np.zeros(4, dtype=np.int32)
        if lib().oracle_ref(self.h, etype, _p(dims), None, None, None, None, None, None, None, None) != 0:
            raise ValueError("element type not in mesh")
        ns, nf, nd, nface = (int(x) for x in dims)
        out = dict(sp=np.zeros((ns, nd)), fp=np.zeros((nf, nd)), nref=np.zeros((nf, nd)),
                   M0=np.zeros((nf, ns)), Dm=np.zeros((nd, ns, ns)), Cor=np.zeros((ns, nf)),
                   wq=np.zeros(ns), fface=np.zeros(nf, dtype=np.int32))
        lib().oracle_ref(self.h, etype, _p(dims), _p(out["sp"]), _p(out["fp"]), _p(out["nref"]),
                         _p(out["M0"]), _p(out["Dm"]), _p(out["Cor"]), _p(out["wq"]), _p(out["fface"]))
        out.update(ns=ns, nf=nf, nd=nd, nface=nface)
        return out


def ref1d(p: int) -> dict:
    n = p + 1
    o = dict(x=np.zeros(n), w=np.zeros(n), D=np.zeros((n, n)), lp=np.zeros(n), lm=np.zeros(n),
             hp=np.zeros(n), hm=np.zeros(n))
    lib().oracle_ref1d(p, *(_p(o[k]) for k in ("x", "w", "D", "lp", "lm", "hp", "hm")))
    return o


def flux(phys, nd: int, u, q=None) -> np.ndarray:
    u = np.ascontiguousarray(u, dtype=np.float64)
    q = np.zeros((nd, phys.nvars)) if q is None else np.ascontiguousarray(q, dtype=np.float64)
    c = np.ascontiguousarray(np.asarray(phys.adv_vel, dtype=np.float64).reshape(3))
    f = np.zeros((nd, phys.nvars))
    lib().oracle_flux(phys.system, nd, phys.nvars, _p(c), phys.gamma, phys.mu, phys.prandtl,
                      _p(u), _p(q), _p(f))
    return f


def common_flux(phys, nd: int, uL, uR, qL, qR, n) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(phys.adv_vel, dtype=np.float64).reshape(3))
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (uL, uR, qL, qR, n)]
    F = np.zeros(phys.nvars)
    lib().oracle_common_flux(phys.system, nd, phys.nvars, _p(c), phys.gamma, phys.mu, phys.prandtl,
                             phys.beta, phys.eta, *(_p(a) for a in arrs), _p(F))
    return F


def lu_solve(A, b) -> np.ndarray:
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    if lib().oracle_lu_solve(A.shape[0], _p(A), _p(b), _p(x)) != 0:
        raise np.linalg.LinAlgError("singular")
    return x
