"""Thin ctypes binding of libfr.so (include/fr.h).

Argument marshalling only: every step of the residual, Jacobian and JVP runs
in the library's HIP kernels.  Device arrays are torch tensors on the GPU
(PyTorch provides the memory and the stream).  A missing library is an
error; there is no other code path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfr.so")

FR_F64, FR_F32, FR_BF16 = 0, 1, 2
_PREC = {"f64": FR_F64, "f32": FR_F32, "bf16": FR_BF16}
_STATUS = {0: "FR_OK", -1: "FR_E_INVALID", -2: "FR_E_UNSUPPORTED", -3: "FR_E_NOMEM", -4: "FR_E_DEVICE",
           -5: "FR_E_SINGULAR", -6: "FR_E_NOT_CONVERGED", -7: "FR_E_NONFINITE"}

EXPORTED = ["fr_ctx_create", "fr_ctx_destroy", "fr_ctx_info", "fr_last_error", "fr_ctx_sync", "fr_rhs", "fr_rhs_noalloc",
            "fr_jacobian_blocks", "fr_block_offsets", "fr_jvp", "fr_set_kernel_timing", "fr_kernel_time"]


class FrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Mesh(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n_elem", C.c_int64), ("degree", C.c_int32),
                ("elem_type", C.c_void_p), ("elem_xyz", C.c_void_p), ("max_vert", C.c_int32),
                ("nbr", C.c_void_p), ("nbr_face", C.c_void_p), ("max_face", C.c_int32),
                ("tri_sol_pts", C.c_void_p), ("tet_sol_pts", C.c_void_p)]


class _Phys(C.Structure):
    _fields_ = [("system", C.c_int32), ("nvars", C.c_int32), ("adv_vel", C.c_double * 3),
                ("gamma", C.c_double), ("mu", C.c_double), ("prandtl", C.c_double),
                ("ldg_beta", C.c_double), ("ldg_penalty", C.c_double), ("scheme", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("n_sol", C.c_int32), ("n_flux", C.c_int32), ("n_face", C.c_int32),
                ("nvars", C.c_int32), ("block_dim", C.c_int32), ("n_elem", C.c_int64), ("n_dof", C.c_int64),
                ("blocks_per_elem", C.c_int64), ("precision", C.c_int32)]


_lib = None


def lib():
    """Loads libfr.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2105_08632_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.fr_ctx_create.argtypes = [C.POINTER(_Mesh), C.POINTER(_Phys), C.c_int, P, C.POINTER(P)]
        L.fr_ctx_destroy.argtypes = [P]
        L.fr_ctx_info.argtypes = [P, C.POINTER(_Info)]
        L.fr_last_error.argtypes = [P]
        L.fr_last_error.restype = C.c_char_p
        L.fr_ctx_sync.argtypes = [P]
        L.fr_rhs.argtypes = [P, P, P]
        L.fr_rhs_noalloc.argtypes = [P, P, P]
        L.fr_jacobian_blocks.argtypes = [P, P, P, C.c_int]
        L.fr_block_offsets.argtypes = [P, P]
        L.fr_jvp.argtypes = [P, P, P, P, P]
        L.fr_set_kernel_timing.argtypes = [P, C.c_int]
        L.fr_kernel_time.argtypes = [P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        for name in EXPORTED:
            getattr(L, name).restype = C.c_int if name != "fr_last_error" else C.c_char_p
        _lib = L
        _extend(L)
    return _lib


_extensions = []


def _extend(L):
    for f in _extensions:
        f(L)


def _check(rc: int, ctx=None):
    if rc != 0:
        msg = lib().fr_last_error(ctx).decode()
        raise FrError(rc, msg)


def _ptr(t) -> int:
    return t.data_ptr()


class Context:
    """One mesh + physics + precision on one HIP stream."""

    def __init__(self, mesh, phys, precision: str = "f64", stream=None, tri_pts=None, tet_pts=None):
        import torch
        L = lib()
        self.mesh, self.phys = mesh, phys
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self._keep = [np.ascontiguousarray(mesh.elem_type, dtype=np.int8),
                      np.ascontiguousarray(mesh.xyz, dtype=np.float64),
                      np.ascontiguousarray(mesh.nbr, dtype=np.int64),
                      np.ascontiguousarray(mesh.nbr_face, dtype=np.int8)]
        tp = None if tri_pts is None else np.ascontiguousarray(tri_pts, dtype=np.float64)
        qp = None if tet_pts is None else np.ascontiguousarray(tet_pts, dtype=np.float64)
        self._keep += [tp, qp]
        m = _Mesh(mesh.ndim, mesh.n_elem, int(mesh.degree[0]),
                  self._keep[0].ctypes.data, self._keep[1].ctypes.data, mesh.max_vert,
                  self._keep[2].ctypes.data, self._keep[3].ctypes.data, mesh.max_face,
                  None if tp is None else tp.ctypes.data, None if qp is None else qp.ctypes.data)
        ph = _Phys(phys.system, phys.nvars, (C.c_double * 3)(*[float(x) for x in phys.adv_vel]),
                   phys.gamma, phys.mu, phys.prandtl, phys.beta, phys.eta, int(getattr(phys, "scheme", 0)))
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        rc = L.fr_ctx_create(C.byref(m), C.byref(ph), _PREC[precision], C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise FrError(rc, L.fr_last_error(None).decode())
        self.h = h
        info = _Info()
        _check(L.fr_ctx_info(h, C.byref(info)), h)
        self.info = info
        self.ns, self.nf, self.nface = info.n_sol, info.n_flux, info.n_face
        self.nv, self.b, self.ne, self.ndof = info.nvars, info.block_dim, info.n_elem, info.n_dof
        self.mixed = bool(np.any(self._keep[0] != self._keep[0][0]))
        off = np.zeros(self.ne + 1, dtype=np.int64)
        _check(L.fr_block_offsets(h, off.ctypes.data), h)
        self.block_offsets = off

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.fr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vec(self, x):
        if x.dtype != self.dtype or not x.is_cuda or not x.is_contiguous() or x.numel() != self.ndof:
            raise ValueError(f"expected a contiguous {self.dtype} CUDA tensor with {self.ndof} entries")
        return x

    def empty_state(self):
        import torch
        if self.mixed:      # element n's entries follow those of elements 0..n-1
            return torch.empty(self.ndof, dtype=self.dtype, device="cuda")
        return torch.empty(self.ne, self.ns, self.nv, dtype=self.dtype, device="cuda")

    def rhs(self, U, out=None):
        U = self._vec(U)
        out = self.empty_state() if out is None else self._vec(out)
        _check(lib().fr_rhs(self.h, _ptr(U), _ptr(out)), self.h)
        return out

    def rhs_noalloc(self, U, out):
        """fr_rhs_noalloc: the residual with its intermediates in the library's per-device scratch."""
        U, out = self._vec(U), self._vec(out)
        _check(lib().fr_rhs_noalloc(self.h, _ptr(U), _ptr(out)), self.h)
        return out

    def jvp(self, U, v, out=None, R_out=None):
        U, v = self._vec(U), self._vec(v)
        out = self.empty_state() if out is None else self._vec(out)
        Rp = None if R_out is None else _ptr(self._vec(R_out))
        _check(lib().fr_jvp(self.h, _ptr(U), _ptr(v), _ptr(out), Rp), self.h)
        return out

    def block_tensor(self, out_prec: str):
        import torch
        dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[out_prec]
        if self.mixed:      # packed blocks, element n's from block_offsets[n]
            return torch.empty(int(self.block_offsets[-1]), dtype=dt, device="cuda")
        return torch.empty(self.ne, 1 + self.nface, self.b, self.b, dtype=dt, device="cuda")

    def block(self, blocks, n: int, slot: int):
        """Block `slot` of element n (0: self, 1+f: the neighbour across face
        f) of a fr_jacobian_blocks array, as a [b_m, b_n] view (column-major
        block: index [c][r])."""
        if not self.mixed:
            return blocks[n, slot]
        p = int(self.mesh.degree[0])
        ns = {0: (p + 1) ** 2, 1: (p + 1) * (p + 2) // 2}
        et = self._keep[0]
        bn = ns[int(et[n])] * self.nv
        o = int(self.block_offsets[n])
        if slot == 0:
            return blocks[o:o + bn * bn].view(bn, bn)
        o += bn * bn
        for f in range(slot):
            m = int(self.mesh.nbr[n, f])
            bm = ns[int(et[m])] * self.nv
            if f == slot - 1:
                return blocks[o:o + bn * bm].view(bm, bn)
            o += bn * bm

    def jacobian_blocks(self, U, out=None, out_prec: str | None = None):
        """Blocks [n, slot, c, r] (each block column-major: index [c][r])."""
        U = self._vec(U)
        if out_prec is None:
            out_prec = self.precision
        if out is None:
            out = self.block_tensor(out_prec)
        _check(lib().fr_jacobian_blocks(self.h, _ptr(U), _ptr(out), _PREC[out_prec]), self.h)
        return out

    def sync(self):
        _check(lib().fr_ctx_sync(self.h), self.h)

    def set_kernel_timing(self, enable: bool = True):
        _check(lib().fr_set_kernel_timing(self.h, int(enable)), self.h)

    def kernel_time(self, which: int = 0):
        """(total ms, launches) of the timed kernel since the last query."""
        ms, n = C.c_double(), C.c_int64()
        _check(lib().fr_kernel_time(self.h, which, C.byref(ms), C.byref(n)), self.h)
        return ms.value, n.value


# ---------------------------------------------------------------- Fourier analysis
def _fourier_symbols(L):
    P = C.c_void_p
    L.fr_fourier_eigs.argtypes = [P, P, C.c_int64, P, C.c_int64, C.c_double, P]
    L.fr_cfl_max.argtypes = [P, P, C.c_int64, P, C.c_int, C.c_double, C.c_double, P]
    L.fr_fourier_eigs.restype = C.c_int
    L.fr_cfl_max.restype = C.c_int


_extensions.append(_fourier_symbols)
EXPORTED += ["fr_fourier_eigs", "fr_cfl_max"]


def _fourier_eigs(self, blocks, elem: int, kappa, scale: float = 1.0, out=None):
    """Eigenvalues of G(kappa) = scale sum_k B_k exp(i kappa . d_k) for each
    row of kappa ([nk, ndim] float64 CUDA tensor): complex tensor [nk, b]."""
    import torch
    kappa = kappa.to(torch.float64).contiguous()
    assert kappa.is_cuda and kappa.dim() == 2 and kappa.shape[1] == self.info.ndim
    nk = kappa.shape[0]
    out = torch.empty(nk, self.b, 2, dtype=torch.float64, device="cuda") if out is None else out
    _check(lib().fr_fourier_eigs(self.h, _ptr(blocks), elem, _ptr(kappa), nk, scale, _ptr(out)), self.h)
    return out


def _cfl_max(self, eigs, coef, tau_max: float = 4.0, tol: float = 1e-12) -> float:
    """Largest tau with |P(tau lambda)| <= 1 + tol for all eigenvalues (eigs:
    [.., 2] float64 CUDA tensor of (re, im) pairs), P(z) = sum_j coef[j] z^j."""
    import torch
    eigs = eigs.contiguous()
    c = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    out = torch.empty(1, dtype=torch.float64, device="cuda")
    _check(lib().fr_cfl_max(self.h, _ptr(eigs), eigs.numel() // 2, c.ctypes.data, len(c) - 1, tau_max, tol,
                            _ptr(out)), self.h)
    return float(out.item())


def _rk54_symbols(L):
    L.fr_rk54.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_int64]
    L.fr_rk54.restype = C.c_int


_extensions.append(_rk54_symbols)
EXPORTED += ["fr_rk54"]


def _rk54(self, U, dt: float, nsteps: int, work=None):
    """Advances U in place by nsteps RK54 steps; work: 2 n_dof scratch values."""
    import torch
    U = self._vec(U)
    work = torch.empty(2 * self.ndof, dtype=self.dtype, device="cuda") if work is None else work
    assert work.dtype == self.dtype and work.numel() >= 2 * self.ndof and work.is_contiguous()
    _check(lib().fr_rk54(self.h, _ptr(U), _ptr(work), dt, nsteps), self.h)
    return U


Context.rk54 = _rk54
Context.fourier_eigs = _fourier_eigs
Context.cfl_max = _cfl_max

# ---------------------------------------------------------------- implicit step
FR_PC_BLOCK_JACOBI, FR_PC_MLP = 0, 1


class _NewtonOpts(C.Structure):
    _fields_ = [("dt", C.c_double), ("newton_rtol", C.c_double), ("newton_maxit", C.c_int32),
                ("gmres_rtol", C.c_double), ("gmres_maxit", C.c_int32), ("pc_refresh", C.c_int32),
                ("use_graph", C.c_int32), ("gmres_augment", C.c_int32),
                ("gmres_stall", C.c_int32)]


class _NewtonStats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("gmres_iters", C.c_int32), ("pc_setups", C.c_int32),
                ("converged", C.c_int32), ("res0", C.c_double), ("res", C.c_double),
                ("last_linear_rel", C.c_double), ("ms", C.c_double),
                ("res_hist", C.c_double * 32), ("gmres_hist", C.c_int32 * 32), ("cycles", C.c_int32)]


def _solver_symbols(L):
    P = C.c_void_p
    L.fr_precond_create.argtypes = [P, C.c_int, C.POINTER(P)]
    L.fr_precond_setup.argtypes = [P, P, C.c_double, C.c_double]
    L.fr_apply_precond.argtypes = [P, P, P]
    L.fr_precond_destroy.argtypes = [P]
    L.fr_solver_create.argtypes = [P, C.c_int, C.POINTER(P)]
    L.fr_solver_destroy.argtypes = [P]
    L.fr_newton_step.argtypes = [P, P, P, P, C.POINTER(_NewtonOpts), C.POINTER(_NewtonStats)]
    for n in ("fr_precond_create", "fr_precond_setup", "fr_apply_precond", "fr_precond_destroy",
              "fr_solver_create", "fr_solver_destroy", "fr_newton_step"):
        getattr(L, n).restype = C.c_int


_extensions.append(_solver_symbols)
EXPORTED += ["fr_precond_create", "fr_precond_setup", "fr_apply_precond", "fr_precond_destroy",
             "fr_solver_create", "fr_solver_destroy", "fr_newton_step"]


class Precond:
    """Block preconditioner (block-Jacobi in FP64: explicit inverses up to
    b = 128, LU factors up to b = 320; or the learned MLP)."""

    def __init__(self, ctx: Context, kind: int = FR_PC_BLOCK_JACOBI):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().fr_precond_create(ctx.h, kind, C.byref(h)), ctx.h)
        self.h = h

    def setup(self, U, shift: float, scale: float):
        _check(lib().fr_precond_setup(self.h, _ptr(self.ctx._vec(U)), shift, scale), self.ctx.h)

    def apply(self, r, z=None):
        z = self.ctx.empty_state() if z is None else self.ctx._vec(z)
        _check(lib().fr_apply_precond(self.h, _ptr(self.ctx._vec(r)), _ptr(z)), self.ctx.h)
        return z

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.fr_precond_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Backward-Euler Newton-GMRES(restart) on an FP64 context."""

    def __init__(self, ctx: Context, restart: int = 30):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().fr_solver_create(ctx.h, restart, C.byref(h)), ctx.h)
        self.h = h

    def newton_step(self, Un, U=None, pc: Precond | None = None, dt: float = 1e-3, newton_rtol: float = 1e-8,
                    newton_maxit: int = 20, gmres_rtol: float = 1e-3, gmres_maxit: int = 300,
                    check: bool = True, pc_refresh: bool = False, use_graph: bool = False,
                    augment: int = 0, stall_cycles: int = 0) -> dict:
        """augment = k > 0 runs loose GMRES: each cycle's last k directions are
        the corrections of the k previous cycles (host-driven Arnoldi).
        stall_cycles: a linear solve stops when its true residual fell by less
        than 1% over this many restart cycles (0: 4)."""
        U = self.ctx.empty_state() if U is None else self.ctx._vec(U)
        o = _NewtonOpts(dt, newton_rtol, newton_maxit, gmres_rtol, gmres_maxit, int(pc_refresh), int(use_graph),
                        int(augment), int(stall_cycles))
        st = _NewtonStats()
        rc = lib().fr_newton_step(self.h, None if pc is None else pc.h, _ptr(self.ctx._vec(Un)), _ptr(U),
                                  C.byref(o), C.byref(st))
        if check:
            _check(rc, self.ctx.h)
        out = {k: getattr(st, k) for k, _ in _NewtonStats._fields_ if not k.endswith("_hist")}
        n = min(32, st.newton_iters + 1)
        out["res_hist"] = list(st.res_hist[:n])
        out["gmres_hist"] = list(st.gmres_hist[:n])
        out["status"] = rc
        out["U"] = U
        return out

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.fr_solver_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned preconditioner
def _mlp_symbols(L):
    P = C.c_void_p
    L.fr_mlp_create.argtypes = [C.c_int, C.c_int, C.c_uint64, C.c_int, P, C.POINTER(P)]
    L.fr_mlp_destroy.argtypes = [P]
    L.fr_mlp_last_error.argtypes = [P]
    L.fr_mlp_last_error.restype = C.c_char_p
    L.fr_mlp_info.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.fr_mlp_set_params.argtypes = [P, P]
    L.fr_mlp_get_params.argtypes = [P, P]
    L.fr_mlp_forward.argtypes = [P, P, C.c_int64, P]
    L.fr_mlp_loss_grad.argtypes = [P, P, C.c_int64, P, P, P]
    L.fr_mlp_train_step.argtypes = [P, P, C.c_int64, C.c_float, P]
    L.fr_precond_set_mlp.argtypes = [P, P, C.c_double]
    L.fr_precond_mlp_inputs.argtypes = [P, P, C.c_double, C.c_double, P, P]
    L.fr_precond_info.argtypes = [P, C.POINTER(C.c_int64)]
    L.fr_precond_set_refine.argtypes = [P, C.c_int, C.c_double, C.c_int]
    L.fr_precond_stats.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_double), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)]
    for n in ("fr_mlp_create", "fr_mlp_destroy", "fr_mlp_info", "fr_mlp_set_params", "fr_mlp_get_params",
              "fr_mlp_forward", "fr_mlp_loss_grad", "fr_mlp_train_step", "fr_precond_set_mlp",
              "fr_precond_mlp_inputs", "fr_precond_info", "fr_precond_set_refine", "fr_precond_stats"):
        getattr(L, n).restype = C.c_int


_extensions.append(_mlp_symbols)
EXPORTED += ["fr_mlp_create", "fr_mlp_destroy", "fr_mlp_last_error", "fr_mlp_info", "fr_mlp_set_params",
             "fr_mlp_get_params", "fr_mlp_forward", "fr_mlp_loss_grad", "fr_mlp_train_step", "fr_precond_set_mlp",
             "fr_precond_mlp_inputs", "fr_precond_info", "fr_precond_set_refine", "fr_precond_stats"]


def _mcheck(rc: int, h):
    if rc != 0:
        raise FrError(rc, lib().fr_mlp_last_error(h).decode())


class Mlp:
    """The learned block-inverse network (b^2 -> hidden -> hidden -> b^2)."""

    def __init__(self, b: int, hidden: int = 256, seed: int = 0, max_batch: int = 4096, stream=None):
        import torch
        self._torch = torch
        s = torch.cuda.current_stream() if stream is None else stream
        self.stream = s
        h = C.c_void_p()
        rc = lib().fr_mlp_create(b, hidden, seed, max_batch, s.cuda_stream, C.byref(h))
        if rc != 0:
            raise FrError(rc, f"fr_mlp_create(b={b}, hidden={hidden}, max_batch={max_batch})")
        self.h = h
        n = C.c_int64()
        lib().fr_mlp_info(h, C.byref(n), None, None, None)
        self.b, self.hidden, self.max_batch, self.n_params = b, hidden, max_batch, n.value
        self._loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def params(self):
        t = self._torch.empty(self.n_params, dtype=self._torch.float32, device="cuda")
        _mcheck(lib().fr_mlp_get_params(self.h, _ptr(t)), self.h)
        return t

    def set_params(self, p):
        p = p.to(self._torch.float32).contiguous()
        assert p.numel() == self.n_params and p.is_cuda
        _mcheck(lib().fr_mlp_set_params(self.h, _ptr(p)), self.h)

    def _x(self, X):
        assert X.dtype == self._torch.bfloat16 and X.is_cuda and X.is_contiguous()
        assert X.shape[-1] == self.b * self.b
        return X

    def forward(self, X, out=None):
        X = self._x(X)
        Y = self._torch.empty_like(X) if out is None else out
        _mcheck(lib().fr_mlp_forward(self.h, _ptr(X), X.shape[0], _ptr(Y)), self.h)
        return Y

    def loss_grad(self, X):
        X = self._x(X)
        g = self._torch.empty(self.n_params, dtype=self._torch.float32, device="cuda")
        res = self._torch.empty(X.shape[0], dtype=self._torch.float32, device="cuda")
        _mcheck(lib().fr_mlp_loss_grad(self.h, _ptr(X), X.shape[0], _ptr(self._loss), _ptr(g), _ptr(res)), self.h)
        return self._loss.clone(), g, res

    def train_step(self, X, lr: float):
        """One Adam step; returns the batch loss as a device tensor (no sync)."""
        X = self._x(X)
        loss = self._torch.empty(1, dtype=self._torch.float32, device="cuda")
        _mcheck(lib().fr_mlp_train_step(self.h, _ptr(X), X.shape[0], lr, _ptr(loss)), self.h)
        return loss

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.fr_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _precond_set_mlp(self, mlp: Mlp | None, theta: float):
    _check(lib().fr_precond_set_mlp(self.h, None if mlp is None else mlp.h, theta), self.ctx.h)
    self.mlp = mlp


def _precond_set_refine(self, max_iters: int, tol: float = 1e-2, start: str = "network"):
    """Newton-Schulz refinement after the network (start="network") or from
    the scaled transpose (start="transpose": the same without the network)."""
    _check(lib().fr_precond_set_refine(self.h, max_iters, tol, {"network": 0, "transpose": 1}[start]), self.ctx.h)


def _precond_stats(self) -> dict:
    nf, it, mr, xr = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
    _check(lib().fr_precond_stats(self.h, C.byref(nf), C.byref(it), C.byref(mr), C.byref(xr)), self.ctx.h)
    return {"n_fallback": nf.value, "mean_refine_iters": it.value, "mean_resid": mr.value, "max_resid": xr.value}


def _precond_mlp_inputs(self, U, shift: float, scale: float, X=None, s=None):
    import torch
    ne, b = self.ctx.ne, self.ctx.b
    X = torch.empty((ne, b * b), dtype=torch.bfloat16, device="cuda") if X is None else X
    s = torch.empty(ne, dtype=torch.float32, device="cuda") if s is None else s
    _check(lib().fr_precond_mlp_inputs(self.h, _ptr(self.ctx._vec(U)), shift, scale, _ptr(X), _ptr(s)), self.ctx.h)
    return X, s


def _precond_n_fallback(self) -> int:
    n = C.c_int64()
    _check(lib().fr_precond_info(self.h, C.byref(n)), self.ctx.h)
    return n.value


Precond.set_mlp = _precond_set_mlp
Precond.set_refine = _precond_set_refine
Precond.stats = _precond_stats
Precond.mlp_inputs = _precond_mlp_inputs
Precond.n_fallback = property(_precond_n_fallback)


# ---------------------------------------------------------------- batches of meshes
def _batch_symbols(L):
    P = C.c_void_p
    PP = C.POINTER(C.c_void_p)
    L.fr_batch_create.argtypes = [PP, C.c_int, C.POINTER(P)]
    L.fr_batch_destroy.argtypes = [P]
    L.fr_batch_last_error.argtypes = [P]
    L.fr_batch_last_error.restype = C.c_char_p
    L.fr_batch_rhs.argtypes = [P, PP, PP]
    L.fr_batch_jacobian_blocks.argtypes = [P, PP, PP]
    L.fr_batch_tune.argtypes = [P, PP, PP, PP, C.c_int]
    L.fr_batch_tuning.argtypes = [P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                  C.POINTER(C.c_int)]
    L.fr_batch_set_tuning.argtypes = [P, C.POINTER(C.c_int), C.c_int, C.c_int, C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]
    for n in ("fr_batch_create", "fr_batch_destroy", "fr_batch_rhs", "fr_batch_jacobian_blocks", "fr_batch_tune",
              "fr_batch_tuning", "fr_batch_set_tuning"):
        getattr(L, n).restype = C.c_int


_extensions.append(_batch_symbols)
EXPORTED += ["fr_batch_create", "fr_batch_destroy", "fr_batch_last_error", "fr_batch_rhs",
             "fr_batch_jacobian_blocks", "fr_batch_tune", "fr_batch_tuning", "fr_batch_set_tuning"]


def _ptrs(ts):
    return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


class Batch:
    """Many FP32 meshes evaluated together: one persistent launch per phase."""

    def __init__(self, ctxs):
        self.ctxs = list(ctxs)
        hs = (C.c_void_p * len(self.ctxs))(*[c.h.value for c in self.ctxs])
        h = C.c_void_p()
        rc = lib().fr_batch_create(hs, len(self.ctxs), C.byref(h))
        if rc != 0:
            msgs = [lib().fr_last_error(c.h).decode() for c in self.ctxs]
            raise FrError(rc, next((m for m in msgs if m), "fr_batch_create"))
        self.h = h

    def _check(self, rc):
        if rc != 0:
            raise FrError(rc, lib().fr_batch_last_error(self.h).decode())

    def rhs(self, Us, Rs=None):
        Us = [c._vec(u) for c, u in zip(self.ctxs, Us)]
        Rs = [c.empty_state() for c in self.ctxs] if Rs is None else Rs
        self._check(lib().fr_batch_rhs(self.h, _ptrs(Us), _ptrs(Rs)))
        return Rs

    def jacobian_blocks(self, Us, Bs=None):
        Us = [c._vec(u) for c, u in zip(self.ctxs, Us)]
        Bs = [c.block_tensor("f32") for c in self.ctxs] if Bs is None else Bs
        self._check(lib().fr_batch_jacobian_blocks(self.h, _ptrs(Us), _ptrs(Bs)))
        return Bs

    def tune(self, Us, reps: int = 3) -> dict:
        Us = [c._vec(u) for c, u in zip(self.ctxs, Us)]
        Rs = [c.empty_state() for c in self.ctxs]
        Bs = [c.block_tensor("f32") for c in self.ctxs]
        self._check(lib().fr_batch_tune(self.h, _ptrs(Us), _ptrs(Rs), _ptrs(Bs), reps))
        return self.tuning()

    def tuning(self) -> dict:
        gr, gj = C.c_int(), C.c_int()
        md = (C.c_int * 2)()
        kr, kj = (C.c_int * 32)(), (C.c_int * 32)()
        self._check(lib().fr_batch_tuning(self.h, md, C.byref(gr), C.byref(gj), kr, kj))
        codes = sorted({8 * int(t) + int(c.mesh.degree[0]) + (16 if c.mixed else 0)
                        for c in self.ctxs for t in set(c.mesh.elem_type.tolist())})
        name = {0: "quad", 1: "tri", 2: "mixed-quad", 3: "mixed-tri"}
        mode = {0: "mixed", 1: "grouped", 2: "grouped_mfma_quads"}
        return {"res_launch": mode[md[0]], "jac_launch": mode[md[1]], "grid_res": gr.value, "grid_jac": gj.value,
                "tiles_per_item": {f"{name[k // 8]}p{k % 8}": kr[k] for k in codes},
                "elems_per_item": {f"{name[k // 8]}p{k % 8}": kj[k] for k in codes}}

    def set_tuning(self, res_launch: str, jac_launch: str, grid_res: int, grid_jac: int, k_res: int = 1,
                   k_jac: int = 1):
        """Loads a table: launch strategies ("mixed" | "grouped", and for the
        Jacobian also "grouped_mfma_quads"), workgroups per launch, and one
        units-per-item value for every (type, degree)."""
        md = (C.c_int * 2)(*[{"mixed": 0, "grouped": 1, "grouped_mfma_quads": 2}[x] for x in (res_launch, jac_launch)])
        kr = (C.c_int * 32)(*([k_res] * 32))
        kj = (C.c_int * 32)(*([k_jac] * 32))
        self._check(lib().fr_batch_set_tuning(self.h, md, grid_res, grid_jac, kr, kj))

    def close(self):
        if getattr(self, "h", None) is not None and _lib is not None:
            _lib.fr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
