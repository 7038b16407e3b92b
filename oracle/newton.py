"""Dense FP64 reference for the implicit step (test infrastructure only).

Backward Euler: find U with F(U) = U - Un - dt R(U) = 0.  Newton's method
written out: J_F = I - dt dR/dU (the oracle's dense Jacobian), each update
from a direct dense solve.  Small meshes only.
"""
import numpy as np


def backward_euler_dense(o, Un, dt, rtol=1e-10, maxit=20):
    Un = np.asarray(Un, dtype=np.float64).reshape(-1)
    U = Un.copy()
    F = U - Un - dt * o.rhs(U)
    f0 = np.linalg.norm(F)
    hist = [f0]
    for _ in range(maxit):
        if np.linalg.norm(F) <= rtol * f0:
            break
        A = np.eye(U.size) - dt * o.jac_full(U)
        U = U + np.linalg.solve(A, -F)
        F = U - Un - dt * o.rhs(U)
        hist.append(np.linalg.norm(F))
    return U, hist


def newton_gmres(o, Un, dt, nvar_block, rtol=1e-8, forcing=1e-3, restart=30, maxit=3000, newton_maxit=12,
                 precond_blocks=None):
    """Backward Euler by Newton-GMRES(m), plainly: F(U) = U - Un - dt R(U);
    each Newton update solves J_F d = -F to the forcing tolerance by
    restarted GMRES with right preconditioning (modified Gram-Schmidt
    Arnoldi, the small least-squares problem by numpy), J_F v = v - dt
    (dR/dU) v from the oracle's complex-step JVP.  The preconditioner is
    block Jacobi: the inverses of A_n = I - dt J_nn at Un (precond_blocks:
    the oracle's self blocks J_nn, [ne][b][b]; none: unpreconditioned).
    No line search (a full Newton step).  Returns U, the residual history
    and the GMRES iteration count.  For the CPU timing beside the GPU's
    Newton step, not for large meshes."""
    Un = np.asarray(Un, dtype=np.float64).reshape(-1)
    U = Un.copy()
    b = nvar_block
    ne = U.size // b
    if precond_blocks is not None:
        Minv = np.linalg.inv(np.eye(b)[None] - dt * np.asarray(precond_blocks))

        def M(x):
            return np.einsum("nrc,nc->nr", Minv, x.reshape(ne, b)).reshape(-1)
    else:
        def M(x):
            return x
    F = U - Un - dt * o.rhs(U)
    f0 = np.linalg.norm(F)
    hist = [f0]
    its = 0
    for _ in range(newton_maxit):
        if np.linalg.norm(F) <= rtol * f0:
            break

        def A(v, U=U):
            return v - dt * o.jvp(U, v)
        rhs = -F
        bn = np.linalg.norm(rhs)
        d = np.zeros_like(U)
        r = rhs.copy()
        while its < maxit:
            beta = np.linalg.norm(r)
            if beta <= forcing * bn:
                break
            V = [r / beta]
            H = np.zeros((restart + 1, restart))
            Z = []
            k = 0
            for k in range(restart):
                z = M(V[k])
                Z.append(z)
                w = A(z)
                for i in range(k + 1):
                    H[i, k] = np.dot(w, V[i])
                    w = w - H[i, k] * V[i]
                H[k + 1, k] = np.linalg.norm(w)
                its += 1
                e1 = np.zeros(k + 2)
                e1[0] = beta
                y = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)[0]
                res = np.linalg.norm(e1 - H[:k + 2, :k + 1] @ y)
                if res <= forcing * bn or H[k + 1, k] == 0.0 or its >= maxit:
                    break
                V.append(w / H[k + 1, k])
            d = d + np.array(Z[:len(y)]).T @ y
            r = rhs - A(d)
        U = U + d
        F = U - Un - dt * o.rhs(U)
        hist.append(np.linalg.norm(F))
    return U, hist, its
