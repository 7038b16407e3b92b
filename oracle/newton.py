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
