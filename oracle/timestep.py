"""Explicit time integration for the oracle: the five-stage, fourth-order,
two-register Runge-Kutta scheme of Carpenter and Kennedy (1994), which the
paper uses for its linear advection-diffusion experiments; written from the
published scheme, stage by stage.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU leg,
never by the library's compute path.
"""
from __future__ import annotations

import numpy as np

# published coefficients of the (5,4) 2N-storage scheme: register update
# weights a_i and solution weights b_i
A = [0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
     -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0]
B = [1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
     1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
     2277821191437.0 / 14882151754819.0]


def rk54(rhs, U, dt: float, nsteps: int) -> np.ndarray:
    """nsteps steps of dU/dt = rhs(U): per stage, k <- a_i k + dt rhs(U),
    U <- U + b_i k."""
    U = np.array(U, dtype=np.float64, copy=True)
    k = np.zeros_like(U)
    for _ in range(nsteps):
        for a, b in zip(A, B):
            k = a * k + dt * rhs(U)
            U = U + b * k
    return U


def amplification_coefficients() -> np.ndarray:
    """Coefficients of the scheme's amplification polynomial P(z), from one
    step applied to y' = z y with z symbolic (polynomials in numpy)."""
    P = np.polynomial.Polynomial
    y, k = P([1.0]), P([0.0])
    z = P([0.0, 1.0])
    for a, b in zip(A, B):
        k = a * k + z * y
        y = y + b * k
    return y.coef
