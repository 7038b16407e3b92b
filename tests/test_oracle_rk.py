"""The oracle's RK54 integrator against the paper: one step of the published
two-register coefficients applied to y' = z y must give the amplification
polynomial the paper prints for RK54 (temporal stability section, eq.
"rk_exponential": the exponential's fourth-order truncation plus z^5/200),
and the integrator is fourth-order accurate on a linear system."""
import numpy as np

from oracle import timestep as T


def test_amplification_polynomial_is_the_papers_rk54():
    c = T.amplification_coefficients()
    ref = np.array([1.0, 1.0, 1 / 2, 1 / 6, 1 / 24, 1 / 200])
    assert c.shape == ref.shape
    assert np.max(np.abs(c - ref)) <= 1e-14


def test_fourth_order_on_a_rotation():
    # y' = A y, A = [[0, -1], [1, -0.1]]: exact solution by the matrix exponential
    A = np.array([[0.0, -1.0], [1.0, -0.1]])
    w, V = np.linalg.eig(A)
    y0 = np.array([1.0, 0.0])
    t = 2.0
    exact = (V @ np.diag(np.exp(w * t)) @ np.linalg.solve(V, y0)).real
    errs = []
    for n in (20, 40, 80):
        errs.append(np.linalg.norm(T.rk54(lambda y: A @ y, y0, t / n, n) - exact))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 4.0) < 0.3), orders
