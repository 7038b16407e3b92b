"""Pins of the oracle on triangles (CPU): the builder-chosen solution points
(symmetric, unisolvent), free-stream preservation and discrete conservation
on jittered affine triangles, linearity and the stencil of the Jacobian
(self + 3 face neighbours for Euler; two layers for BR1)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_08632_amd import inputs as I


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_tri_points_symmetric_and_unisolvent(p):
    pts = I.tri_points(p)
    assert len(pts) == I.n_sol_points(I.TRI, p)
    # barycentric coordinates: the set is invariant under their permutations
    lam = np.stack([-(pts[:, 0] + pts[:, 1]) / 2, (1 + pts[:, 0]) / 2, (1 + pts[:, 1]) / 2], axis=1)
    assert np.all(lam > 0)
    key = lambda a: set(map(tuple, np.round(a, 12)))
    for perm in ([1, 2, 0], [2, 0, 1], [0, 2, 1]):
        assert key(lam[:, perm]) == key(lam)
    # Vandermonde of the monomials x^a y^b, a + b <= p, is non-singular
    V = np.stack([pts[:, 0] ** a * pts[:, 1] ** b for a in range(p + 1) for b in range(p + 1 - a)], axis=1)
    assert np.linalg.cond(V) < 1e4


@pytest.mark.parametrize("system,p", [("euler", 2), ("ns", 2), ("adv", 3)])
def test_tri_free_stream(system, p):
    m = I.tri_mesh(4, degree=p, jitter=0.05, K=1, seed=3)
    ph = {"euler": I.euler_physics(2), "ns": I.ns_physics(2, 1000.0, 0.72),
          "adv": I.advection_physics((1.0, 0.5))}[system]
    o = O.Oracle(m, ph, p, I.tri_points(p))
    ns = I.n_sol_points(I.TRI, p)
    state = np.array([1.3]) if ph.nvars == 1 else I.conservative(np.array(1.2), np.array([0.3, -0.2]),
                                                                  np.array(17.0), 1.4)
    U = np.tile(state, (m.n_elem, ns, 1))
    assert np.max(np.abs(o.rhs(U))) < 1e-12 * np.max(np.abs(state)) * 20 / m.h


def test_tri_conservation_ns():
    p = 3
    m = I.tri_mesh(5, degree=p, jitter=0.05, K=1, seed=4)
    tp = I.tri_points(p)
    o = O.Oracle(m, I.ns_physics(2, 1000.0, 0.72), p, tp)
    U = I.ns2d_state(m, p, tri_pts=tp)
    ns = I.n_sol_points(I.TRI, p)
    R = o.rhs(U).reshape(m.n_elem, ns, 4)
    w = o.ref(I.TRI)["wq"]
    tot, sc = np.zeros(4), np.zeros(4)
    for e in range(m.n_elem):
        dj = o.elem_geom(e, ns, o.ref(I.TRI)["nf"])["detJ"]
        tot += np.einsum("r,ra->a", w * dj, R[e])
        sc += np.einsum("r,ra->a", w * dj, np.abs(R[e]))
    assert np.max(np.abs(tot) / sc) < 1e-13


def test_tri_advection_matches_dense_jacobian_and_sparsity():
    """Linear advection on triangles: R = J U with the complex-step Jacobian,
    and J is non-zero only on the self block and the three face neighbours."""
    p = 2
    m = I.tri_mesh(4, degree=p, jitter=0.05, K=1, seed=5)
    tp = I.tri_points(p)
    o = O.Oracle(m, I.advection_physics((1.0, 0.5)), p, tp)
    U = I.advection_state(m, p, seed=2, tri_pts=tp)
    J = o.jac_full(U)
    R = o.rhs(U)
    assert np.max(np.abs(J @ U.reshape(-1) - R)) < 1e-12 * np.max(np.abs(R))
    ns = I.n_sol_points(I.TRI, p)
    for e in range(m.n_elem):
        allowed = {e, *m.nbr[e]}
        for k in range(m.n_elem):
            blk = J[e * ns:(e + 1) * ns, k * ns:(k + 1) * ns]
            if k not in allowed:
                assert np.all(blk == 0.0)
