"""Pins of the oracle on conforming meshes that mix triangles and
quadrilaterals (CPU): free-stream preservation and discrete conservation on
jittered hybrid meshes, exactness for polynomial data under linear advection
on an affine hybrid mesh (FR-DG reproduces -c . grad u exactly when u is a
polynomial of degree p: the traces agree across every face, triangle-quad
faces included, so the upwind flux adds no correction), and the stencil and
linearity of the Jacobian with its rectangular triangle-quad blocks."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_08632_amd import inputs as I


def _elem_slices(m, p, nv):
    ns = {I.TRI: I.n_sol_points(I.TRI, p), I.QUAD: I.n_sol_points(I.QUAD, p)}
    off, out = 0, []
    for e in range(m.n_elem):
        k = ns[int(m.elem_type[e])] * nv
        out.append(slice(off, off + k))
        off += k
    return out


def test_mixed_mesh_is_grouped_and_conforming():
    m = I.mixed_mesh(6, 0.5, degree=2, jitter=0.05, seed=3)
    et = m.elem_type
    assert np.all(np.diff(et.astype(int)) <= 0)          # triangles first, then quadrilaterals
    assert set(et.tolist()) == {I.TRI, I.QUAD}
    for e in range(m.n_elem):
        nf = 3 if et[e] == I.TRI else 4
        for f in range(nf):
            k, f2 = int(m.nbr[e, f]), int(m.nbr_face[e, f])
            assert m.nbr[k, f2] == e and m.nbr_face[k, f2] == f
        if nf == 3:
            assert m.nbr[e, 3] == -1


@pytest.mark.parametrize("system,p", [("euler", 2), ("ns", 3), ("adv", 4)])
def test_mixed_free_stream(system, p):
    m = I.mixed_mesh(5, 0.5, degree=p, jitter=0.05, K=1, seed=3)
    ph = {"euler": I.euler_physics(2), "ns": I.ns_physics(2, 1000.0, 0.72),
          "adv": I.advection_physics((1.0, 0.5))}[system]
    o = O.Oracle(m, ph, p, I.tri_points(p))
    state = np.array([1.3]) if ph.nvars == 1 else I.conservative(np.array(1.2), np.array([0.3, -0.2]),
                                                                  np.array(17.0), 1.4)
    U = np.tile(state, o.ndof // ph.nvars)
    assert np.max(np.abs(o.rhs(U))) < 1e-12 * np.max(np.abs(state)) * 20 / m.h


def test_mixed_conservation_ns():
    p = 3
    m = I.mixed_mesh(6, 0.5, degree=p, jitter=0.05, K=1, seed=4)
    tp = I.tri_points(p)
    o = O.Oracle(m, I.ns_physics(2, 1000.0, 0.72), p, tp)
    U = I.ns2d_state(m, p, tri_pts=tp)
    R = o.rhs(U)
    sl = _elem_slices(m, p, 4)
    tot, sc = np.zeros(4), np.zeros(4)
    for e in range(m.n_elem):
        et = int(m.elem_type[e])
        ref = o.ref(et)
        dj = o.elem_geom(e, ref["ns"], ref["nf"])["detJ"]
        Re = R[sl[e]].reshape(ref["ns"], 4)
        tot += np.einsum("r,ra->a", ref["wq"] * dj, Re)
        sc += np.einsum("r,ra->a", ref["wq"] * dj, np.abs(Re))
    assert np.max(np.abs(tot) / sc) < 1e-13


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mixed_advection_exact_for_polynomials(p):
    """u = a random polynomial of degree p on an unjittered hybrid mesh: at
    every element away from the periodic seam R = -c . grad u exactly."""
    N = 6
    m = I.mixed_mesh(N, 0.5, degree=p, jitter=0.0, seed=11)
    c = np.array([1.0, 0.5])
    tp = I.tri_points(p)
    o = O.Oracle(m, I.advection_physics(tuple(c)), p, tp)
    x = I.sol_points_phys(m, p, tp)
    rng = np.random.default_rng(p)
    terms = [(a, b, rng.normal()) for a in range(p + 1) for b in range(p + 1 - a)]
    X, Y = x[:, 0], x[:, 1]
    u = sum(k * X ** a * Y ** b for a, b, k in terms)
    ux = sum(k * a * X ** max(a - 1, 0) * Y ** b for a, b, k in terms if a > 0)
    uy = sum(k * b * X ** a * Y ** max(b - 1, 0) for a, b, k in terms if b > 0)
    R = o.rhs(u)
    ref = -(c[0] * ux + c[1] * uy)
    sl = _elem_slices(m, p, 1)
    inner = [e for e in range(m.n_elem) if np.all((m.xyz[e] > 1e-12) & (m.xyz[e] < 1 - 1e-12))]
    assert len(inner) > m.n_elem // 4
    kinds = {int(m.elem_type[e]) for e in inner}
    assert kinds == {I.TRI, I.QUAD}
    # elements with a neighbour of the other type are among those checked
    assert any(any(m.elem_type[m.nbr[e, f]] != m.elem_type[e] for f in range(3 if m.elem_type[e] == I.TRI else 4))
               for e in inner)
    scale = np.max(np.abs(ref))
    for e in inner:
        assert np.max(np.abs(R[sl[e]] - ref[sl[e]])) < 1e-11 * scale, e
    # and a dropped correction or a wrong pairing would show at the seam too:
    # the residual there differs (the data jump across the periodic seam)
    seam = [e for e in range(m.n_elem) if e not in inner]
    assert max(np.max(np.abs(R[sl[e]] - ref[sl[e]])) for e in seam) > 1e-3 * scale


def test_mixed_advection_jacobian_stencil_and_linearity():
    """Linear advection on a hybrid mesh: R = J U with the complex-step
    Jacobian; J is non-zero only on the self block and the face neighbours
    (the upwind ones: the upwind flux ignores the downwind state), whose
    blocks are rectangular (b_n x b_m) across triangle-quad faces."""
    p = 2
    m = I.mixed_mesh(4, 0.5, degree=p, jitter=0.05, K=1, seed=5)
    tp = I.tri_points(p)
    o = O.Oracle(m, I.advection_physics((1.0, 0.5)), p, tp)
    U = I.advection_state(m, p, seed=2, tri_pts=tp).reshape(-1)
    J = o.jac_full(U)
    R = o.rhs(U)
    assert np.max(np.abs(J @ U - R)) < 1e-12 * np.max(np.abs(R))
    sl = _elem_slices(m, p, 1)
    mixed_pairs = 0
    for e in range(m.n_elem):
        nf = 3 if m.elem_type[e] == I.TRI else 4
        allowed = {e, *[int(k) for k in m.nbr[e, :nf]]}
        for k in range(m.n_elem):
            blk = J[sl[e], sl[k]]
            if k not in allowed:
                assert np.all(blk == 0.0)
            elif m.elem_type[k] != m.elem_type[e] and np.max(np.abs(blk)) > 0.0:
                mixed_pairs += 1          # upwind neighbours across triangle-quad faces
    assert mixed_pairs > 0
