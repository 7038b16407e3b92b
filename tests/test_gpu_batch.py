"""Batches of meshes (mixed triangles / quadrilaterals and degrees) in
persistent launches per phase: every mesh's residual, and its Jacobian
blocks wherever the batch runs the mesh's own kernels, are bitwise equal to
the same mesh evaluated alone, before and after the autotuner changes the
work decomposition; one small mesh is also checked against the FP64
oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_08632_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _meshes(system):
    spec = [("tri", 1, 4), ("quad", 2, 5), ("tri", 3, 3), ("quad", 4, 4), ("tri", 4, 3), ("quad", 1, 6),
            ("quad", 3, 4), ("tri", 2, 5)]
    out = []
    for i, (kind, p, n) in enumerate(spec):
        if kind == "tri":
            m, tp = I.tri_mesh(n, degree=p, jitter=0.05, K=1, seed=10 + i), I.tri_points(p)
        else:
            m, tp = I.quad_mesh(n, degree=p, jitter=0.05, K=1), None
        ph = I.euler_physics(2) if system == "euler" else I.ns_physics(2, 200.0, 0.72)
        # smooth random state (the isentropic vortex core is narrower than one element of these small meshes)
        U = I.ns2d_state(m, p, seeds=(20 + i, 30 + i, 40 + i), tri_pts=tp)
        out.append((m, p, tp, ph, U))
    return out


@pytest.mark.parametrize("system", ["euler", "ns"])
def test_batch_matches_meshes_alone(system):
    from paper_2105_08632_amd import fr
    cases = _meshes(system)
    ctxs = [fr.Context(m, ph, "f32", tri_pts=tp) for (m, p, tp, ph, U) in cases]
    Us = [torch.from_numpy(U).float().cuda().contiguous() for (m, p, tp, ph, U) in cases]
    alone_R = [c.rhs(u).clone() for c, u in zip(ctxs, Us)]
    alone_B = [c.jacobian_blocks(u, out_prec="f32").clone() for c, u in zip(ctxs, Us)]
    torch.cuda.synchronize()
    b = fr.Batch(ctxs)
    settings = [("mixed", "mixed", 1024, 512, 1, 1), ("grouped", "grouped", 64, 32, 3, 2),
                ("mixed", "grouped", 7, 5, 2, 3), ("grouped", "grouped_mfma_quads", 16, 0, 2, 1)]

    def check(tag):
        Rs = b.rhs(Us)
        Bs = b.jacobian_blocks(Us)
        torch.cuda.synchronize()
        jl = b.tuning()["jac_launch"]
        for i, (m, p, tp, ph, U) in enumerate(cases):
            assert torch.equal(Rs[i], alone_R[i]), (tag, i)
            if tp is not None or jl == "grouped_mfma_quads":
                # same kernels as the mesh alone: bitwise
                assert torch.equal(Bs[i], alone_B[i]), (tag, i, jl)
            else:
                # quadrilaterals in the persistent launches take the scalar
                # assembly bodies, alone the matrix-core path: FP32 parity
                err = float((Bs[i] - alone_B[i]).abs().max() / alone_B[i].abs().max())
                assert err <= 1e-5, (tag, i, jl, err)

    assert b.tuning()["jac_launch"] == "grouped_mfma_quads"    # the default
    check("default")
    for st in settings:
        b.set_tuning(*st)
        check(st)
    info = b.tune(Us, reps=1)
    assert info["grid_res"] >= 0 and info["grid_jac"] >= 0   # 0: one workgroup per item
    check("tuned")


def test_batch_mesh_against_oracle():
    """A quadrilateral and a triangle mesh inside a batch against the FP64
    oracle (FP32 bar 1e-5)."""
    from paper_2105_08632_amd import fr
    cases = _meshes("euler")[:2]
    ctxs = [fr.Context(m, ph, "f32", tri_pts=tp) for (m, p, tp, ph, U) in cases]
    Us = [torch.from_numpy(U).float().cuda().contiguous() for (m, p, tp, ph, U) in cases]
    b = fr.Batch(ctxs)
    Rs = b.rhs(Us)
    Bs = b.jacobian_blocks(Us)
    torch.cuda.synchronize()
    for i, (m, p, tp, ph, U) in enumerate(cases):
        Uq = Us[i].double().cpu().numpy()
        o = O.Oracle(m, ph, p, tp)
        Rr = o.rhs(Uq)
        R = Rs[i].double().cpu().numpy().reshape(-1)
        assert np.max(np.abs(R - Rr)) <= 1e-5 * np.max(np.abs(Rr))
        el = [0, m.n_elem - 1]
        Bo = o.jac_blocks(Uq, el, ctxs[i].b, ctxs[i].nface)
        Bn = Bs[i].double().cpu().numpy().transpose(0, 1, 3, 2)
        for j, e in enumerate(el):
            assert np.max(np.abs(Bn[e] - Bo[j])) <= 1e-5 * np.max(np.abs(Bo[j]))


def test_batch_rejects_mixed_systems():
    from paper_2105_08632_amd import fr
    (m1, p1, tp1, ph1, U1), = _meshes("euler")[:1]
    (m2, p2, tp2, ph2, U2), = _meshes("ns")[1:2]
    with pytest.raises(fr.FrError):
        fr.Batch([fr.Context(m1, ph1, "f32", tri_pts=tp1), fr.Context(m2, ph2, "f32", tri_pts=tp2)])


def _blocks_vs_oracle(ctx, o, Uq, B, m, elems, tol):
    """Every block of the listed elements (rectangular across triangle-quad
    faces) against the oracle's."""
    ns = {I.TRI: I.n_sol_points(I.TRI, int(m.degree[0])), I.QUAD: I.n_sol_points(I.QUAD, int(m.degree[0]))}
    for n in elems:
        nf = 3 if m.elem_type[n] == I.TRI else 4
        bn = ns[int(m.elem_type[n])] * ctx.nv
        s0 = None
        for slot in range(1 + nf):
            k = n if slot == 0 else int(m.nbr[n, slot - 1])
            bk = ns[int(m.elem_type[k])] * ctx.nv
            ref = o.jac_block(Uq, n, k, bn, bk)
            s0 = np.max(np.abs(ref)) if slot == 0 else s0
            got = ctx.block(B, n, slot).double().cpu().numpy().T
            assert np.max(np.abs(got - ref)) <= tol * s0, (n, slot)


def test_batch_with_mixed_meshes():
    """Meshes that mix triangles and quadrilaterals inside an Euler batch
    (with single-type meshes beside them): every launch strategy gives each
    mesh's residual and blocks bit for bit as the mesh alone, and one mixed
    mesh matches the FP64 oracle."""
    from paper_2105_08632_amd import fr
    ph = I.euler_physics(2)
    cases = []
    for i, (p, n, frac) in enumerate([(1, 6, 0.5), (3, 5, 0.3), (2, 4, 0.7), (4, 4, 0.5)]):
        m, tp = I.mixed_mesh(n, frac, degree=p, jitter=0.05, K=1, seed=50 + i), I.tri_points(p)
        cases.append((m, p, tp, I.ns2d_state(m, p, seeds=(60 + i, 70 + i, 80 + i), tri_pts=tp).reshape(-1)))
    for (m, p, tp, ph2, U) in _meshes("euler")[:3]:
        cases.append((m, p, tp, U.reshape(-1)))
    ctxs = [fr.Context(m, ph, "f32", tri_pts=tp) for (m, p, tp, U) in cases]
    Us = [torch.from_numpy(np.ascontiguousarray(U)).float().cuda() for (m, p, tp, U) in cases]
    alone_R = [c.rhs(u).clone() for c, u in zip(ctxs, Us)]
    alone_B = [c.jacobian_blocks(u, out_prec="f32").clone() for c, u in zip(ctxs, Us)]
    torch.cuda.synchronize()
    b = fr.Batch(ctxs)
    settings = [("mixed", "mixed", 1024, 512, 1, 1), ("grouped", "grouped", 64, 32, 3, 2),
                ("mixed", "grouped", 7, 5, 2, 3), ("grouped", "grouped_mfma_quads", 16, 0, 2, 1)]

    def check(tag):
        Rs = b.rhs(Us)
        Bs = b.jacobian_blocks(Us)
        torch.cuda.synchronize()
        jl = b.tuning()["jac_launch"]
        for i, c in enumerate(ctxs):
            assert torch.equal(Rs[i].reshape(-1), alone_R[i].reshape(-1)), (tag, i)
            if c.mixed or cases[i][2] is not None or jl == "grouped_mfma_quads":
                assert torch.equal(Bs[i], alone_B[i]), (tag, i, jl)
            else:
                err = float((Bs[i] - alone_B[i]).abs().max() / alone_B[i].abs().max())
                assert err <= 1e-5, (tag, i, jl, err)
        return Rs, Bs

    Rs, Bs = check("default")
    m, p, tp, U = cases[1]
    Uq = Us[1].double().cpu().numpy()
    o = O.Oracle(m, ph, p, tp)
    Rr = o.rhs(Uq)
    assert np.max(np.abs(Rs[1].double().cpu().numpy() - Rr)) <= 1e-5 * np.max(np.abs(Rr))
    _blocks_vs_oracle(ctxs[1], o, Uq, Bs[1], m, [0, m.n_elem - 1], 1e-5)
    for st in settings:
        b.set_tuning(*st)
        check(st)
    b.tune(Us, reps=1)
    check("tuned")


def test_batch_refuses_viscous_mixed_meshes():
    from paper_2105_08632_amd import fr
    m, tp = I.mixed_mesh(4, 0.5, degree=2, jitter=0.05, K=1, seed=3), I.tri_points(2)
    ctx = fr.Context(m, I.ns_physics(2, 200.0, 0.72), "f32", tri_pts=tp)
    with pytest.raises(fr.FrError) as ei:
        fr.Batch([ctx])
    assert ei.value.status == -2


def test_cfg3_full_size_batch():
    """The 64-mesh Euler workload (about 185k elements; every mesh mixes
    triangles and quadrilaterals, degrees 1-4) as one batch, default and
    autotuned: every mesh's residual and Jacobian blocks equal the mesh alone
    bit for bit; the first mesh is also checked against the FP64 oracle on
    sampled elements, one triangle and one quadrilateral (FP32 bar 1e-5)."""
    from paper_2105_08632_amd import fr
    meshes = I.mixed_batch()
    ph = I.euler_physics(2)
    ctxs = [fr.Context(m, ph, "f32", tri_pts=tp) for (m, p, tp, U) in meshes]
    Us = [torch.from_numpy(U).float().cuda().contiguous() for (m, p, tp, U) in meshes]
    assert sum(c.ne for c in ctxs) > 100000 and all(c.mixed for c in ctxs)
    b = fr.Batch(ctxs)

    def check(tag):
        Rs = b.rhs(Us)
        Bs = b.jacobian_blocks(Us)
        torch.cuda.synchronize()
        for i, (c, u) in enumerate(zip(ctxs, Us)):
            assert torch.equal(Rs[i], c.rhs(u)), (tag, i)
            Ba = c.jacobian_blocks(u)
            assert torch.equal(Bs[i], Ba), (tag, i)
            del Ba
        return Rs, Bs

    Rs, Bs = check("default")
    m, p, tp, U = meshes[0]
    Uq = Us[0].double().cpu().numpy()
    o = O.Oracle(m, ph, p, tp)
    Rr = o.rhs(Uq)
    assert np.max(np.abs(Rs[0].double().cpu().numpy() - Rr)) <= 1e-5 * np.max(np.abs(Rr))
    _blocks_vs_oracle(ctxs[0], o, Uq, Bs[0], m, [0, m.n_elem - 1], 1e-5)
    del Rs, Bs
    b.tune(Us, reps=1)
    check("tuned")
