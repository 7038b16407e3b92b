"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Error metric: normwise relative, max|x - x_ref| / max|x_ref| per array, the
oracle evaluated on exactly the inputs the GPU saw (states rounded to the
device precision first).  Bars: 1e-12 (FP64), 1e-5 (FP32), 2e-2 (BF16).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_08632_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-2}


def _ctx(m, ph, prec, tri_pts=None):
    from paper_2105_08632_amd import fr
    return fr.Context(m, ph, prec, tri_pts=tri_pts)


def rel(x, ref):
    x = np.asarray(x, dtype=np.float64)
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


def _dev(a, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(dt).cuda().contiguous()


def _blocks_rowmajor(B):
    """[n, slot, c, r] (column-major blocks) -> numpy [n, slot, r, c] fp64."""
    return B.float().double().cpu().numpy().transpose(0, 1, 3, 2) if B.dtype == torch.bfloat16 else \
        B.double().cpu().numpy().transpose(0, 1, 3, 2)


def check_case(m, ph, p, U, prec, elems, blocks=True, jvp=True, tri_pts=None):
    Ud = _dev(U, prec)
    Uq = Ud.double().cpu().numpy()            # the rounded input the GPU sees
    o = O.Oracle(m, ph, p, tri_pts)
    ctx = _ctx(m, ph, prec, tri_pts)
    R = ctx.rhs(Ud)
    torch.cuda.synchronize()
    ctx.sync()
    e_r = rel(R.double().cpu().numpy().reshape(-1), o.rhs(Uq))
    out = {"R": e_r}
    if jvp:
        v = I.random_direction(U.size, 11).reshape(U.shape)
        vd = _dev(v, prec)
        vq = vd.double().cpu().numpy()
        Jv = ctx.jvp(Ud, vd)
        out["Jv"] = rel(Jv.double().cpu().numpy().reshape(-1), o.jvp(Uq, vq))
    if blocks:
        B = ctx.jacobian_blocks(Ud)
        Bn = _blocks_rowmajor(B)
        Bo = o.jac_blocks(Uq, elems, ctx.b, ctx.nface)
        out["blocks"] = max(rel(Bn[e], Bo[i]) for i, e in enumerate(elems))
    ctx.sync()
    return out


def _assert(out, prec, tag=""):
    for k, v in out.items():
        assert v <= TOL[prec], (tag, k, v, out)


def test_advection_cfg0_fp64_full_jacobian():
    """8x8 periodic quads, p=2, c=(1,0.5): R and the full 576x576 Jacobian."""
    p = 2
    m = I.quad_mesh(8, degree=p)
    ph = I.advection_physics((1.0, 0.5))
    U = I.advection_state(m, p, seed=1)
    o = O.Oracle(m, ph, p)
    ctx = _ctx(m, ph, "f64")
    Ud = _dev(U, "f64")
    R = ctx.rhs(Ud).cpu().numpy().reshape(-1)
    assert rel(R, o.rhs(U)) <= 1e-12
    B = _blocks_rowmajor(ctx.jacobian_blocks(Ud))
    b = 9
    J = np.zeros((576, 576))
    for n in range(m.n_elem):
        for s, k in enumerate([n] + [int(x) for x in m.nbr[n]]):
            J[n * b:(n + 1) * b, k * b:(k + 1) * b] += B[n, s]
    Jo = o.jac_full(U.reshape(-1))
    assert rel(J, Jo) <= 1e-12
    # R(U) = J U for the linear residual, with the assembled GPU Jacobian
    assert rel(J @ U.reshape(-1), R) <= 1e-12


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("system", ["adv", "euler", "ns"])
def test_quad_fp64(p, system):
    N = 5
    m = I.quad_mesh(N, degree=p, jitter=0.05, K=1)
    if system == "adv":
        ph, U = I.advection_physics((1.0, 0.5)), I.advection_state(m, p, seed=3)
    elif system == "euler":
        ph, U = I.euler_physics(2), I.ns2d_state(m, p)
    else:
        ph, U = I.ns_physics(2, 100.0, 0.72), I.ns2d_state(m, p)
    out = check_case(m, ph, p, U, "f64", [0, 7, m.n_elem - 1])
    _assert(out, "f64", (p, system))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("system", ["ns", "euler"])
def test_quad_fp32(system, p):
    """FP32 contexts: the matrix-core Jacobian path (every degree, both
    systems), FP64-evaluated residual, FP32 JVP."""
    m = I.quad_mesh(6, degree=p, jitter=0.05, K=1)
    ph = I.ns_physics(2, 1000.0, 0.72) if system == "ns" else I.euler_physics(2)
    out = check_case(m, ph, p, I.ns2d_state(m, p), "f32", [0, 13, 35])
    _assert(out, "f32", (system, p))


def test_ragged_tile_tail():
    """A mesh whose element count is not a multiple of any tile size."""
    p = 2
    m = I.quad_mesh(7, degree=p, jitter=0.05, K=1)       # 49 elements
    out = check_case(m, I.ns_physics(2, 100.0, 0.72), p, I.ns2d_state(m, p), "f64", [48])
    _assert(out, "f64")


@pytest.mark.parametrize("p", [1, 2])
def test_hex_ns_fp64(p):
    m = I.hex_mesh(4, degree=p, jitter=0.05, K=1)
    U = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    out = check_case(m, I.ns_physics(3, 50.0, 0.71), p, U, "f64", [0, 21], blocks=(p == 1))
    _assert(out, "f64", p)


def _rotate_quads(m, seed):
    """The same mesh with each element's local frame rotated by a seeded
    random quarter turn (vertex order shifted; local face f joins vertices f
    and f+1), neighbour face indices updated to match: the face-point
    pairings then differ from element to element."""
    import copy
    r = copy.deepcopy(m)
    sh = np.random.default_rng(seed).integers(0, 4, m.n_elem)
    for e in range(m.n_elem):
        k = int(sh[e])
        r.xyz[e] = np.roll(m.xyz[e], -k, axis=0)
        r.nbr[e] = np.roll(m.nbr[e], -k)
        r.nbr_face[e] = np.roll(m.nbr_face[e], -k)
    for e in range(m.n_elem):
        for f in range(4):
            nb = int(r.nbr[e, f])
            r.nbr_face[e, f] = (int(r.nbr_face[e, f]) - int(sh[nb])) % 4
    return r, sh


def _rotate_hexes(m, seed):
    """The same hex mesh with each element's local frame turned by a seeded
    random proper rotation of the reference cube (one of 24): vertices and
    face data permuted to match, neighbour face indices remapped.  Faces
    0..5 are z-, y-, x+, y+, x-, z+; vertex v is corner offs[v]."""
    import copy
    import itertools
    offs = np.array([(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])
    corner = 2 * offs - 1
    face_of = {(2, -1): 0, (1, -1): 1, (0, 1): 2, (1, 1): 3, (0, -1): 4, (2, 1): 5}
    axis_sign = {f: k for k, f in face_of.items()}
    rots = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((-1, 1), repeat=3):
            R = np.zeros((3, 3), int)
            for i in range(3):
                R[i, perm[i]] = signs[i]
            if round(np.linalg.det(R)) == 1:
                rots.append(R)
    assert len(rots) == 24
    r = copy.deepcopy(m)
    pick = np.random.default_rng(seed).integers(0, 24, m.n_elem)
    tau = np.zeros((m.n_elem, 6), int)     # new face -> old face
    for e in range(m.n_elem):
        R = rots[pick[e]]
        sig = [int(np.where((corner == R.T @ corner[v]).all(axis=1))[0][0]) for v in range(8)]
        r.xyz[e] = m.xyz[e][sig]
        for f in range(6):
            a, sg = axis_sign[f]
            old = R.T @ (sg * np.eye(3, dtype=int)[a])
            ao = int(np.nonzero(old)[0][0])
            tau[e, f] = face_of[(ao, int(old[ao]))]
        r.nbr[e] = m.nbr[e][tau[e]]
        r.nbr_face[e] = m.nbr_face[e][tau[e]]
    for e in range(m.n_elem):
        for f in range(6):
            nb, fo = int(r.nbr[e, f]), int(r.nbr_face[e, f])
            r.nbr_face[e, f] = int(np.nonzero(tau[nb] == fo)[0][0])
    return r, pick


@pytest.mark.parametrize("p,elems", [(2, [0, 21, 63]), (3, [42])])
def test_hex_fp32_rotated_frames(p, elems):
    """Matrix-core path on hexes with rotated local frames (up to 8 face
    orientations): the shared geometry-free sensitivities must follow each
    block's own face-point pairing."""
    m0 = I.hex_mesh(4, degree=p, jitter=0.05, K=1)
    m, pick = _rotate_hexes(m0, 5)
    assert len(set(pick.tolist())) > 12
    ph = I.ns_physics(3, 50.0, 0.71)
    U = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    out = check_case(m, ph, p, U, "f32", elems)
    _assert(out, "f32", p)


@pytest.mark.parametrize("p", [2, 3])
def test_quad_fp32_rotated_frames(p):
    """Matrix-core path on elements with rotated local frames: blocks whose
    geometry-free sensitivities are shared must share the same pairing."""
    m0 = I.quad_mesh(5, degree=p, jitter=0.05, K=1)
    m, sh = _rotate_quads(m0, 3)
    assert len(set(sh.tolist())) == 4
    ph = I.ns_physics(2, 1000.0, 0.72)
    out = check_case(m, ph, p, I.ns2d_state(m, p), "f32", [0, 7, 13, 24])
    _assert(out, "f32", p)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("system", ["adv", "euler", "ns"])
def test_hex_fp32(system, p):
    """FP32 hexahedra: the matrix-core Jacobian path (slabs of solution
    points, split pair tiles for five variables), FP64-evaluated residual,
    FP32 JVP."""
    m = I.hex_mesh(4, degree=p, jitter=0.05, K=1)
    if system == "adv":
        ph, U = I.advection_physics((1.0, 0.5, -0.7)), I.advection_state(m, p, seed=4)
    else:
        ph = I.ns_physics(3, 50.0, 0.71) if system == "ns" else I.euler_physics(3)
        U = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    elems = [0, m.n_elem - 1] if (p < 3 or system == "adv") else [37]
    out = check_case(m, ph, p, U, "f32", elems)
    _assert(out, "f32", (system, p))


def _sampled_blocks(ctx, Ud, elems, out_prec=None):
    """Jacobian blocks of the whole mesh on the device, only the sampled
    elements copied back (row-major, FP64)."""
    B = ctx.jacobian_blocks(Ud) if out_prec is None else ctx.jacobian_blocks(Ud, out_prec=out_prec)
    idx = torch.tensor(elems, device=B.device)
    Bs = B.index_select(0, idx)
    del B
    return _blocks_rowmajor(Bs)


def test_cfg2_full_size_fp32():
    """3D NS, p=3, 24^3 jittered periodic hexes (13824 elements, seven
    320x320 blocks each), FP32: R and the JVP over the whole mesh, Jacobian
    blocks of the whole mesh checked on a seeded sample of elements."""
    p = 3
    m = I.hex_mesh(24, degree=p, jitter=0.05)
    ph = I.ns_physics(3, 1600.0, 0.71)
    U = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    elems = [int(np.random.default_rng(0).integers(m.n_elem)), m.n_elem - 1]
    out = check_case(m, ph, p, U, "f32", elems, blocks=False)
    from paper_2105_08632_amd import fr
    ctx = fr.Context(m, ph, "f32")
    Ud = _dev(U, "f32")
    Uq = Ud.double().cpu().numpy()
    Bn = _sampled_blocks(ctx, Ud, elems)
    torch.cuda.synchronize()
    Bo = O.Oracle(m, ph, p).jac_blocks(Uq, elems, ctx.b, ctx.nface)
    out["blocks"] = max(rel(Bn[i], Bo[i]) for i in range(len(elems)))
    _assert(out, "f32")


def test_cfg2_full_size_bf16():
    """The same 24^3 hex mesh with BF16 blocks (BF16 operands on the matrix
    cores, FP32 accumulation), checked on a seeded sample of elements."""
    p = 3
    m = I.hex_mesh(24, degree=p, jitter=0.05)
    ph = I.ns_physics(3, 1600.0, 0.71)
    U = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    elems = [int(np.random.default_rng(1).integers(m.n_elem)), 0]
    from paper_2105_08632_amd import fr
    ctx = fr.Context(m, ph, "f32")
    Ud = _dev(U, "f32")
    Bn = _sampled_blocks(ctx, Ud, elems, out_prec="bf16")
    torch.cuda.synchronize()
    Bo = O.Oracle(m, ph, p).jac_blocks(Ud.double().cpu().numpy(), elems, ctx.b, ctx.nface)
    err = max(rel(Bn[i], Bo[i]) for i in range(len(elems)))
    assert 1e-6 < err <= TOL["bf16"]


def test_cfg1_full_size_fp32():
    """2D NS, p=3, 128x128 jittered periodic quads, FP32: R and the JVP over
    the whole mesh, Jacobian blocks on a seeded sample of elements."""
    p = 3
    m = I.quad_mesh(128, degree=p, jitter=0.05)
    ph = I.ns_physics(2, 1000.0, 0.72)
    U = I.ns2d_state(m, p)
    elems = list(np.random.default_rng(0).choice(m.n_elem, 12, replace=False)) + [0, m.n_elem - 1]
    out = check_case(m, ph, p, U, "f32", elems)
    _assert(out, "f32")


def test_bf16_blocks():
    p = 3
    m = I.quad_mesh(6, degree=p, jitter=0.05, K=1)
    ph = I.ns_physics(2, 1000.0, 0.72)
    U = I.ns2d_state(m, p)
    Ud = _dev(U, "f32")
    ctx = _ctx(m, ph, "f32")
    B = _blocks_rowmajor(ctx.jacobian_blocks(Ud, out_prec="bf16"))
    Bo = O.Oracle(m, ph, p).jac_blocks(Ud.double().cpu().numpy(), [0, 20], 64, 4)
    err = max(rel(B[e], Bo[i]) for i, e in enumerate([0, 20]))
    assert err <= 2e-2
    assert err > 1e-6     # really stored in bf16


def test_hex_bf16_blocks():
    """BF16 blocks of the 3D NS p=3 Jacobian (the cfg2 block size, 320)."""
    p = 3
    m = I.hex_mesh(4, degree=p, jitter=0.05, K=1)
    ph = I.ns_physics(3, 50.0, 0.71)
    U = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    Ud = _dev(U, "f32")
    ctx = _ctx(m, ph, "f32")
    B = _sampled_blocks(ctx, Ud, [21], out_prec="bf16")
    Bo = O.Oracle(m, ph, p).jac_blocks(Ud.double().cpu().numpy(), [21], ctx.b, ctx.nface)
    err = rel(B[0], Bo[0])
    assert 1e-6 < err <= 2e-2


def test_errors_are_reported():
    from paper_2105_08632_amd import fr
    m = I.quad_mesh(3, degree=2, jitter=0.0)
    # viscous Jacobian needs a second layer that does not fold onto the first
    with pytest.raises(fr.FrError) as ei:
        fr.Context(m, I.ns_physics(2, 100.0, 0.72), "f64")
    assert ei.value.status == -2
    ctx = fr.Context(I.quad_mesh(4, degree=2), I.advection_physics(), "f32")
    with pytest.raises(fr.FrError):
        ctx.jacobian_blocks(ctx.empty_state().zero_(), out_prec="f64")
    with pytest.raises(ValueError):
        ctx.rhs(torch.zeros(3, device="cuda"))


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("system", ["euler", "ns"])
def test_tri_fp64(system, p):
    """Periodic split-cell triangles (random diagonals, jittered vertices)."""
    tp = I.tri_points(p)
    m = I.tri_mesh(5, degree=p, jitter=0.05, K=1, seed=6)
    ph = I.euler_physics(2) if system == "euler" else I.ns_physics(2, 100.0, 0.72)
    U = I.ns2d_state(m, p, tri_pts=tp)
    out = check_case(m, ph, p, U, "f64", [0, 7, m.n_elem - 1], tri_pts=tp)
    _assert(out, "f64", (p, system))


def test_tri_ns_fp32():
    p = 3
    tp = I.tri_points(p)
    m = I.tri_mesh(6, degree=p, jitter=0.05, K=1, seed=7)
    ph = I.ns_physics(2, 1000.0, 0.72)
    U = I.ns2d_state(m, p, tri_pts=tp)
    out = check_case(m, ph, p, U, "f32", [0, 11, m.n_elem - 1], tri_pts=tp)
    _assert(out, "f32", p)
