"""Properties of the GPU residual and Jacobian that hold at any size, checked
at the full workload sizes (128x128 quads and 24^3 hexahedra of degree 3):

* free-stream preservation: R(U) = 0 for a uniform state on curved meshes
  (the metric identities of the FR method's transformed equations);
* for the Euler equations the face stencil is the whole Jacobian, so the
  blocks applied to a vector equal the exact Jacobian-vector product, and
  at a uniform state they annihilate every uniform direction (R stays zero
  along it).
"""
import numpy as np
import pytest

from paper_2105_08632_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _uniform(m, p, nv):
    ns = I.n_sol_points(int(m.elem_type[0]), p)
    state = I.conservative(np.array(1.2), np.array([0.3, -0.2, 0.1][:m.ndim]), np.array(17.0), 1.4)
    assert state.shape[-1] == nv
    return np.tile(state, (m.n_elem, ns, 1)), state


def _apply_blocks(B, nbr, v):
    """sum_slot B[n, slot] v[nbr(n, slot)] with B[n, slot, c, r] = dR_n[r] / dU_m[c];
    returns (J v, sum_slot |B| |v|) as [n, b] FP64."""
    ne, ns_, b, _ = B.shape
    idx = torch.cat([torch.arange(ne, device=B.device)[:, None], torch.from_numpy(nbr).to(B.device)], 1)
    out = torch.zeros(ne, b, dtype=torch.float64, device=B.device)
    mag = torch.zeros_like(out)
    for s in range(ns_):
        Bs = B[:, s].double().contiguous()                    # [n, c, r]
        vs = v[idx[:, s]].double().contiguous()               # [n, c]
        out += torch.bmm(vs[:, None, :], Bs)[:, 0]
        mag += torch.bmm(vs.abs()[:, None, :], Bs.abs())[:, 0]
        del Bs
    return out, mag


@pytest.mark.parametrize("case", ["quad128", "hex24"])
def test_free_stream_full_size(case):
    from paper_2105_08632_amd import fr
    if case == "quad128":
        m, ph = I.quad_mesh(128, degree=3, jitter=0.05), I.ns_physics(2, 1000.0, 0.72)
    else:
        m, ph = I.hex_mesh(24, degree=3, jitter=0.05), I.ns_physics(3, 1600.0, 0.71)
    U, state = _uniform(m, 3, ph.nvars)
    fscale = np.max(np.abs(state)) * 20 / m.h
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        ctx = fr.Context(m, ph, prec)
        R = ctx.rhs(torch.from_numpy(U).to(dt).cuda().contiguous())
        assert R.abs().max().item() < 1e-12 * fscale, prec
        del ctx


@pytest.mark.parametrize("case", ["quad128", "hex24"])
def test_euler_blocks_are_the_jacobian_full_size(case):
    """FP32 blocks of the whole mesh applied to a seeded vector against the
    exact (FP64-evaluated) JVP; at a uniform state, against zero for a
    uniform direction.  Bar: 1e-5 of sum |B| |v|, the scale of FP32 rounding
    in the product."""
    from paper_2105_08632_amd import fr
    if case == "quad128":
        m, ph = I.quad_mesh(128, degree=3, jitter=0.05), I.euler_physics(2)
        U = I.ns2d_state(m, 3)
    else:
        m, ph = I.hex_mesh(24, degree=3, jitter=0.05), I.euler_physics(3)
        U = I.tgv_state(m, 3, L=1.0 / (2 * np.pi))
    ctx = fr.Context(m, ph, "f32")
    Ud = torch.from_numpy(U).float().cuda().contiguous()
    v = torch.from_numpy(I.random_direction(U.shape, 7)).float().cuda().contiguous()
    B = ctx.jacobian_blocks(Ud)
    Jv = ctx.jvp(Ud, v).double().view(ctx.ne, ctx.b)
    Bv, mag = _apply_blocks(B, m.nbr, v.view(ctx.ne, ctx.b))
    assert ((Bv - Jv).abs() / mag.max()).max().item() < 1e-5
    assert (Bv - Jv).abs().max().item() > 0.0            # two different evaluations
    Uu, state = _uniform(m, 3, ph.nvars)
    ctx.jacobian_blocks(torch.from_numpy(Uu).float().cuda().contiguous(), B)
    delta = torch.tensor([1.0, 0.1, -0.2, 0.05, 3.0][:ph.nvars], device="cuda")
    d = delta.repeat(ctx.b // ph.nvars)[None, :].expand(ctx.ne, ctx.b).float().contiguous()
    Bd, mag = _apply_blocks(B, m.nbr, d)
    assert (Bd.abs() / mag.max()).max().item() < 1e-5


@pytest.mark.parametrize("case", ["quad128", "hex24"])
def test_conservation_full_size(case):
    """Discrete conservation on the periodic mesh: sum_n sum_i w_i detJ_i R_n,i
    vanishes for every variable (antisymmetric common fluxes, FR-DG
    correction), for the GPU residual of FP64 and FP32 contexts; quadrature
    weights and detJ come from the oracle."""
    from oracle import oracle as O
    from paper_2105_08632_amd import fr
    if case == "quad128":
        m, ph, et = I.quad_mesh(128, degree=3, jitter=0.05), I.ns_physics(2, 1000.0, 0.72), I.QUAD
        U = I.ns2d_state(m, 3)
    else:
        m, ph, et = I.hex_mesh(24, degree=3, jitter=0.05), I.ns_physics(3, 1600.0, 0.71), I.HEX
        U = I.tgv_state(m, 3, L=1.0 / (2 * np.pi))
    o = O.Oracle(m, ph, 3)
    ref = o.ref(et)
    wdj = np.stack([ref["wq"] * o.elem_geom(e, ref["ns"], ref["nf"])["detJ"] for e in range(m.n_elem)])
    for prec, dt in (("f64", torch.float64), ("f32", torch.float32)):
        ctx = fr.Context(m, ph, prec)
        R = ctx.rhs(torch.from_numpy(U).to(dt).cuda().contiguous()).double().cpu().numpy()
        R = R.reshape(m.n_elem, ref["ns"], ph.nvars)
        tot = np.einsum("nr,nra->a", wdj, R)
        scale = np.einsum("nr,nra->a", wdj, np.abs(R))
        # FP32 contexts round each R value to FP32 (relative 2^-24): the sum
        # may then miss zero by up to 2^-24 of its scale
        bar = 1e-12 if prec == "f64" else 1e-12 + 2.0 ** -24
        assert np.max(np.abs(tot) / scale) < bar, prec
        del ctx
