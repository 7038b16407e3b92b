"""fr_rhs_noalloc: the residual with its intermediates in the library's
per-device scratch array instead of the context's workspaces.  Checked
against fr_rhs on the same inputs (the same kernels, so bitwise) on two calls
in a row, the second with a smaller mesh, and against the size limit."""
import numpy as np
import pytest

from paper_2105_08632_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _ctx(N, p, system, prec):
    from paper_2105_08632_amd import fr
    m = I.quad_mesh(N, degree=p, jitter=0.05, K=max(1, N // 4))
    if system == "ns":
        ph, U = I.ns_physics(2, 1000.0, 0.72), I.ns2d_state(m, p)
    else:
        ph, U = I.euler_physics(2), I.isentropic_vortex_state(m, p)
    ctx = fr.Context(m, ph, prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    return ctx, torch.from_numpy(np.ascontiguousarray(U)).to(dt).cuda()


def _check(ctx, Ud):
    R_ref = ctx.rhs(Ud)
    R = torch.full_like(R_ref, float("nan"))
    ctx.rhs_noalloc(Ud, R)
    ctx.sync()
    a, b = R.double().cpu().numpy(), R_ref.double().cpu().numpy()
    rel = float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
    assert rel <= 1e-12, rel                 # FP64 arithmetic in every context
    assert torch.equal(R, R_ref)             # same kernels, same order


def test_noalloc_rhs_matches_rhs_on_two_calls():
    # first call: 2-D Navier-Stokes p = 3 on 64x64 (traces and gradients: 10.5 MB)
    print("noalloc case 1: ns p3 64x64 f64", flush=True)
    big, Ub = _ctx(64, 3, "ns", "f64")
    _check(big, Ub)
    # second call, smaller input of another shape: Euler p = 2 on 12x12, FP32 state
    print("noalloc case 2: euler p2 12x12 f32", flush=True)
    small, Us = _ctx(12, 2, "euler", "f32")
    _check(small, Us)
    # and back to the first context: the scratch holds the second call's values
    print("noalloc case 3: ns p3 64x64 f64 again", flush=True)
    _check(big, Ub)


def test_noalloc_rhs_rejects_meshes_beyond_the_scratch():
    from paper_2105_08632_amd import fr
    print("noalloc case 4: ns p3 192x192 f64 (needs 94 MB)", flush=True)
    ctx, Ud = _ctx(192, 3, "ns", "f64")
    R = ctx.empty_state()
    with pytest.raises(fr.FrError) as ei:
        ctx.rhs_noalloc(Ud, R)
    assert ei.value.status == -2 and "scratch" in str(ei.value), str(ei.value)
    ctx.rhs(Ud)                              # the context still works
    ctx.sync()
