"""The device status word: a NaN in the state reaches R, Jv and the Jacobian
blocks of the element and its face neighbours; the kernels record it and
fr_ctx_sync turns it into FR_E_NONFINITE, naming the outputs and the
smallest element that stored a non-finite value, then clears it.  A plain
value, not a fault: the kernels run to completion."""
import numpy as np
import pytest

from paper_2105_08632_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _setup(prec):
    from paper_2105_08632_amd import fr
    N, p = 6, 2
    m = I.quad_mesh(N, degree=p, jitter=0.05, K=1)
    ph = I.euler_physics(2)
    U = I.isentropic_vortex_state(m, p)
    ctx = fr.Context(m, ph, prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    return fr, m, ctx, torch.from_numpy(np.ascontiguousarray(U)).to(dt).cuda()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nan_in_state_is_reported(prec):
    fr, m, ctx, Ud = _setup(prec)
    bad = 20
    # Euler: R of element n depends on U of n and of its face neighbours only
    stencil = [bad] + [int(x) for x in m.nbr[bad]]
    first = min(stencil)
    print("nonfinite case", prec, "element", bad, "expected first", first, flush=True)
    ctx.sync()                                       # clean before
    Un = Ud.clone()
    Un.view(-1)[bad * ctx.ns * ctx.nv + 3] = float("nan")
    R = ctx.rhs(Un)
    with pytest.raises(fr.FrError) as ei:
        ctx.sync()
    assert ei.value.status == -7
    msg = str(ei.value)
    assert " R" in msg and f"first element {first}" in msg, msg
    ctx.sync()                                       # cleared by the report
    Rn = R.double().cpu().numpy()
    assert np.isnan(Rn[bad]).any() and np.isfinite(np.delete(Rn, stencil, axis=0)).all()
    # Jv and blocks
    v = torch.ones_like(Ud)
    ctx.jvp(Un, v)
    ctx.jacobian_blocks(Un)
    with pytest.raises(fr.FrError) as ei:
        ctx.sync()
    msg = str(ei.value)
    assert ei.value.status == -7 and "Jv" in msg and "Jacobian-blocks" in msg and f"first element {first}" in msg, msg
    # a finite state after the report: no status
    ctx.rhs(Ud)
    ctx.jacobian_blocks(Ud)
    ctx.sync()


def test_newton_reports_nonfinite_state():
    from paper_2105_08632_amd import fr
    N, p = 4, 2
    m = I.quad_mesh(N, degree=p, jitter=0.05, K=1)
    ph = I.ns_physics(2, 100.0, 0.72)
    U = I.ns2d_state(m, p)
    ctx = fr.Context(m, ph, "f64")
    Un = torch.from_numpy(U).cuda()
    Un.view(-1)[5] = float("nan")
    solver = fr.Solver(ctx, 10)
    Uo = torch.empty_like(Un)
    with pytest.raises(fr.FrError) as ei:
        solver.newton_step(Un, Uo, dt=1e-3, newton_rtol=1e-8, newton_maxit=3, gmres_rtol=1e-3, gmres_maxit=50)
    assert ei.value.status == -7
    ctx.sync()                                       # the step cleared the word
