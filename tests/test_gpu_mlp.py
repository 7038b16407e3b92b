"""Learned block preconditioner on the GPU: network forward and gradients
against the FP64 network oracle at identical (BF16-rounded) weights and
batch, its training inputs against the FP64 residual oracle's Jacobian
blocks, and what the trained network gains inside Newton-GMRES."""
import numpy as np
import pytest

from oracle import mlp as OM
from oracle import oracle as O
from paper_2105_08632_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BF16_TOL = 2e-2


def _ctx(N=8, p=3, Re=1000.0, seeds=(2, 3, 4)):
    from paper_2105_08632_amd import fr
    m = I.quad_mesh(N, degree=p, jitter=0.05, K=1)
    ph = I.ns_physics(2, Re, 0.72)
    U = I.ns2d_state(m, p, seeds=seeds)
    ctx = fr.Context(m, ph, "f64")
    return fr, m, ph, U, ctx


def _dt(m, U, cfl):
    rho = U[..., 0]
    v = U[..., 1:3] / rho[..., None]
    p = 0.4 * (U[..., 3] - 0.5 * rho * np.sum(v * v, axis=-1))
    smax = np.max(np.linalg.norm(v, axis=-1) + np.sqrt(1.4 * p / rho))
    return cfl * (1.0 / round(np.sqrt(m.n_elem))) / smax


def _rounded_params(net):
    """The weights as the matrix cores see them: W in BF16, biases FP32."""
    p = net.params().cpu().numpy().astype(np.float64)
    b, H = net.b, net.hidden
    n = b * b
    q = p.copy()
    sl = [(0, H * n), (H * n + H, H * n + H + H * H), (H * n + 2 * H + H * H, H * n + 2 * H + H * H + n * H)]
    for a, e in sl:
        q[a:e] = torch.from_numpy(p[a:e]).to(torch.bfloat16).double().numpy()
    return q


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def test_inputs_match_oracle_blocks():
    fr, m, ph, U, ctx = _ctx()
    dt = _dt(m, U, 2.0)
    pc = fr.Precond(ctx, fr.FR_PC_MLP)
    X, s = pc.mlp_inputs(torch.from_numpy(U).cuda(), 1.0, -dt)
    X = X.double().cpu().numpy()
    s = s.double().cpu().numpy()
    o = O.Oracle(m, ph, 3)
    b = ctx.b
    for n in (0, 17, m.n_elem - 1):
        A = np.eye(b) - dt * o.jac_block(U, n, n, b, b)
        sr = np.max(np.abs(A))
        assert abs(s[n] - sr) <= 1e-6 * sr                      # s is stored in FP32
        Xr = (A / sr).T.reshape(-1)                             # column-major vec()
        assert np.max(np.abs(X[n] - Xr)) <= 2.0 ** -8 * 1.0 + 1e-12   # one BF16 rounding of values <= 1


def _blocks(seeds_list, cfls, N=8):
    from paper_2105_08632_amd import fr
    out = []
    for seeds in seeds_list:
        fr_, m, ph, U, ctx = _ctx(N=N, seeds=seeds)
        pc = fr.Precond(ctx, fr.FR_PC_MLP)
        Ud = torch.from_numpy(U).cuda()
        for c in cfls:
            X, _ = pc.mlp_inputs(Ud, 1.0, -_dt(m, U, c))
            out.append(X.clone())
    return torch.cat(out)


@pytest.mark.parametrize("nb,max_batch", [(64, 128), (100, 48)])
def test_forward_matches_oracle(nb, max_batch):
    from paper_2105_08632_amd import fr
    X = _blocks([(2, 3, 4), (5, 6, 7)], [1.0])[:nb].contiguous()
    net = fr.Mlp(64, 256, seed=3, max_batch=max_batch)
    Y = net.forward(X).double().cpu().numpy()
    Yr = OM.forward(_rounded_params(net), X.double().cpu().numpy(), 64, 256)
    assert _rel(Y, Yr) <= BF16_TOL


def test_loss_and_gradient_match_oracle():
    from paper_2105_08632_amd import fr
    X = _blocks([(2, 3, 4)], [1.0, 4.0])[:96].contiguous()
    net = fr.Mlp(64, 256, seed=4, max_batch=128)
    # a few steps first, so the output layer is not near zero
    for _ in range(5):
        net.train_step(X, 1e-3)
    loss, g, res = net.loss_grad(X)
    p = _rounded_params(net)
    Lr, gr = OM.loss_grad(p, X.double().cpu().numpy(), 64, 256)
    assert abs(float(loss.item()) - Lr) <= BF16_TOL * Lr
    g = g.double().cpu().numpy()
    H, n = 256, 64 * 64
    groups = {"W1": (0, H * n), "b1": (H * n, H * n + H), "W2": (H * n + H, H * n + H + H * H),
              "b2": (H * n + H + H * H, H * n + 2 * H + H * H), "W3": (H * n + 2 * H + H * H, g.size - n),
              "b3": (g.size - n, g.size)}
    errs = {k: _rel(g[a:e], gr[a:e]) for k, (a, e) in groups.items()}
    assert all(v <= BF16_TOL for v in errs.values()), errs
    Yr = OM.forward(p, X.double().cpu().numpy(), 64, 256)
    rr = OM.residual_norms(X.double().cpu().numpy(), Yr, 64)
    assert _rel(res.double().cpu().numpy(), rr) <= BF16_TOL


def test_trained_network_preconditions_newton_gmres():
    """Trained on blocks of other states, the network alone (no fallback)
    cuts GMRES iterations against no preconditioner on an unseen state."""
    from paper_2105_08632_amd import fr
    train = _blocks([(11 + 3 * i, 12 + 3 * i, 13 + 3 * i) for i in range(12)], [0.5, 1.0, 2.0])
    net = fr.Mlp(64, 256, seed=5, max_batch=512)
    g = torch.Generator(device="cuda").manual_seed(0)
    first = None
    for it in range(1500):
        idx = torch.randint(0, train.shape[0], (256,), device="cuda", generator=g)
        lr = 1e-3 if it < 1000 else 3e-4
        L = net.train_step(train[idx].contiguous(), lr)
        if first is None:
            first = float(L.item())
    fr_, m, ph, U, ctx = _ctx(seeds=(2, 3, 4))
    dt = _dt(m, U, 1.0)
    Ud = torch.from_numpy(U).cuda()
    pc = fr.Precond(ctx, fr.FR_PC_MLP)
    Xh, _ = pc.mlp_inputs(Ud, 1.0, -dt)
    _, _, res = net.loss_grad(Xh.contiguous())
    held = float(res.mean().item())
    assert held < 0.5 * np.sqrt(first), (held, first)
    pc.set_mlp(net, 1e30)
    sol = fr.Solver(ctx, restart=30)
    a = sol.newton_step(Ud, pc=pc, dt=dt, gmres_maxit=500)
    assert pc.n_fallback == 0
    b = sol.newton_step(Ud, pc=None, dt=dt, gmres_maxit=500, check=False)
    assert a["converged"] == 1 and a["res"] <= 1e-8 * a["res0"]
    assert a["gmres_iters"] < b["gmres_iters"], (a["gmres_iters"], b["gmres_iters"])
    # with the safeguard on, elements beyond theta fall back to FP64 LU
    pc.set_mlp(net, 0.0)
    c = sol.newton_step(Ud, pc=pc, dt=dt, gmres_maxit=500)
    assert pc.n_fallback == m.n_elem and c["converged"] == 1
    # Newton-Schulz refinement: from the network's output it needs fewer steps
    # than from the scaled transpose (the same method without the network),
    # and the refined preconditioner does as well as FP64 block-Jacobi LU
    pc.set_mlp(net, 0.05)
    steps = {}
    for start in ("network", "transpose"):
        pc.set_refine(64, 1e-2, start)
        pc.setup(Ud, 1.0, -dt)
        st = pc.stats()
        print("refine", start, st, flush=True)
        assert st["n_fallback"] <= (0 if start == "transpose" else 0.1 * m.n_elem), st
        steps[start] = st["mean_refine_iters"]
    assert steps["network"] < steps["transpose"], steps
    pc.set_refine(16, 1e-2, "network")
    d = sol.newton_step(Ud, pc=pc, dt=dt, gmres_maxit=500)
    e = sol.newton_step(Ud, pc=fr.Precond(ctx), dt=dt, gmres_maxit=500)
    assert d["converged"] == 1 and d["res"] <= 1e-8 * d["res0"]
    assert d["gmres_iters"] <= 1.25 * e["gmres_iters"] + 2, (d["gmres_iters"], e["gmres_iters"])


@pytest.mark.parametrize("start,p", [("transpose", 3), ("transpose", 2), ("network", 3)])
def test_refined_inverse_residual_bounds_the_solve(start, p):
    """A z - r = -(I - A^ M) r exactly for z = M r / s, so the reported
    residual bounds the preconditioner's error against the oracle's blocks;
    from an untrained network the refinement diverges and the safeguard
    hands those elements to FP64 LU, which must then agree with the
    oracle's LU solve."""
    from paper_2105_08632_amd import fr
    fr_, m, ph, U, ctx = _ctx(N=5, p=p)
    dt = _dt(m, U, 5.0)
    Ud = torch.from_numpy(U).cuda()
    pc = fr.Precond(ctx, fr.FR_PC_MLP)
    net = fr.Mlp(ctx.b, 256, seed=5, max_batch=64) if start == "network" else None
    pc.set_mlp(net, 1e-3)
    pc.set_refine(40, 2e-4, start)
    print("refine case", start, p, flush=True)
    pc.setup(Ud, 1.0, -dt)
    st = pc.stats()
    r = I.random_direction(U.shape, 4)
    z = pc.apply(torch.from_numpy(r).cuda()).cpu().numpy().reshape(m.n_elem, -1)
    r = r.reshape(m.n_elem, -1)
    o = O.Oracle(m, ph, p)
    b = ctx.b
    if start == "transpose":
        assert st["n_fallback"] == 0 and st["max_resid"] <= 1e-3, st
        assert st["mean_refine_iters"] >= 1
    for n in (0, 7, m.n_elem - 1):
        A = np.eye(b) - dt * o.jac_block(U, n, n, b, b)
        if start == "transpose":
            bound = 1.01 * st["max_resid"] * np.linalg.norm(r[n]) + 1e-12 * np.linalg.norm(r[n])
            assert np.linalg.norm(A @ z[n] - r[n]) <= bound
        else:
            zr = O.lu_solve(A, r[n])
            assert np.max(np.abs(z[n] - zr)) <= 1e-10 * np.max(np.abs(zr))
