"""Fourier (von Neumann) analysis on the GPU from the library's own Jacobian
blocks: the eigenvalues of G(kappa) against numpy's eigenvalues of the
symbol built from the oracle's blocks, and the CFL limits of FR-DG for
linear advection against the values the paper prints (temporal linear
stability tables for quadrilaterals, theta0 = pi/6, and hexahedra,
theta0 = pi/6, theta1 = pi/4; golden file with its citation)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2105_08632_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
RK = {"rk3": [1.0, 1.0, 1 / 2, 1 / 6], "rk4": [1.0, 1.0, 1 / 2, 1 / 6, 1 / 24],
      "rk54": [1.0, 1.0, 1 / 2, 1 / 6, 1 / 24, 1 / 200]}


def _setup(etype, p, theta0, theta1, prec):
    from paper_2105_08632_amd import fr
    if etype == I.QUAD:
        c = (np.cos(theta0), np.sin(theta0))
        m = I.quad_mesh(4, degree=p)
    else:
        c = (np.cos(theta0) * np.cos(theta1), np.sin(theta0), np.cos(theta0) * np.sin(theta1))
        m = I.hex_mesh(3, degree=p)
    ph = I.advection_physics(c)
    ctx = fr.Context(m, ph, prec)
    dt = torch.float64 if prec == "f64" else torch.float32
    U = torch.zeros(ctx.ndof, dtype=dt, device="cuda")
    B = ctx.jacobian_blocks(U)
    return fr, m, ph, np.asarray(c), ctx, B


def _matched(a, b):
    """Largest distance from an element of a to the nearest element of b."""
    return float(np.max(np.min(np.abs(a[:, None] - b[None, :]), axis=1)))


@pytest.mark.parametrize("etype,p,prec", [(I.QUAD, 2, "f64"), (I.QUAD, 4, "f64"), (I.HEX, 1, "f64"),
                                          (I.HEX, 2, "f32"), (I.HEX, 3, "f32")])
def test_eigenvalues_match_oracle_symbol(etype, p, prec):
    fr, m, ph, c, ctx, B = _setup(etype, p, np.pi / 6, np.pi / 4, prec)
    print("fourier eigs case", etype, p, prec, flush=True)
    rng = np.random.default_rng(3)
    kap = rng.uniform(-3 * np.pi, 3 * np.pi, size=(12, m.ndim)) * round(m.n_elem ** (1 / m.ndim))
    E = ctx.fourier_eigs(B, 0, torch.from_numpy(kap).cuda(), scale=1.0).cpu().numpy()
    lam = E[..., 0] + 1j * E[..., 1]
    # the symbol from the oracle's blocks, offsets from element centroids
    o = O.Oracle(m, ph, p)
    b = ctx.b
    U = np.zeros(m.n_elem * b)
    ctr = m.xyz.mean(axis=1)
    blocks = []
    for k in [0] + [int(x) for x in m.nbr[0]]:
        d = ctr[k] - ctr[0]
        d -= np.round(d)
        blocks.append((o.jac_block(U, 0, k, b, b), d))
    tol = 1e-9 if prec == "f64" else 3e-5
    for q in range(len(kap)):
        G = sum(Bk * np.exp(1j * (kap[q] @ d)) for Bk, d in blocks)
        ref = np.linalg.eigvals(G)
        scale = np.max(np.abs(ref))
        assert _matched(lam[q], ref) <= tol * scale and _matched(ref, lam[q]) <= tol * scale, q


@pytest.mark.parametrize("etype,p", [(I.QUAD, 1), (I.QUAD, 2), (I.QUAD, 3), (I.QUAD, 4),
                                     (I.HEX, 1), (I.HEX, 2), (I.HEX, 3)])
def test_cfl_max_matches_printed_table(etype, p):
    g = json.load(open(os.path.join(GOLD, "cfl_fr_dg.json")))["quad" if etype == I.QUAD else "hex"]
    prec = "f64" if (etype == I.QUAD or p == 1) else "f32"
    fr, m, ph, c, ctx, B = _setup(etype, p, g["theta0"], g["theta1"], prec)
    print("cfl case", etype, p, prec, flush=True)
    N = round(m.n_elem ** (1 / m.ndim))
    h = 1.0 / N
    nk = 1500 if etype == I.QUAD else 400
    kh = np.linspace(1e-3, 4 * np.pi, nk)
    kap = (kh / h)[:, None] * c[None, :]
    E = ctx.fourier_eigs(B, 0, torch.from_numpy(kap).cuda(), scale=h)     # |c| = 1: CFL = dt / h
    re_max = float(E[..., 0].max().item())
    assert re_max < (1e-10 if prec == "f64" else 1e-5), re_max          # the semi-discretisation is stable
    tol = 1e-12 if prec == "f64" else 1e-6
    got = {s: ctx.cfl_max(E, RK[s], tau_max=2.0, tol=tol) for s in RK}
    print("cfl", etype, p, got, flush=True)
    tight = ("rk4", "rk54") if etype == I.QUAD else ("rk3", "rk54")
    for s in RK:
        lim = 0.002 if s in tight else (0.008 if etype == I.QUAD else 0.01)
        assert abs(got[s] - g[s][p - 1]) <= lim, (s, got[s], g[s][p - 1])


def test_fourier_rejects_triangles_and_large_blocks():
    from paper_2105_08632_amd import fr
    m = I.tri_mesh(3, degree=1)
    ctx = fr.Context(m, I.advection_physics((1.0, 0.5)), "f64", tri_pts=I.tri_points(1))
    U = torch.zeros(ctx.ndof, dtype=torch.float64, device="cuda")
    B = ctx.jacobian_blocks(U)
    kap = torch.zeros(1, 2, dtype=torch.float64, device="cuda")
    with pytest.raises(fr.FrError) as ei:
        ctx.fourier_eigs(B, 0, kap)
    assert ei.value.status == -2
