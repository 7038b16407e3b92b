#!/usr/bin/env python3
"""Benchmark of the FR-DG residual + Jacobian-block assembly on one MI355X.

Headline workload: 3-D compressible Navier-Stokes (gamma 1.4, Re 1600,
Pr 0.71), FR-DG degree 3 on a 24^3 periodic hexahedral mesh with 5% vertex
jitter, Rusanov + BR1 fluxes, Taylor-Green state at Mach 0.1 with random
phases.  One step = R(U) plus the seven 320x320 Jacobian blocks of every
element (FP32 block storage, 39.6 GB), inputs resident in HBM.  Beside it:
the same step with BF16 blocks, the FP64 block-Jacobi LU of the diagonal
blocks, the 2-D NS p=3 step on 128^2 quads, the mixed-mesh batch, the
Newton-GMRES step with block-Jacobi LU and the learned preconditioner, and
the FP64 oracle timed on the host with each output's error against it.
Prints one JSON line.

Options: --gpus N (only 1: the benchmark drives one GPU), --steps K, --warmup W.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Jacobian+RHS DOF/s (% roofline); Newton-GMRES s/step learned vs plain PC"
HBM_PEAK_GBS = 8000.0


def workload():
    from paper_2105_08632_amd import inputs as I
    p = 3
    m = I.quad_mesh(128, degree=p, jitter=0.05)
    ph = I.ns_physics(2, reynolds=1000.0, prandtl=0.72)
    U = I.ns2d_state(m, p, seeds=(2, 3, 4), mach=0.2)
    return m, ph, p, U


def jac_bytes_per_element(ns, nv, nd, nf, nface, bytes_out=4):
    """Algorithmic HBM bytes of one element's block assembly: the blocks
    written once, the state and the geometry read once."""
    b = ns * nv
    out = (1 + nface) * b * b * bytes_out
    state = ns * nv * 4
    geom = (2 * ns * nd * nd + ns + nf * nd + nf + nf) * 4 + nface * 4
    return out + state + geom


JAC_SOURCES = ("fr_kernels.hpp", "fr_jac_tp.hpp", "fr_jac_mf.hpp", "physics.hpp", "dual.hpp", "fr_impl.hpp")


def kernel_source_hash(files=JAC_SOURCES):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2105_08632_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(name, kernel=None):
    """HBM bytes per launch (of all the summary's kernels, or of one) from a
    committed rocprofv3 counter summary, if it was taken on the current
    kernel source."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != kernel_source_hash(tuple(d.get("sources", JAC_SOURCES))):
        return None
    if kernel:
        k = d["per_kernel"][kernel]
        return k["hbm_read_bytes"] + k["hbm_write_bytes"]
    return d.get("hbm_bytes_per_launch")


def _dt(m, U, cfl, gamma=1.4):
    """Backward-Euler step for an acoustic CFL: cfl * h / max(|v| + c)."""
    rho = U[..., 0]
    v = U[..., 1:3] / rho[..., None]
    pr = (gamma - 1.0) * (U[..., 3] - 0.5 * rho * np.sum(v * v, axis=-1))
    smax = np.max(np.linalg.norm(v, axis=-1) + np.sqrt(gamma * pr / rho))
    return cfl / round(np.sqrt(m.n_elem)) / smax


def train_mlp(torch, fr, I, steps, log):
    """The learned preconditioner, trained on the library's own diagonal
    blocks I - dt dR_n/dU_n from 128x128 NS p=3 states (seeds 11-18), at
    Re 500 and 1000 (so the 256x256 mesh's cell Reynolds numbers are inside
    the training set) and CFL 2..100; Adam, batch 1024."""
    t0 = time.perf_counter()
    m1 = I.quad_mesh(128, degree=3, jitter=0.05)
    blocks = []
    for Re in (500.0, 1000.0):
        ph = I.ns_physics(2, reynolds=Re, prandtl=0.72)
        for i in range(8):
            U = I.ns2d_state(m1, 3, seeds=(11 + i, 111 + i, 211 + i))
            ctx = fr.Context(m1, ph, "f64")
            pc = fr.Precond(ctx, fr.FR_PC_MLP)
            Ud = torch.from_numpy(U).cuda()
            for c in (2.0, 5.0, 10.0, 25.0, 50.0, 100.0):
                X, _ = pc.mlp_inputs(Ud, 1.0, -_dt(m1, U, c))
                blocks.append(X.clone())
            del pc, ctx
    train = torch.cat(blocks)
    del blocks
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = fr.Mlp(64, 256, seed=5, max_batch=4096)
    g = torch.Generator(device="cuda").manual_seed(0)
    t0 = time.perf_counter()
    loss = None
    for it in range(steps):
        idx = torch.randint(0, train.shape[0], (1024,), device="cuda", generator=g)
        lr = 1e-3 if it < 0.6 * steps else (3e-4 if it < 0.85 * steps else 1e-4)
        loss = net.train_step(train[idx].contiguous(), lr)
        if it % 4000 == 0:
            log(f"mlp step {it} loss {float(loss.item()):.3f}")
    torch.cuda.synchronize()
    info = {"samples": int(train.shape[0]), "steps": steps, "batch": 1024, "data_s": round(t_data, 2),
            "train_s": round(time.perf_counter() - t0, 2), "final_batch_loss": round(float(loss.item()), 4)}
    del train
    return net, info


def _pc_times(torch, pc, Ud, dt, r, z, reps=3):
    """Setup and apply times of a preconditioner (HIP events, ms)."""
    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n
    return timed(lambda: pc.setup(Ud, 1.0, -dt), reps), timed(lambda: pc.apply(r, z), 10)


def newton_bench(torch, fr, I, train_steps, log):
    """Seconds per backward-Euler Newton step (to |F| <= 1e-8 |F0|, GMRES(30),
    forcing 1e-3) on 256x256 NS p=3: FP64 block-Jacobi (Gauss-Jordan
    inverses) against the learned preconditioner (network, then Newton-Schulz
    refinement, FP64 block-Jacobi fallback where ||I - A^ M||_F > theta), the
    network alone, and the same refinement started without the network; each
    set up at U^n (setup time included)."""
    net, info = train_mlp(torch, fr, I, train_steps, log)
    ph = I.ns_physics(2, reynolds=1000.0, prandtl=0.72)
    m = I.quad_mesh(256, degree=3, jitter=0.05)
    theta = 0.05
    out = {"workload": "2D NS p=3, 256x256 jittered periodic quads (4.19 M DOF), backward Euler, Newton to "
                       "1e-8 relative, GMRES(30) forcing 1e-3, preconditioner set up at U^n, host-driven "
                       "Arnoldi (lu_graph: restart cycles replayed from a captured hipGraph)",
           "mlp_training": info, "theta": theta,
           "variants": {"lu": "FP64 block-Jacobi, Gauss-Jordan inverses (the comparator)",
                        "learned": "network + Newton-Schulz refinement to ||I - A^M||_F <= 1e-2 (FP32, at most "
                                   "16 steps), FP32 inverse, FP64 LU fallback above theta",
                        "mlp_only": "network output (BF16) as is, FP64 LU fallback above theta = 1",
                        "ns_no_network": "the same refinement from the scaled transpose (no network, at most 64 "
                                         "steps)"}}
    runs = {}
    per = {}
    held = []
    cfl = 5.0
    for s in (8, 9, 10):
        U = I.ns2d_state(m, 3, seeds=(s, 100 + s, 200 + s))
        ctx = fr.Context(m, ph, "f64")
        Ud = torch.from_numpy(U).cuda()
        dt = _dt(m, U, cfl)
        sol = fr.Solver(ctx, restart=30)
        pcl = fr.Precond(ctx)
        pcs = {"lu": (pcl, False), "lu_graph": (pcl, True)}
        for name, refine, start, th in (("learned", 16, "network", theta), ("mlp_only", 0, "network", 1.0),
                                        ("ns_no_network", 64, "transpose", theta)):
            pc = fr.Precond(ctx, fr.FR_PC_MLP)
            pc.set_mlp(net if start == "network" else None, th)
            pc.set_refine(refine, 1e-2, start)
            pcs[name] = (pc, False)
        if s == 8:
            Xh, _ = pcs["learned"][0].mlp_inputs(Ud, 1.0, -dt)
            held.append(float(torch.cat([net.loss_grad(Xh[i:i + 4096].contiguous())[2]
                                         for i in range(0, Xh.shape[0], 4096)]).mean().item()))
            del Xh
            r = torch.randn_like(Ud)
            z = torch.empty_like(Ud)
            for name, (pc, _) in pcs.items():
                if name == "lu_graph":
                    continue
                t_setup, t_apply = _pc_times(torch, pc, Ud, dt, r, z)
                per[name] = {"setup_ms": round(t_setup, 3), "apply_ms": round(t_apply, 4)}
                if name != "lu":
                    per[name].update({k: (round(v, 4) if isinstance(v, float) else v) for k, v in pc.stats().items()})
            log(f"preconditioners: {per}")
        for name, (pc, graph) in pcs.items():
            r = sol.newton_step(Ud, pc=pc, dt=dt, gmres_maxit=3000, newton_maxit=12, check=False, use_graph=graph)
            r["n_fallback"] = pc.stats()["n_fallback"] if name not in ("lu", "lu_graph") else 0
            runs.setdefault(name, []).append(r)
            log(f"newton cfl {cfl} seed {s} {name}: conv {r['converged']} newton {r['newton_iters']} "
                f"gmres {r['gmres_iters']} s {r['ms'] / 1e3:.3f} fallback {r['n_fallback']}")
        if s == 8:
            # largest CFL at which the LU-preconditioned step converges on 256^2
            study = {}
            for c in (10.0, 20.0, 50.0, 100.0):
                for name in ("lu", "learned"):
                    pc, _ = pcs[name]
                    r = sol.newton_step(Ud, pc=pc, dt=_dt(m, U, c), gmres_maxit=3000, newton_maxit=12,
                                        check=False)
                    study.setdefault(str(c), {})[name] = {
                        "converged": bool(r["converged"]), "newton_iters": r["newton_iters"],
                        "gmres_iters": r["gmres_iters"], "final_rel_residual": r["res"] / r["res0"],
                        "s": round(r["ms"] / 1e3, 3)}
                    log(f"newton cfl {c} {name}: conv {r['converged']} gmres {r['gmres_iters']} "
                        f"rel {r['res'] / r['res0']:.2e} s {r['ms'] / 1e3:.3f}")
            out["cfl_study_256"] = study
        del sol, pcs, pcl, ctx
    # CFL 100 on 64x64, where GMRES(30) with a one-level block preconditioner
    # still converges
    m64 = I.quad_mesh(64, degree=3, jitter=0.05)
    U = I.ns2d_state(m64, 3, seeds=(8, 108, 208))
    ctx = fr.Context(m64, ph, "f64")
    Ud = torch.from_numpy(U).cuda()
    sol = fr.Solver(ctx, restart=30)
    pcl = fr.Precond(ctx)
    pcm = fr.Precond(ctx, fr.FR_PC_MLP)
    pcm.set_mlp(net, theta)
    pcm.set_refine(16, 1e-2, "network")
    small = {}
    for name, pc, aug in (("lu", pcl, 0), ("lu_loose3", pcl, 3), ("learned", pcm, 0), ("learned_loose3", pcm, 3)):
        r = sol.newton_step(Ud, pc=pc, dt=_dt(m64, U, 100.0), gmres_maxit=3000, newton_maxit=12, check=False,
                            augment=aug)
        small[name] = {"converged": bool(r["converged"]), "newton_iters": r["newton_iters"],
                       "gmres_iters": r["gmres_iters"], "final_rel_residual": r["res"] / r["res0"],
                       "s": round(r["ms"] / 1e3, 3)}
        log(f"newton cfl 100 64x64 {name}: conv {r['converged']} gmres {r['gmres_iters']} s {r['ms'] / 1e3:.3f}")
    out["cfl100_64x64"] = small
    del sol, pcm, pcl, ctx
    for name, rs in runs.items():
        ms = float(np.median([r["ms"] for r in rs]))
        it = float(np.median([r["gmres_iters"] for r in rs]))
        out[name] = {"s_per_step_median": round(ms / 1e3, 4),
                     "converged": [bool(r["converged"]) for r in rs],
                     "newton_iters": [r["newton_iters"] for r in rs], "gmres_iters": [r["gmres_iters"] for r in rs],
                     "n_fallback": [r["n_fallback"] for r in rs]}
        if name in per:
            out[name].update(per[name])
            out[name]["ms_per_gmres_iter"] = round((ms - per[name]["setup_ms"]) / max(it, 1.0), 4)
    out["cfl"] = cfl
    out["mlp_heldout_resid_mean"] = round(float(np.mean(held)), 3)
    lu_best = min(out["lu"]["s_per_step_median"], out["lu_graph"]["s_per_step_median"])
    out["learned_over_lu_time"] = round(out["learned"]["s_per_step_median"] / lu_best, 3)
    out["mlp_only_over_lu_time"] = round(out["mlp_only"]["s_per_step_median"] / lu_best, 3)
    return out


def newton_step_profile(torch, fr, I, log):
    """One backward-Euler Newton step on 256x256 NS p=3 at CFL 5 with FP64
    block-Jacobi, host-driven and then graph-replayed (after one untimed step
    of each), for kernel traces of the GMRES loop."""
    ph = I.ns_physics(2, reynolds=1000.0, prandtl=0.72)
    m = I.quad_mesh(256, degree=3, jitter=0.05)
    U = I.ns2d_state(m, 3, seeds=(8, 108, 208))
    ctx = fr.Context(m, ph, "f64")
    Ud = torch.from_numpy(U).cuda()
    dt = _dt(m, U, 5.0)
    sol = fr.Solver(ctx, restart=30)
    pc = fr.Precond(ctx)
    out = {"workload": "2D NS p=3, 256x256 jittered periodic quads, backward Euler at CFL 5, Newton to 1e-8 "
                       "relative, GMRES(30), FP64 block-Jacobi"}
    for mode in ("host", "graph"):
        for rep in range(2):
            r = sol.newton_step(Ud, pc=pc, dt=dt, gmres_maxit=3000, newton_maxit=12, check=False,
                                use_graph=(mode == "graph"))
            log(f"newton {mode} rep {rep}: conv {r['converged']} newton {r['newton_iters']} "
                f"gmres {r['gmres_iters']} ms {r['ms']:.1f}")
        out[mode] = {"converged": bool(r["converged"]), "newton_iters": r["newton_iters"],
                     "gmres_iters": r["gmres_iters"], "ms": round(r["ms"], 2),
                     "ms_per_gmres_iter": round(r["ms"] / max(1, r["gmres_iters"]), 4)}
    return out


def rk54_pm_bench(torch, fr, I, log, N=40, steps=4):
    """The paper's own performance metric on its own case: wall time per
    degree of freedom per Runge-Kutta stage, PM = T / (N_iter N_s N_V n_elem
    N_RK), for the Taylor-Green vortex on N^3 hexahedra, degree 3,
    Navier-Stokes, RK54 at a constant time step (one R(U) evaluation and one
    stage update per stage), for FR-DG, FR-SDRT and SDRT.  FP64 state and
    arithmetic."""
    import dataclasses
    p = 3
    m = I.hex_mesh(N, degree=p)
    U0 = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    rho = U0[..., 0]
    v = U0[..., 1:4] / rho[..., None]
    pr = 0.4 * (U0[..., 4] - 0.5 * rho * np.sum(v * v, axis=-1))
    dt = 0.1 / N / float(np.max(np.linalg.norm(v, axis=-1) + np.sqrt(1.4 * pr / rho)))
    paper = {"fr_dg": 0.67, "fr_sdrt": 0.67, "sdrt": 0.85}
    out = {"workload": f"Taylor-Green vortex, 3-D Navier-Stokes degree 3 on {N}^3 hexahedra, RK54, FP64",
           "steps": steps, "paper_hardware": "one NVIDIA V100 (PyFR), precision not stated"}
    for name, scheme in (("fr_dg", 0), ("fr_sdrt", 1), ("sdrt", 2)):
        ph = dataclasses.replace(I.ns_physics(3, 1600.0, 0.71), scheme=scheme)
        ctx = fr.Context(m, ph, "f64")
        U = torch.from_numpy(U0).cuda().contiguous().view(-1)
        work = torch.empty(2 * ctx.ndof, dtype=torch.float64, device="cuda")
        ctx.rk54(U, dt, 1, work)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.rk54(U, dt, steps, work)
        e1.record()
        torch.cuda.synchronize()
        ctx.sync()
        ms = e0.elapsed_time(e1)
        pm = ms * 1e6 / (steps * ctx.ndof * 5)
        out["dof"] = ctx.ndof
        out[name] = {"ms_per_step": round(ms / steps, 3), "pm_ns_per_dof_stage": round(pm, 4),
                     "paper_pm_ns": paper[name], "finite": bool(torch.isfinite(U).all())}
        log(f"rk54 pm {name}: {pm:.4f} ns per DOF per stage ({ms / steps:.2f} ms per step)")
        del ctx, U, work
        torch.cuda.empty_cache()
    return out


def fourier_bench(torch, fr, I, log):
    """Von Neumann analysis on the GPU from the library's own Jacobian blocks:
    FR-DG linear advection (theta0 = pi/6, theta1 = pi/4), eigenvalues of the
    Fourier symbol along the ray kappa h in (0, 4 pi] and the RK3 / RK4 / RK54
    CFL limits, against the paper's printed values."""
    rk = {"rk3": [1.0, 1.0, 1 / 2, 1 / 6], "rk4": [1.0, 1.0, 1 / 2, 1 / 6, 1 / 24],
          "rk54": [1.0, 1.0, 1 / 2, 1 / 6, 1 / 24, 1 / 200]}
    printed = {"quad": {"rk3": 0.096, "rk4": 0.106, "rk54": 0.162}, "hex": {"rk3": 0.075, "rk4": 0.084, "rk54": 0.127}}
    out = {}
    t0, t1 = np.pi / 6, np.pi / 4
    for name, nk in (("quad", 1500), ("hex", 400)):
        p = 3
        if name == "quad":
            c = np.array([np.cos(t0), np.sin(t0)])
            m, prec = I.quad_mesh(4, degree=p), "f64"
        else:
            c = np.array([np.cos(t0) * np.cos(t1), np.sin(t0), np.cos(t0) * np.sin(t1)])
            m, prec = I.hex_mesh(3, degree=p), "f32"
        ctx = fr.Context(m, I.advection_physics(c), prec)
        U = torch.zeros(ctx.ndof, dtype=torch.float64 if prec == "f64" else torch.float32, device="cuda")
        h = 1.0 / round(m.n_elem ** (1 / m.ndim))
        kap = torch.from_numpy((np.linspace(1e-3, 4 * np.pi, nk) / h)[:, None] * c[None, :]).cuda()
        tol = 1e-12 if prec == "f64" else 1e-6

        def run():
            B = ctx.jacobian_blocks(U)
            E = ctx.fourier_eigs(B, 0, kap, scale=h)
            return {s: ctx.cfl_max(E, rk[s], tau_max=2.0, tol=tol) for s in rk}

        run()
        torch.cuda.synchronize()
        ts = time.perf_counter()
        got = run()
        ms = (time.perf_counter() - ts) * 1e3
        out[name + "_p3"] = {"wavenumbers": nk, "block": ctx.b, "blocks_precision": prec, "ms": round(ms, 2),
                             "cfl": {s: round(v, 4) for s, v in got.items()}, "printed": printed[name]}
        log(f"fourier {name} p3: {ms:.1f} ms {got}")
    return out


def batch_bench(torch, fr, I, reps, log):
    """64 independent periodic 2-D Euler meshes (FP32; triangles and quads,
    degrees 1-4, 500-5000 elements each): residual + all Jacobian blocks,
    per-mesh calls vs one persistent launch per phase, before and after the
    autotuner."""
    meshes = I.mixed_batch()
    ph = I.euler_physics(2)
    ctxs = [fr.Context(m, ph, "f32", tri_pts=tp) for (m, p, tp, U) in meshes]
    Us = [torch.from_numpy(U).float().cuda().contiguous() for (m, p, tp, U) in meshes]
    Rs = [c.empty_state() for c in ctxs]
    Bs = [c.block_tensor("f32") for c in ctxs]
    dof = sum(c.ndof for c in ctxs)
    # algorithmic bytes: every block written once (FP32), U read and R
    # written once, and per element its geometry (S and J^-1 at the solution
    # points, 1/detJ, normals, |N|, partner indices, neighbours) read once
    alg = 0
    for c, (m, p, tp, U) in zip(ctxs, meshes):
        alg += int(c.block_offsets[-1]) * 4 + c.ndof * 4 * 2
        for t in set(m.elem_type.tolist()):
            ne_t = int(np.sum(m.elem_type == t))
            ns, nface = I.n_sol_points(t, p), (3 if t == I.TRI else 4)
            nf = nface * (p + 1)
            alg += ne_t * ((2 * ns * 4 + ns + nf * 2 + nf + nf) * 4 + nface * 4)
    batch = fr.Batch(ctxs)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def alone():
        for c, u, r, bb in zip(ctxs, Us, Rs, Bs):
            c.rhs(u, r)
            c.jacobian_blocks(u, bb, "f32")

    def batched():
        batch.rhs(Us, Rs)
        batch.jacobian_blocks(Us, Bs)

    t_alone = timed(alone)
    t_batch = timed(batched)
    t0 = time.perf_counter()
    table = batch.tune(Us, reps=2)
    t_tune = time.perf_counter() - t0
    t_tuned = timed(batched)
    finite = all(bool(torch.isfinite(bb).all()) and bool(torch.isfinite(r).all()) for r, bb in zip(Rs, Bs))
    log(f"batch: alone {t_alone:.2f} ms, batched {t_batch:.2f} ms, tuned {t_tuned:.2f} ms")
    floor_ms = alg / (HBM_PEAK_GBS * 1e9) * 1e3
    return {"workload": "64 periodic 2-D Euler meshes, each mixing triangles and quadrilaterals (random "
                        "quad-to-two-triangle splits, 30-70%), smooth subsonic state, FP32, p 1-4, 500-5000 "
                        "elements each: R(U) + all Jacobian blocks (rectangular across triangle-quad faces)",
            "meshes": len(ctxs), "elements": int(sum(c.ne for c in ctxs)), "dof": int(dof),
            "alg_bytes": int(alg), "hbm_floor_ms": round(floor_ms, 3),
            "ms_per_mesh_calls": round(t_alone, 3), "ms_batched_default": round(t_batch, 3),
            "ms_batched_tuned": round(t_tuned, 3), "tune_s": round(t_tune, 2),
            "dof_per_s_tuned": dof / (t_tuned * 1e-3), "frac_of_hbm_floor": round(floor_ms / t_tuned, 4),
            "tuning": table, "outputs_finite": finite}


def _omp():
    """The OpenMP runtime the oracle is linked against (thread count control)."""
    import ctypes
    try:
        g = ctypes.CDLL("libgomp.so.1")
        g.omp_get_max_threads.restype = ctypes.c_int
        return g
    except OSError:
        return None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def cpu_baseline(m, ph, p, U32, R_gpu, Jv_gpu, v, blocks, budget_s, log):
    """The FP64 oracle (as is) on a bounded sample of the headline workload:
    the full-mesh residual, then all Jacobian blocks of a seeded sample of
    elements (complex-step columns), timed on every host core and on one
    thread; the same oracle results give each GPU output's error.

    U32: the state as the GPU saw it (FP32, widened to FP64), so input
    rounding is not charged to the kernels.  blocks: {prec: (elements,
    GPU blocks [n, slot, c, r] as float64)} for the sampled elements."""
    from oracle import oracle as O
    o = O.Oracle(m, ph, p)
    omp = _omp()
    cores = omp.omp_get_max_threads() if omp else int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    nface = m.max_face
    b = R_gpu.shape[1] * R_gpu.shape[2]
    t0 = time.perf_counter()
    R_ref = o.rhs(U32)
    t_rhs = time.perf_counter() - t0
    errors = {"R": _rel(R_gpu.reshape(-1), R_ref)}
    Jv_ref = o.jvp(U32, v)
    errors["Jv"] = _rel(Jv_gpu.reshape(-1), Jv_ref)
    elems = next(iter(blocks.values()))[0]
    t0 = time.perf_counter()
    ref = o.jac_blocks(U32, elems, b, nface)
    t_blk = time.perf_counter() - t0
    for prec, (el, B) in blocks.items():
        assert np.array_equal(el, elems)
        Bg = B.transpose(0, 1, 3, 2)                 # [n, slot, r, c] like the oracle's
        errors["blocks_" + prec] = max(_rel(Bg[i], ref[i]) for i in range(len(el)))
    n = len(elems)
    t = t_blk + t_rhs * n / m.n_elem
    out = {"value": n * b / t, "unit": "DOF/s", "cores": cores, "kind": "oracle",
           "sample": f"full-mesh R ({t_rhs:.2f} s, scaled to the sample) + all {1 + nface} Jacobian blocks of "
                     f"{n} seeded elements of {m.n_elem} ({t_blk:.1f} s); FP64, complex-step columns",
           "cpu_model": cpu_model()}
    if omp is not None:
        omp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        o.jac_blocks(U32, elems[:1], b, nface)
        t1 = time.perf_counter() - t0
        omp.omp_set_num_threads(cores)
        out["one_thread"] = {"value": b / (t1 + t_rhs * cores / m.n_elem), "unit": "DOF/s", "cores": 1,
                             "sample": f"all blocks of 1 element ({t1:.1f} s) + its share of the residual "
                                       f"(all-core R time x cores / elements, {t_rhs * cores / m.n_elem * 1e3:.2f} ms)"}
    log(f"cpu baseline: {out['value']:.1f} DOF/s on {cores} threads; errors {errors}")
    return out, errors


def _threads(omp, n):
    if omp is not None:
        omp.omp_set_num_threads(n)


def cpu_table(torch, fr, I, log, budget_s):
    """The oracle timed on one host thread and on all of them beside the
    GPU, per workload: the 8x8 advection case (R and the full Jacobian), the
    128^2 NS step (R and all blocks: the full residual plus a seeded sample of
    elements, extrapolated), the 64-mesh mixed batch (the residuals of two
    meshes and the blocks of a seeded sample of elements, extrapolated to the
    64 meshes), and one backward-Euler Newton-GMRES step with block Jacobi
    on a 64^2 NS mesh (the oracle's plain Newton-GMRES; the one-thread figure
    from its first GMRES iterations, extrapolated).  Each row states its
    sample.  The 24^3 hexahedral row is the main line's cpu_baseline."""
    from oracle import newton as ON
    from oracle import oracle as O
    omp = _omp()
    cores = omp.omp_get_max_threads() if omp else (os.cpu_count() or 1)
    rows = {"cores": cores, "cpu_model": cpu_model()}

    def clock(fn):
        t0 = time.perf_counter()
        r = fn()
        return time.perf_counter() - t0, r

    # ---- 8x8 periodic advection, p=2: R and the full 576x576 Jacobian (FP64)
    p = 2
    m = I.quad_mesh(8, degree=p)
    ph = I.advection_physics((1.0, 0.5))
    U = I.advection_state(m, p, seed=1).reshape(-1)
    o = O.Oracle(m, ph, p)
    t_all, J = clock(lambda: (o.rhs(U), o.jac_full(U)))
    _threads(omp, 1)
    t_one, _ = clock(lambda: (o.rhs(U), o.jac_full(U)))
    _threads(omp, cores)
    ctx = fr.Context(m, ph, "f64")
    Ud = torch.from_numpy(U).cuda()
    B = ctx.block_tensor("f64")
    R = ctx.empty_state()

    def step():
        ctx.rhs(Ud, R)
        ctx.jacobian_blocks(Ud, B, "f64")
    wall, _, _ = _timed_steps(torch, ctx, step, 20, 3)
    Bn = B.cpu().numpy().transpose(0, 1, 3, 2)
    Jg = np.zeros((U.size, U.size))
    b = Bn.shape[-1]
    for n in range(m.n_elem):
        for sl, k in enumerate([n] + [int(x) for x in m.nbr[n]]):
            Jg[n * b:(n + 1) * b, k * b:(k + 1) * b] += Bn[n, sl]
    rows["cfg0"] = {"workload": "2-D advection p=2, 8x8 periodic quads: R + full 576x576 Jacobian, FP64",
                    "oracle_1core_dof_s": U.size / t_one, "oracle_allcore_dof_s": U.size / t_all,
                    "gpu_dof_s": U.size * 20 / wall, "gpu_ms": 1e3 * wall / 20,
                    "max_rel_error": max(_rel(R.cpu().numpy().reshape(-1), o.rhs(U)), _rel(Jg, J[1])),
                    "sample": "whole workload"}
    log(f"cpu table cfg0: {rows['cfg0']}")
    del ctx, B, R, o

    # ---- 128^2 NS p=3: full R + all blocks of a seeded element sample
    m, ph, p, U = workload()
    U32 = U.astype(np.float32).astype(np.float64)
    o = O.Oracle(m, ph, p)
    t_r, Rref = clock(lambda: o.rhs(U32))
    rng = np.random.default_rng(1)
    el = np.sort(rng.choice(m.n_elem, 64, replace=False))
    b = U.shape[1] * U.shape[2]
    t_b, Bref = clock(lambda: o.jac_blocks(U32, el, b, 4))
    _threads(omp, 1)
    t_b1, _ = clock(lambda: o.jac_blocks(U32, el[:4], b, 4))
    t_r1, _ = clock(lambda: o.rhs(U32))
    _threads(omp, cores)
    per_all = t_r + t_b * m.n_elem / len(el)
    per_one = t_r1 + t_b1 * m.n_elem / 4
    ctx = fr.Context(m, ph, "f32")
    Ud = torch.from_numpy(U32).float().cuda().contiguous()
    B = ctx.block_tensor("f32")
    R = ctx.empty_state()
    ctx.rhs(Ud, R)
    ctx.jacobian_blocks(Ud, B, "f32")
    sel = torch.from_numpy(el).cuda()
    Bg = B[sel].double().cpu().numpy().transpose(0, 1, 3, 2)
    err = max(_rel(R.double().cpu().numpy().reshape(-1), Rref), max(_rel(Bg[i], Bref[i]) for i in range(len(el))))
    rows["cfg1"] = {"workload": "2-D NS p=3, 128^2 jittered quads: R + the five 64x64 blocks per element; GPU FP32 "
                                "blocks, oracle FP64 at the GPU's FP32 inputs",
                    "oracle_1core_dof_s": U.size / per_one, "oracle_allcore_dof_s": U.size / per_all,
                    "max_rel_error": err,
                    "sample": f"full R; blocks of 64 seeded elements (all cores, {t_b:.1f} s) / 4 (one thread, "
                              f"{t_b1:.1f} s), extrapolated to 16384"}
    log(f"cpu table cfg1: {rows['cfg1']}")
    del ctx, B, R, o

    # ---- the 64-mesh mixed batch
    meshes = I.mixed_batch()
    errs = []
    rng = np.random.default_rng(2)
    picks = rng.choice(len(meshes), 2, replace=False)
    frac_time_all = frac_time_one = 0.0
    dof_sampled = 0
    ph = I.euler_physics(2)
    for mi in picks:
        m, p, tp, Um = meshes[mi]
        o = O.Oracle(m, ph, p, tp)
        Uq = np.ascontiguousarray(Um.reshape(-1)).astype(np.float32).astype(np.float64)
        t_r, Rref = clock(lambda: o.rhs(Uq))
        el = np.sort(rng.choice(m.n_elem, 8, replace=False))
        t_b = 0.0
        refs = {}
        for n in el:
            nf = 3 if m.elem_type[n] == I.TRI else 4
            bn = I.n_sol_points(int(m.elem_type[n]), p) * ph.nvars
            t, r = clock(lambda n=n, nf=nf, bn=bn: [o.jac_block(Uq, int(n), k, bn, I.n_sol_points(
                int(m.elem_type[k]), p) * ph.nvars) for k in [int(n)] + [int(x) for x in m.nbr[n, :nf]]])
            t_b += t
            refs[int(n)] = r
        _threads(omp, 1)
        t_r1, _ = clock(lambda: o.rhs(Uq))
        n0 = int(el[0])
        nf0 = 3 if m.elem_type[n0] == I.TRI else 4
        bn0 = I.n_sol_points(int(m.elem_type[n0]), p) * ph.nvars
        t_b1, _ = clock(lambda: [o.jac_block(Uq, n0, k, bn0, I.n_sol_points(int(m.elem_type[k]), p) * ph.nvars)
                                 for k in [n0] + [int(x) for x in m.nbr[n0, :nf0]]])
        _threads(omp, cores)
        frac_time_all += t_r + t_b * m.n_elem / len(el)
        frac_time_one += t_r1 + t_b1 * m.n_elem
        dof_sampled += Um.size
        ctx = fr.Context(m, ph, "f32", tri_pts=tp)
        Ud = torch.from_numpy(Uq).float().cuda()
        R = ctx.rhs(Ud)
        B = ctx.jacobian_blocks(Ud)
        ctx.sync()
        errs.append(_rel(R.double().cpu().numpy().reshape(-1), Rref))
        for n in el:
            nf = 3 if m.elem_type[n] == I.TRI else 4
            s0 = np.max(np.abs(refs[int(n)][0]))
            for sl in range(1 + nf):
                g = ctx.block(B, int(n), sl).double().cpu().numpy().T
                errs.append(float(np.max(np.abs(g - refs[int(n)][sl])) / s0))
        del ctx, B, R, o
    rows["cfg3"] = {"workload": "64 mixed triangle/quadrilateral 2-D Euler meshes, p 1-4 (185k elements): R + all "
                                "blocks; GPU FP32 (batched, tuned: the main line's batch entry), oracle FP64",
                    "oracle_1core_dof_s": dof_sampled / frac_time_one, "oracle_allcore_dof_s": dof_sampled / frac_time_all,
                    "max_rel_error": max(errs),
                    "sample": f"meshes {sorted(int(x) for x in picks)}: full R, the blocks of 8 seeded elements each "
                              "(one element on one thread), extrapolated per mesh; DOF/s over those two meshes"}
    log(f"cpu table cfg3: {rows['cfg3']}")

    # ---- one Newton-GMRES step with block Jacobi on 64^2 NS p=3
    ph = I.ns_physics(2, reynolds=1000.0, prandtl=0.72)
    p = 3
    m = I.quad_mesh(64, degree=p, jitter=0.05)
    U = I.ns2d_state(m, p, seeds=(8, 108, 208))
    dt = _dt(m, U, 5.0)
    b = U.shape[1] * U.shape[2]
    o = O.Oracle(m, ph, p)
    Uf = U.reshape(-1)

    def setup():
        return o.jac_blocks(Uf, np.arange(m.n_elem), b, 4)[:, 0]
    t_set, blocks = clock(setup)
    t_it, (Uc, hist, its) = clock(lambda: ON.newton_gmres(o, Uf, dt, b, precond_blocks=blocks, maxit=3000))
    t_all = t_set + t_it
    _threads(omp, 1)
    t_set1, _ = clock(lambda: o.jac_blocks(Uf, np.arange(0, m.n_elem, 16), b, 4))
    t_it1, (_, _, its5) = clock(lambda: ON.newton_gmres(o, Uf, dt, b, precond_blocks=blocks, maxit=5,
                                                        newton_maxit=1))
    _threads(omp, cores)
    t_one = t_set1 * 16 + t_it1 / max(its5, 1) * its
    ctx = fr.Context(m, ph, "f64")
    Ud = torch.from_numpy(U).cuda()
    sol = fr.Solver(ctx, restart=30)
    pc = fr.Precond(ctx)
    sol.newton_step(Ud, pc=pc, dt=dt, gmres_maxit=3000, newton_maxit=12, check=False)
    rg = sol.newton_step(Ud, pc=pc, dt=dt, gmres_maxit=3000, newton_maxit=12, check=False)
    torch.cuda.synchronize()
    rows["cfg4"] = {"workload": "one backward-Euler Newton step to 1e-8 relative, GMRES(30) forcing 1e-3, FP64 block "
                                "Jacobi, 2-D NS p=3 on 64^2 quads at CFL 5 (the 256^2 workload scaled down)",
                    "oracle_allcore_s": t_all, "oracle_gmres_iters": its, "oracle_newton_iters": len(hist) - 1,
                    "oracle_1core_s": t_one, "gpu_s": rg["ms"] / 1e3,
                    "gpu_gmres_iters": rg["gmres_iters"], "gpu_newton_iters": rg["newton_iters"],
                    "update_rel_difference": float(np.max(np.abs(rg["U"].cpu().numpy().reshape(-1) - Uc)) /
                                                   max(np.max(np.abs(Uc - Uf)), 1e-300)),
                    "sample": "all cores: the whole step; one thread: the diagonal blocks of every 16th element "
                              "(x16) and the first 5 GMRES iterations (per iteration x the all-core count)"}
    log(f"cpu table cfg4: {rows['cfg4']}")
    return rows


def budget_sample(ne, budget_s, per_elem_s, cores, rng):
    """Seeded element sample sized to about budget_s of oracle time."""
    n = int(max(cores, min(ne, budget_s * cores / per_elem_s)))
    return np.sort(rng.choice(ne, n, replace=False))


def cfg2_workload():
    from paper_2105_08632_amd import inputs as I
    p, N = 3, 24
    m = I.hex_mesh(N, degree=p, jitter=0.05)
    ph = I.ns_physics(3, 1600.0, 0.71)
    U = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    return m, ph, p, U


def _timed_steps(torch, ctx, step, steps, warmup):
    """warmup untimed steps, then steps timed with the host clock and HIP
    events (the context stream is torch's current stream); the dominant
    kernels (tables + assembly) are bracketed by the library's own events."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.sync()
    ctx.set_kernel_timing(True)
    ctx.kernel_time(0)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    jac_ms, jac_n = ctx.kernel_time(0)
    ctx.set_kernel_timing(False)
    return wall, ev0.elapsed_time(ev1), jac_ms / max(jac_n, 1)


def _roofline(ctx, kernel_ms, bytes_out, traffic_file, kernel_name, ms_per_step):
    per_launch = jac_bytes_per_element(ctx.ns, ctx.nv, ctx.info.ndim, ctx.nf, ctx.nface, bytes_out) * ctx.ne
    achieved = per_launch / (kernel_ms * 1e-3) / 1e9
    # one step: the Jacobian's bytes plus the residual written once (U and
    # the geometry are read once by a fused step)
    step_bytes = per_launch + ctx.ndof * 4
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(traffic_file),
            "kernel": kernel_name, "kernel_ms": round(kernel_ms, 4), "alg_bytes_per_launch": per_launch,
            "step_alg_bytes": step_bytes,
            "step_frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def cfg1_bench(torch, fr, steps, warmup, log):
    """2-D NS p=3 on 128x128 quads: R(U) + the five 64x64 FP32 blocks per element."""
    m, ph, p, U = workload()
    Ud = torch.from_numpy(U).to(torch.float32).cuda().contiguous()
    ctx = fr.Context(m, ph, "f32")
    R = ctx.empty_state()
    B = ctx.block_tensor("f32")

    def step():
        ctx.rhs(Ud, R)
        ctx.jacobian_blocks(Ud, B, "f32")

    wall, gpu_ms, kms = _timed_steps(torch, ctx, step, steps, warmup)
    ms = 1e3 * wall / steps
    out = {"workload": "2D Navier-Stokes FR-DG p=3, 128x128 jittered periodic quads, R(U) + 5 Jacobian blocks "
                       "64x64 per element (FP32 blocks, FP64 residual)",
           "n_elem": ctx.ne, "dof": ctx.ndof, "ms_per_step": round(ms, 4), "dof_per_s": ctx.ndof / (ms * 1e-3),
           "roofline": _roofline(ctx, kms, 4, "k_jac_mf_ns2d_p3_128_traffic.json",
                                 "k_jac_mf_tab + k_jac_mf_asm (quads p=3)", ms)}
    log(f"cfg1: {ms:.4f} ms per step, Jacobian kernels {kms:.4f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-newton", action="store_true", help="skip the Newton-GMRES part of the metric")
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed-mesh batch measurement")
    ap.add_argument("--no-cfg1", action="store_true", help="skip the 2-D quadrilateral measurement")
    ap.add_argument("--no-lu", action="store_true", help="skip the block-Jacobi LU of the 3-D blocks")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16 block assembly")
    ap.add_argument("--only", choices=["cfg2", "cfg2_bf16", "cfg1", "lu", "newton", "mlp", "batch"], default=None,
                    help="time only this workload's step: the 3-D step with FP32 or BF16 blocks, the 2-D "
                         "step, the block-Jacobi LU of the 3-D blocks, one LU-preconditioned Newton step "
                         "on 256x256 (host-driven, then graph-replayed), --mlp-steps steps of network "
                         "training, or the 64-mesh mixed batch (profiling runs)")
    ap.add_argument("--mlp-steps", type=int, default=24000)
    ap.add_argument("--cpu-table", action="store_true",
                    help="time the oracle on one thread and on all host threads beside the GPU for the 8x8 "
                         "advection case, the 128^2 step, the mixed batch and a 64^2 Newton step (prints one "
                         "JSON line; a few minutes of host time)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the timed region, launch a plain device copy of MIB MiB three times "
                         "(calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE against known bytes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py drives exactly one GPU: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731

    import torch
    from paper_2105_08632_amd import fr
    from paper_2105_08632_amd import inputs as I

    if args.cpu_table:
        print(json.dumps(cpu_table(torch, fr, I, log, args.cpu_seconds)), flush=True)
        return
    if args.only == "newton":
        print(json.dumps(newton_step_profile(torch, fr, I, log)), flush=True)
        return
    if args.only == "batch":
        print(json.dumps(batch_bench(torch, fr, I, 5, log)), flush=True)
        return
    if args.only == "mlp":
        _, info = train_mlp(torch, fr, I, args.mlp_steps, log)
        info["ms_per_step"] = round(1e3 * info["train_s"] / args.mlp_steps, 4)
        print(json.dumps(info), flush=True)
        return
    if args.only == "cfg1":
        out = cfg1_bench(torch, fr, args.steps, args.warmup, log)
        if args.copy_probe > 0:
            _copy_probe(torch, args.copy_probe)
        print(json.dumps(out), flush=True)
        return

    # ---- headline: 3-D NS p=3 on 24^3 hexahedra, R(U) + seven 320x320 FP32 blocks per element
    m, ph, p, U = cfg2_workload()
    dev = torch.device("cuda:0")
    Ud = torch.from_numpy(U).to(torch.float32).to(dev).contiguous()
    ctx = fr.Context(m, ph, "f32")
    R = ctx.empty_state()
    B = ctx.block_tensor("f32")
    dof = ctx.ndof

    if args.only == "lu":
        out = block_lu_bench(torch, fr, ctx, U, Ud, R, log)
        if args.copy_probe > 0:
            _copy_probe(torch, args.copy_probe)
        print(json.dumps(out), flush=True)
        return
    if args.only == "cfg2_bf16":
        del B
        torch.cuda.empty_cache()
        B16 = ctx.block_tensor("bf16")

        def step16():
            ctx.rhs(Ud, R)
            ctx.jacobian_blocks(Ud, B16, "bf16")

        w16, g16, k16 = _timed_steps(torch, ctx, step16, args.steps, args.warmup)
        ms16 = 1e3 * w16 / args.steps
        out = {"ms_per_step": round(ms16, 4), "kernel_ms": round(k16, 4)}
        if args.copy_probe > 0:
            _copy_probe(torch, args.copy_probe)
        print(json.dumps(out), flush=True)
        return

    def step():
        ctx.rhs(Ud, R)
        ctx.jacobian_blocks(Ud, B, "f32")

    wall, gpu_ms, kms = _timed_steps(torch, ctx, step, args.steps, args.warmup)
    ms_per_step = 1e3 * wall / args.steps
    roof = _roofline(ctx, kms, 4, "k_jac_mf_ns3d_hex_p3_24_traffic.json",
                     "k_jac_mf_tab + k_jac_mf_asm (Jacobian tables + matrix-core block assembly, hexes p=3)",
                     ms_per_step)
    log(f"cfg2 f32: {ms_per_step:.3f} ms per step, Jacobian kernels {kms:.3f} ms")
    out = {"metric": METRIC, "value": dof * args.steps / wall, "unit": "DOF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "3D Navier-Stokes FR-DG p=3, 24^3 jittered periodic hexahedra (Taylor-Green, "
                                  "Re 1600, Ma 0.1), R(U) + 7 Jacobian blocks 320x320 per element (FP32 blocks, "
                                  "FP64 residual arithmetic)",
                      "n_elem": ctx.ne, "dof": dof, "gpu_ms_per_step": round(gpu_ms / args.steps, 4)},
           "roofline": roof}
    if args.copy_probe > 0:
        _copy_probe(torch, args.copy_probe)
    if args.only == "cfg2":
        print(json.dumps(out), flush=True)
        return

    # outputs kept for the oracle comparison (the CPU leg): R, a JVP, and the
    # blocks of a seeded element sample
    rng = np.random.default_rng(0)
    omp = _omp()
    cores = omp.omp_get_max_threads() if omp else (os.cpu_count() or 1)
    sample = budget_sample(ctx.ne, args.cpu_seconds, 8.0, cores, rng)
    v = I.random_direction(U.shape, 1)
    vd = torch.from_numpy(v).to(torch.float32).cuda().contiguous()
    Jv = ctx.jvp(Ud, vd)
    sel = torch.from_numpy(sample).cuda()
    kept = {"R": R.double().cpu().numpy(), "Jv": Jv.double().cpu().numpy(),
            "blocks": {"f32": (sample, B[sel].double().cpu().numpy())}}
    ctx.sync()
    del B
    torch.cuda.empty_cache()
    if not args.no_bf16:
        B16 = ctx.block_tensor("bf16")

        def step16():
            ctx.rhs(Ud, R)
            ctx.jacobian_blocks(Ud, B16, "bf16")

        w16, g16, k16 = _timed_steps(torch, ctx, step16, args.steps, args.warmup)
        ms16 = 1e3 * w16 / args.steps
        out["bf16"] = {"ms_per_step": round(ms16, 4), "dof_per_s": dof / (ms16 * 1e-3),
                       "roofline": _roofline(ctx, k16, 2, "k_jac_mf_ns3d_hex_p3_24_bf16_traffic.json",
                                             "k_jac_mf_tab + k_jac_mf_asm, BF16 operands and blocks", ms16)}
        log(f"cfg2 bf16: {ms16:.3f} ms per step, Jacobian kernels {k16:.3f} ms")
        kept["blocks"]["bf16"] = (sample, B16[sel].double().cpu().numpy())
        del B16
        torch.cuda.empty_cache()
    if not args.no_lu:
        out["block_lu"] = block_lu_bench(torch, fr, ctx, U, Ud, R, log)
    del ctx, R
    torch.cuda.empty_cache()
    if not args.no_cfg1:
        out["cfg1"] = cfg1_bench(torch, fr, args.steps, args.warmup, log)
        torch.cuda.empty_cache()
    if not args.no_batch:
        out["batch"] = batch_bench(torch, fr, I, 5, log)
        torch.cuda.empty_cache()
    out["fourier"] = fourier_bench(torch, fr, I, log)
    out["rk54_pm"] = rk54_pm_bench(torch, fr, I, log)
    torch.cuda.empty_cache()
    if not args.no_newton:
        out["newton"] = newton_bench(torch, fr, I, args.mlp_steps, log)
    if not args.no_cpu_baseline:
        U32 = U.astype(np.float32).astype(np.float64)
        v32 = v.astype(np.float32).astype(np.float64)
        out["cpu_baseline"], out["errors_vs_oracle"] = cpu_baseline(
            m, ph, p, U32, kept["R"], kept["Jv"], v32, kept["blocks"], args.cpu_seconds, log)
        out["errors_vs_oracle"]["metric"] = ("normwise relative: max |x - x_oracle| / max |x_oracle| per output "
                                             "(blocks: per sampled element, largest), oracle at the GPU's FP32 "
                                             "inputs; bars FP32 1e-5, BF16 2e-2")
    print(json.dumps(out), flush=True)


def _copy_probe(torch, mib):
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def block_lu_bench(torch, fr, ctx, U, Ud, R, log):
    """FP64 block-Jacobi of the 3-D blocks: the diagonal blocks of
    I - dt dR/dU (FP32 assembly) and the LU of each 320x320 block in FP64
    (setup), then one application."""
    N = round(ctx.ne ** (1.0 / 3.0))
    rho = U[..., 0]
    v = U[..., 1:4] / rho[..., None]
    pr = 0.4 * (U[..., 4] - 0.5 * rho * np.sum(v * v, axis=-1))
    dt = 5.0 / N / float(np.max(np.linalg.norm(v, axis=-1) + np.sqrt(1.4 * pr / rho)))
    pc = fr.Precond(ctx)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    pc.setup(Ud, 1.0, -dt)
    torch.cuda.synchronize()
    ctx.set_kernel_timing(True)
    ctx.kernel_time(0)
    t_setup = timed(lambda: pc.setup(Ud, 1.0, -dt), 2)
    ctx.sync()
    jac_ms, jac_n = ctx.kernel_time(0)            # the diagonal-block assembly inside each setup
    ctx.set_kernel_timing(False)
    z = ctx.empty_state()
    t_apply = timed(lambda: pc.apply(R, z), 5)
    flop = ctx.ne * (2.0 / 3.0) * ctx.b ** 3
    lu_ms = t_setup - jac_ms / max(jac_n, 1)       # one timed assembly launch per setup
    tflops = flop / (lu_ms * 1e-3) / 1e12
    out = {"setup_ms": round(t_setup, 2), "apply_ms": round(t_apply, 3), "lu_gflop": round(flop / 1e9, 1),
           "lu_ms": round(lu_ms, 2),
           "roofline": {"bound": "fp64", "achieved": round(tflops, 2), "peak": 78.6, "unit": "TFLOP/s",
                        "frac": round(tflops / 78.6, 4), "kernel": "k_block_lu",
                        "traffic": measured_traffic("k_block_lu_hex_p3_24_traffic.json", "k_block_lu")},
           "note": "setup = diagonal blocks (FP32) + FP64 LU of each; lu_ms = setup minus the timed assembly",
           "finite": bool(torch.isfinite(z).all())}
    log(f"cfg2 block LU: setup {out['setup_ms']} ms, apply {out['apply_ms']} ms")
    pc.close()
    return out


if __name__ == "__main__":
    main()
