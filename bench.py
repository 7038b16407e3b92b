#!/usr/bin/env python3
"""Benchmark of the FR-DG residual + Jacobian-block assembly on one MI355X.

Workload: 2-D compressible Navier-Stokes (gamma 1.4, Re 1000, Pr 0.72), FR-DG
degree 3 on a 128x128 periodic quad mesh with 5% sinusoidal vertex jitter,
Rusanov + BR1 fluxes, smooth random state (rho = 1 + 0.1 s, Mach 0.2).  One
step = R(U) plus the five 64x64 Jacobian blocks of every element (FP32 block
storage), inputs resident in HBM.  Prints one JSON line.

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


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fr_kernels.hpp", "fr_jac_tp.hpp", "fr_jac_mf.hpp", "physics.hpp", "dual.hpp", "fr_impl.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2105_08632_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(per_launch_alg):
    """HBM bytes per launch of the block-assembly kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_jac_mf_ns2d_p3_128_traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
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


def newton_bench(torch, fr, I, train_steps, log):
    """Seconds per backward-Euler Newton step (to |F| <= 1e-8 |F0|, GMRES(30),
    forcing 1e-3) on 256x256 NS p=3: FP64 block-Jacobi LU vs the learned
    preconditioner, each set up at U^n (setup time included)."""
    net, info = train_mlp(torch, fr, I, train_steps, log)
    ph = I.ns_physics(2, reynolds=1000.0, prandtl=0.72)
    m = I.quad_mesh(256, degree=3, jitter=0.05)
    out = {"workload": "2D NS p=3, 256x256 jittered periodic quads (4.19 M DOF), backward Euler, Newton to "
                       "1e-8 relative, GMRES(30) forcing 1e-3, preconditioner set up at U^n; restart cycles "
                       "replayed from a captured hipGraph (lu_host_arnoldi: host-driven Arnoldi for comparison)",
           "mlp_training": info}
    runs = {"lu": [], "mlp": []}
    held = []
    cfl = 5.0
    for s in (8, 9, 10):
        U = I.ns2d_state(m, 3, seeds=(s, 100 + s, 200 + s))
        ctx = fr.Context(m, ph, "f64")
        Ud = torch.from_numpy(U).cuda()
        dt = _dt(m, U, cfl)
        sol = fr.Solver(ctx, restart=30)
        pcm = fr.Precond(ctx, fr.FR_PC_MLP)
        pcm.set_mlp(net, 1e30)
        Xh, _ = pcm.mlp_inputs(Ud, 1.0, -dt)
        held.append(float(torch.cat([net.loss_grad(Xh[i:i + 4096].contiguous())[2]
                                     for i in range(0, Xh.shape[0], 4096)]).mean().item()))
        del Xh
        pcl = fr.Precond(ctx)
        for name, pc, graph in (("lu", pcl, True), ("lu_host_arnoldi", pcl, False), ("mlp", pcm, True)):
            r = sol.newton_step(Ud, pc=pc, dt=dt, gmres_maxit=3000, newton_maxit=12, check=False, use_graph=graph)
            runs.setdefault(name, []).append(r)
            log(f"newton cfl {cfl} seed {s} {name}: conv {r['converged']} newton {r['newton_iters']} "
                f"gmres {r['gmres_iters']} s {r['ms'] / 1e3:.3f}")
        if s == 8:
            hard = {}
            for name, pc in (("lu", fr.Precond(ctx)), ("mlp", pcm)):
                r = sol.newton_step(Ud, pc=pc, dt=_dt(m, U, 100.0), gmres_maxit=3000, newton_maxit=12, check=False,
                                    use_graph=True)
                hard[name] = {"converged": bool(r["converged"]), "newton_iters": r["newton_iters"],
                              "gmres_iters": r["gmres_iters"], "final_rel_residual": r["res"] / r["res0"],
                              "s": round(r["ms"] / 1e3, 3)}
                log(f"newton cfl 100 {name}: conv {r['converged']} rel {r['res'] / r['res0']:.2e}")
            out["cfl100"] = hard
        del sol, pcm, ctx
    # CFL 100 on 64x64, where GMRES(30) with a one-level block preconditioner
    # still converges; plain and loose GMRES (3 of each cycle's 30 directions
    # are earlier cycles' corrections)
    m64 = I.quad_mesh(64, degree=3, jitter=0.05)
    U = I.ns2d_state(m64, 3, seeds=(8, 108, 208))
    ctx = fr.Context(m64, ph, "f64")
    Ud = torch.from_numpy(U).cuda()
    sol = fr.Solver(ctx, restart=30)
    pcm = fr.Precond(ctx, fr.FR_PC_MLP)
    pcm.set_mlp(net, 1e30)
    pcl = fr.Precond(ctx)
    small = {}
    for name, pc, aug in (("lu", pcl, 0), ("lu_loose3", pcl, 3), ("mlp", pcm, 0), ("mlp_loose3", pcm, 3)):
        r = sol.newton_step(Ud, pc=pc, dt=_dt(m64, U, 100.0), gmres_maxit=3000, newton_maxit=12, check=False,
                            augment=aug)
        small[name] = {"converged": bool(r["converged"]), "newton_iters": r["newton_iters"],
                       "gmres_iters": r["gmres_iters"], "final_rel_residual": r["res"] / r["res0"],
                       "s": round(r["ms"] / 1e3, 3)}
        log(f"newton cfl 100 64x64 {name}: conv {r['converged']} gmres {r['gmres_iters']} s {r['ms'] / 1e3:.3f}")
    out["cfl100_64x64"] = small
    del sol, pcm, pcl, ctx
    for name, rs in runs.items():
        out[name] = {"s_per_step_median": round(float(np.median([r["ms"] for r in rs])) / 1e3, 4),
                     "converged": [bool(r["converged"]) for r in rs],
                     "newton_iters": [r["newton_iters"] for r in rs], "gmres_iters": [r["gmres_iters"] for r in rs]}
    out["cfl"] = cfl
    out["mlp_heldout_resid_mean"] = round(float(np.mean(held)), 3)
    out["learned_over_lu_time"] = round(out["mlp"]["s_per_step_median"] / out["lu"]["s_per_step_median"], 3)
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
    alg = 0
    for c in ctxs:
        alg += c.ne * ((1 + c.nface) * c.b * c.b * 4 + c.ns * c.nv * 4 * 2 +
                       (2 * c.ns * 4 + c.ns + c.nf * 2 + c.nf + c.nf) * 4 + c.nface * 4)
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
    return {"workload": "64 periodic 2-D Euler meshes (isentropic vortex), FP32, triangles and quadrilaterals, "
                        "p 1-4, 500-5000 elements each: R(U) + all Jacobian blocks",
            "meshes": len(ctxs), "elements": int(sum(c.ne for c in ctxs)), "dof": int(dof),
            "alg_bytes": int(alg), "hbm_floor_ms": round(floor_ms, 3),
            "ms_per_mesh_calls": round(t_alone, 3), "ms_batched_default": round(t_batch, 3),
            "ms_batched_tuned": round(t_tuned, 3), "tune_s": round(t_tune, 2),
            "dof_per_s_tuned": dof / (t_tuned * 1e-3), "frac_of_hbm_floor": round(floor_ms / t_tuned, 4),
            "tuning": table, "outputs_finite": finite}


def hex3d_bench(torch, fr, I, reps, log):
    """3-D Navier-Stokes FR-DG p=3 on 24^3 jittered periodic hexahedra
    (Taylor-Green vortex, Re 1600): R(U), all seven 320 x 320 Jacobian
    blocks per element in FP32 and BF16, and the FP64 block-Jacobi LU of the
    diagonal blocks (setup from the state, then one application)."""
    p, N = 3, 24
    m = I.hex_mesh(N, degree=p, jitter=0.05)
    ph = I.ns_physics(3, 1600.0, 0.71)
    U = I.tgv_state(m, p, L=1.0 / (2 * np.pi))
    ctx = fr.Context(m, ph, "f32")
    Ud = torch.from_numpy(U).float().cuda().contiguous()
    R = ctx.empty_state()

    def timed(fn, n=reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    out = {"workload": "3D Navier-Stokes FR-DG p=3, 24^3 jittered periodic hexes (Taylor-Green, Re 1600), FP32: "
                       "R(U), 7 Jacobian blocks 320x320 per element, FP64 block-Jacobi LU",
           "n_elem": ctx.ne, "dof": ctx.ndof, "block": ctx.b}
    out["rhs_ms"] = round(timed(lambda: ctx.rhs(Ud, R)), 4)
    for prec, sz in (("f32", 4), ("bf16", 2)):
        B = ctx.block_tensor(prec)
        ctx.set_kernel_timing(True)
        ctx.kernel_time(0)
        t = timed(lambda: ctx.jacobian_blocks(Ud, B, prec))
        ctx.sync()
        kms, kn = ctx.kernel_time(0)
        ctx.set_kernel_timing(False)
        ob = B.numel() * sz
        out["jac_" + prec] = {"ms": round(t, 3), "kernel_ms": round(kms / max(kn, 1), 3), "out_GB": round(ob / 1e9, 2),
                              "out_GB_per_s": round(ob / (t * 1e-3) / 1e9, 1)}
        del B
        torch.cuda.empty_cache()
    out["dof_per_s_rhs_plus_jac_f32"] = ctx.ndof / ((out["rhs_ms"] + out["jac_f32"]["ms"]) * 1e-3)
    rho = U[..., 0]
    v = U[..., 1:4] / rho[..., None]
    pr = 0.4 * (U[..., 4] - 0.5 * rho * np.sum(v * v, axis=-1))
    dt = 5.0 / N / float(np.max(np.linalg.norm(v, axis=-1) + np.sqrt(1.4 * pr / rho)))
    pc = fr.Precond(ctx)
    t_setup = timed(lambda: pc.setup(Ud, 1.0, -dt), 2)
    z = ctx.empty_state()
    t_apply = timed(lambda: pc.apply(R, z))
    flop = ctx.ne * (2.0 / 3.0) * ctx.b ** 3
    out["block_lu"] = {"setup_ms": round(t_setup, 2), "apply_ms": round(t_apply, 3),
                       "lu_gflop": round(flop / 1e9, 1), "note": "setup = diagonal blocks (FP32) + FP64 LU of each",
                       "finite": bool(torch.isfinite(z).all())}
    log(f"hex3d: rhs {out['rhs_ms']} ms, jac f32 {out['jac_f32']['ms']} ms, bf16 {out['jac_bf16']['ms']} ms, "
        f"LU setup {out['block_lu']['setup_ms']} ms, apply {out['block_lu']['apply_ms']} ms")
    pc.close()
    return out


def cpu_baseline(m, ph, p, U, budget_s):
    """The FP64 oracle (as is) on a bounded sample: the full-mesh residual,
    then the five Jacobian blocks of a seeded sample of elements."""
    from oracle import oracle as O
    o = O.Oracle(m, ph, p)
    t0 = time.perf_counter()
    o.rhs(U)
    t_rhs = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    b = 16 * 4
    cal = rng.choice(m.n_elem, 16, replace=False)
    t0 = time.perf_counter()
    o.jac_blocks(U, cal, b, 4)
    t_cal = (time.perf_counter() - t0) / len(cal)
    n = int(max(16, min(m.n_elem, budget_s / max(t_cal, 1e-6))))
    sample = rng.choice(m.n_elem, n, replace=False)
    t0 = time.perf_counter()
    o.jac_blocks(U, sample, b, 4)
    t_blk = time.perf_counter() - t0
    t = t_blk + t_rhs * n / m.n_elem
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n * b / t, "unit": "DOF/s", "cores": cores, "kind": "oracle",
            "sample": f"full-mesh R ({t_rhs:.2f} s, scaled to the sample) + 5 Jacobian blocks of {n} of "
                      f"{m.n_elem} elements ({t_blk:.1f} s); FP64, complex-step columns"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-newton", action="store_true", help="skip the Newton-GMRES part of the metric")
    ap.add_argument("--no-batch", action="store_true", help="skip the mixed-mesh batch measurement")
    ap.add_argument("--no-hex", action="store_true", help="skip the 3-D hexahedral measurement")
    ap.add_argument("--mlp-steps", type=int, default=24000)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the timed region, launch a plain device copy of MIB MiB three times "
                         "(calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE against known bytes)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py drives exactly one GPU: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2105_08632_amd import fr

    m, ph, p, U = workload()
    dev = torch.device("cuda:0")
    Ud = torch.from_numpy(U).to(torch.float32).to(dev).contiguous()
    ctx = fr.Context(m, ph, "f32")
    R = ctx.empty_state()
    B = ctx.block_tensor("f32")
    dof = ctx.ndof

    def step():
        ctx.rhs(Ud, R)
        ctx.jacobian_blocks(Ud, B, "f32")

    for _ in range(args.warmup):
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
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()
    jac_ms, jac_n = ctx.kernel_time(0)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = 1e3 * wall / args.steps

    per_launch = jac_bytes_per_element(ctx.ns, ctx.nv, 2, ctx.nf, ctx.nface) * ctx.ne
    avg_jac_s = jac_ms / max(jac_n, 1) / 1e3
    achieved = per_launch / avg_jac_s / 1e9
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(per_launch),
            "kernel": "k_jac_mf_tab + k_jac_mf_asm (Jacobian tables + matrix-core block assembly)",
            "kernel_ms": round(avg_jac_s * 1e3, 4),
            "alg_bytes_per_launch": per_launch}
    out = {"metric": METRIC, "value": dof * args.steps / wall, "unit": "DOF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "2D Navier-Stokes FR-DG p=3, 128x128 jittered periodic quads, "
                                  "R(U) + 5 Jacobian blocks 64x64 per element (FP32 blocks, FP64 residual)",
                      "n_elem": ctx.ne, "dof": dof, "gpu_ms_per_step": round(gpu_ms / args.steps, 4)},
           "roofline": roof}
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_batch or not args.no_newton or not args.no_hex:
        del B, R
        torch.cuda.empty_cache()
    if not args.no_batch:
        from paper_2105_08632_amd import inputs as I
        out["batch"] = batch_bench(torch, fr, I, 5, lambda s: print(s, file=sys.stderr, flush=True))
        torch.cuda.empty_cache()
    if not args.no_hex:
        from paper_2105_08632_amd import inputs as I
        out["hex3d"] = hex3d_bench(torch, fr, I, 3, lambda s: print(s, file=sys.stderr, flush=True))
        torch.cuda.empty_cache()
    if not args.no_newton:
        from paper_2105_08632_amd import inputs as I
        out["newton"] = newton_bench(torch, fr, I, args.mlp_steps, lambda s: print(s, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, ph, p, U, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
