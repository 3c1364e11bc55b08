#!/usr/bin/env python3
"""IFE-CGP benchmark on one MI355X.

Workload: flow past a cylinder (radius 0.05 at (0.2, 0.2)) in a 2.2 x 0.41
channel, Re = 100, dt = 1e-3; seeded coarse mesh of ~250k P1 triangles, fine
mesh of ~1M triangles after one 1:4 subdivision (l = 1), injection
restriction and consistent-mass correction (the paper's scheme).  A step is
one pass of the whole CGP path: convective assembly and momentum solve on the
fine mesh, restriction and coarse divergence, coarse pressure Poisson solve,
prolongation, velocity correction.

Warm-up steps develop the flow from an impulsive start with the plain FP64
path; the next steps, also plain FP64, are recorded as training data (Poisson
right-hand sides and pressures) for the POD basis and the two networks of the
learned initial guess, which are then built and trained on the GPU.  Every
path is then timed from the same state, all with PCG to a relative residual of
1e-8:
  * fp64:                plain FP64 CGP, x0 = previous pressure;
  * fp64+pod_galerkin:   x0 = previous pressure + Galerkin correction in the POD space;
  * fp64+learned:        x0 from the absolute network;
  * fp64+learned_corr:   x0 = previous pressure + the incremental network's correction;
  * fp64+online_pod:     Galerkin guess in a POD basis rebuilt after every solve from the last
                         solutions (a recycled Krylov subspace);
  * mixed, mixed+online_pod, mixed+learned_corr: FP32 PCG inside FP64 iterative refinement.
Per path: steps/s over the timed steps, per-phase times averaged over them,
max |u| and kinetic energy at the first and last timed step (the flow stays
bounded), and the one-step error against plain FP64 from the same state both
right after the restart and at the end of the timed window.  ``value`` is the
steps/s of the fastest path whose errors are within 1e-6; every path is listed.
Beside it: the paper's coarsening levels l = 0..3 on one fine mesh, the
backward-facing step at l = 1 and l = 0, SpMV and PCG size sweeps, the batched
sweep, and the FP64 oracle on the host cores (one thread and OpenMP).
One JSON line goes to stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0
ERR_BAR = 1e-6
# measured launch shapes of the batched Poisson kernel per size class (cgp_batch_autotune's cache)
TUNING_CACHE = ROOT / "paper_1610_06993_amd" / "tuning" / "batch_tuning.json"


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    import numpy as np
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


# sources that define the Poisson iteration kernels and what they compile against: a change to any of
# them invalidates the HBM counters recorded for those kernels
KERNEL_SOURCES = ("krylov.hip", "devutil.h", "internal.h", "kernels.h")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update((ROOT / "paper_1610_06993_amd" / "csrc" / name).read_bytes())
    return h.hexdigest()[:16]


def dominant_kernel(precision: str, launch: str, nnz: int, n: int):
    """Name and algorithmic bytes per launch (= per iteration) of the Poisson kernel of a path.

    Each array is counted once per iteration, as if every gathered vector entry came from HBM once."""
    w = 4 if precision == "f32" else 8
    t = "float" if w == 4 else "double"
    if launch == "fused":
        # values + columns per nonzero; per row: row pointer, D^-1, r, w, s, p, x read, x, p, s, r, w written
        return f"k_cg1_iter<{t}>", (w + 4) * nnz + (4 + 6 * w + 5 * w) * n
    if launch == "loop":
        # SpMV + p update: values + columns per nonzero; row pointer, z, p_old read, p_new, q written per row
        return f"k_cg_spmv<{t}>", (w + 4) * nnz + (4 + 4 * w) * n
    # one persistent PCG iteration: the SpMV phase plus x, p, r, q, D^-1 read and x, r, z written
    return f"k_pcg_persistent<{t}>", (w + 4) * nnz + (4 + 12 * w) * n


def run_spmv_sweep(args, log):
    """Fine-mesh SpMV with two right-hand sides (the momentum operator's kernel) on jittered unit squares
    of growing size, past the 256 MB Infinity Cache; plus a plain copy as the attainable ceiling."""
    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    sizes = [(128, 1), (256, 1), (256, 2), (256, 3)] + ([(512, 3)] if args.spmv_large else [])
    out = []
    for n, lev in sizes:
        t0 = time.perf_counter()
        m = cgp.Mesh(W.unit_square_tg(n, seed=1), lev)
        m.assemble(1.0, 0.01, 1e-3)
        nf, nnz = m.info["n_f"], m.info["nnz_f"]
        x = torch.from_numpy(np.random.default_rng(0).normal(size=(nf, 2))).cuda()
        y = torch.zeros_like(x)
        for _ in range(3):
            m.spmv(cgp._native.OP_M_F, x, y)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            m.spmv(cgp._native.OP_M_F, x, y)
        e1.record()
        e1.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        nbytes = 12 * nnz + 36 * nf  # values + columns per nonzero; row pointer, x read, y written per row
        gbs = nbytes / (us * 1e-6) / 1e9
        out.append(dict(fine_nodes=nf, nnz=nnz, mbytes=round(nbytes / 1e6, 1), us=round(us, 2), gbs=round(gbs, 1),
                        frac=round(gbs / HBM_PEAK_GBS, 4)))
        log(f"spmv2 {nf} rows, {nnz} nnz, {nbytes / 1e6:.0f} MB: {us:.1f} us -> {gbs:.0f} GB/s "
            f"({gbs / HBM_PEAK_GBS:.2f} of peak); setup {time.perf_counter() - t0:.1f}s")
        m.close()
        del x, y
    # attainable ceiling: a 2 GiB device-to-device elementwise copy
    n = (2 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.mul(src, 1.0, out=dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    e1.record()
    e1.synchronize()
    copy_gbs = 2 * n * 8 / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9
    log(f"copy ceiling: {copy_gbs:.0f} GB/s ({copy_gbs / HBM_PEAK_GBS:.2f} of peak)")
    del src, dst
    return dict(kernel="k_spmv2 (fine mass matrix, 2 right-hand sides)", points=out, copy_gbs=round(copy_gbs, 1),
                copy_frac=round(copy_gbs / HBM_PEAK_GBS, 4))


def run_cg_sweep(args, log):
    """The fused FP64 PCG iteration on coarse operators of growing size (cylinder meshes without
    refinement): microseconds per iteration and algorithmic GB/s, from the small latency-bound sizes to
    sizes that stream from HBM."""
    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts
    iters = 400
    points = []
    for tris in (250_000, 1_000_000, 4_000_000):
        t0 = time.perf_counter()
        mesh = cgp.Mesh(W.cylinder_channel(tris, seed=3), 0)
        mesh.assemble(1.0, 1e-3, 1e-3)
        n, nnz = mesh.info["n_c"], mesh.info["nnz_c"]
        b = torch.from_numpy(np.random.default_rng(1).normal(size=n)).cuda()
        x = torch.zeros_like(b)
        opts = SolverOpts(tol=1e-300, max_iter=iters, x0_mode=cgp._native.X0_ZERO)
        mesh.poisson_solve(b, x, opts, allow_noconv=True)  # sizes the first chunk: one poll per solve
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        mesh.poisson_solve(b, x, opts, allow_noconv=True)
        torch.cuda.synchronize()
        us = 1e6 * (time.perf_counter() - t1) / iters
        mbytes = (12 * nnz + 92 * n) / 1e6
        gbs = mbytes * 1e3 / us
        points.append(dict(rows=n, nnz=nnz, mbytes=round(mbytes, 1), us_per_iteration=round(us, 2),
                           gbs=round(gbs, 1), frac=round(gbs / HBM_PEAK_GBS, 4)))
        log(f"cg sweep {n} rows, {nnz} nnz, {mbytes:.0f} MB per iteration: {us:.2f} us -> {gbs:.0f} GB/s "
            f"({gbs / HBM_PEAK_GBS:.2f} of peak); setup {t1 - t0:.1f}s")
        mesh.close()
    return dict(kernel="k_cg1_iter<double> (whole PCG iteration, wall time over 400 iterations, host polls included)",
                points=points)


def refined_coarse(coarse, k):
    """The coarse mesh subdivided k times, as a coarse-mesh description (the library's own subdivision,
    read back from a host-only mesh), so that meshes with different l share one fine mesh."""
    import paper_1610_06993_amd as cgp
    import workloads as W
    if k == 0:
        return coarse
    h = cgp.Mesh(coarse, k, host_only=True)
    out = W.CoarseMesh(h.export("xy", k), h.export("tri", k), h.export("bedge", k), h.export("bkind", k),
                       name=f"{coarse.name}_refined{k}", meta=dict(coarse.meta))
    h.close()
    return out


def time_plain_steps(case, coarse, levels, warm, steps, mom_tol, mass_tol, log, label):
    """Plain FP64 CGP (the paper's scheme) from the impulsive start: `warm` untimed steps, then `steps`
    timed ones with per-phase events; steps/s, phase means, Poisson iterations, flow bound."""
    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    from paper_1610_06993_amd import SolverOpts, StepOpts
    X0 = cgp._native
    t0 = time.perf_counter()
    mesh = cgp.Mesh(coarse, levels)
    mesh.assemble(case.rho, case.mu, case.dt)
    info = mesh.info
    xy, vd = mesh.export("xy"), mesh.export("vdir")
    g = torch.from_numpy(case.dirichlet(xy, 0.0)).cuda()
    u = torch.from_numpy(case.initial(xy, vd)).cuda()
    pf = torch.zeros(info["n_f"], dtype=torch.float64, device="cuda")
    pc = torch.zeros(info["n_c"], dtype=torch.float64, device="cuda")
    setup = time.perf_counter() - t0

    def opts(timing=0):
        return StepOpts(momentum=SolverOpts(tol=mom_tol, max_iter=5000, x0_mode=X0.X0_PROJECT),
                        poisson=SolverOpts(tol=1e-8, max_iter=200000),
                        mass=SolverOpts(tol=mass_tol, max_iter=2000), timing=timing)
    for _ in range(warm):
        mesh.step(g, u, pf, pc, opts=opts())
    torch.cuda.synchronize()
    keys = ("ms_momentum", "ms_restrict", "ms_poisson", "ms_prolong", "ms_correct")
    ph = {k: 0.0 for k in keys}
    its = []
    t1 = time.perf_counter()
    for _ in range(steps):
        st = mesh.step(g, u, pf, pc, opts=opts(timing=1))
        its.append(st["p_iters"])
        for k in keys:
            ph[k] += st[k]
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    umax = float(torch.sqrt((u * u).sum(1).max()))
    out = dict(levels=levels, resolution=f"{info['t_f']}:{info['t_c']}", fine_nodes=info["n_f"],
               coarse_nodes=info["n_c"], steps_per_s=round(steps / el, 3), ms_per_step=round(1e3 * el / steps, 3),
               poisson_iters_mean=float(np.mean(its)), phase_ms_mean={k: round(v / steps, 4) for k, v in ph.items()},
               max_abs_u_last=round(umax, 6), timed_steps=[warm + 1, warm + steps], setup_s=round(setup, 2))
    log(f"{label} l={levels} ({out['resolution']}): {out['steps_per_s']} steps/s, Poisson {np.mean(its):.0f} "
        f"iterations / {ph['ms_poisson'] / steps:.2f} ms, momentum {ph['ms_momentum'] / steps:.2f} ms per step; "
        f"max|u| {umax:.3f}")
    mesh.close()
    return out


def run_levels(args, log):
    """The paper's M:N comparison (Section 3, Tables 1 and 4): one fine mesh of ~1M triangles, the
    Poisson equation on the mesh coarsened l = 3, 2, 1 times and on the fine mesh itself (l = 0, the
    standard projection method)."""
    import workloads as W
    base = W.case_cylinder(max(1000, args.target_tris * 4 // 64))
    pts = []
    for l in (3, 2, 1, 0):
        coarse = refined_coarse(base.mesh, 3 - l)
        pts.append(time_plain_steps(base, coarse, l, args.level_warmup, args.level_steps, args.mom_tol, args.mass_tol,
                                    log, "cylinder"))
    l0 = next(p for p in pts if p["levels"] == 0)["steps_per_s"]
    for p in pts:
        p["speedup_vs_l0"] = round(p["steps_per_s"] / l0, 3)
    return dict(workload=f"cylinder channel Re=100, dt=1e-3, plain FP64 CGP (injection, consistent mass), one fine "
                         f"mesh of {pts[0]['resolution'].split(':')[0]} triangles", points=pts)


def run_bfs(args, log):
    """Backward-facing step (Section 3.2): ~51k coarse / ~206k fine triangles, Re = 400, dt = 5e-3,
    CGP with l = 1 and the standard method (l = 0) on the same fine mesh."""
    import workloads as W
    ny = max(4, 2 * round(args.bfs_nx * 21 / 612))
    case = W.case_bfs(nx=args.bfs_nx, ny=ny)
    pts = [time_plain_steps(case, case.mesh, 1, args.level_warmup, args.level_steps, args.mom_tol, args.mass_tol, log,
                            "backward step"),
           time_plain_steps(case, refined_coarse(case.mesh, 1), 0, args.level_warmup, args.level_steps, args.mom_tol,
                            args.mass_tol, log, "backward step")]
    pts[0]["speedup_vs_l0"] = round(pts[0]["steps_per_s"] / pts[1]["steps_per_s"], 3)
    return dict(workload=f"backward-facing step [0,30]x[0,2], {args.bfs_nx}x{ny} cells, Re=400, dt=5e-3, plain FP64",
                points=pts)


def _body_edges(mesh, center=(0.2, 0.2), radius=0.05):
    import numpy as np
    xy, be = mesh.xy, mesh.bedge
    mid = 0.5 * (xy[be[:, 0]] + xy[be[:, 1]])
    return np.where(np.hypot(mid[:, 0] - center[0], mid[:, 1] - center[1]) < 1.2 * radius)[0]


def strouhal(times, lift, diameter=0.1, speed=1.0):
    """Shedding frequency from the upward zero crossings of the lift (linear interpolation) over the
    given history, as St = f D / U; None without two full periods."""
    import numpy as np
    t, c = np.asarray(times), np.asarray(lift) - np.mean(lift)
    ups = [t[k] - c[k] * (t[k + 1] - t[k]) / (c[k + 1] - c[k]) for k in range(len(c) - 1) if c[k] < 0 <= c[k + 1]]
    if len(ups) < 3:
        return None
    return float((len(ups) - 1) / (ups[-1] - ups[0]) * diameter / speed)


def run_gmres(args, log):
    """The paper's Poisson solver against the fused Jacobi-PCG on the benchmark's pressure systems:
    ILU(0)-GMRES(m) with level-scheduled triangular solves (one launch per level) and the fused
    PCG, on the Poisson right-hand side of step 20 of plain CGP, for the full cylinder and a
    16k-triangle one; iterations, ms per solve and ms per iteration (GMRES capped at
    `gmres_max_iter` iterations at the full size)."""
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts, StepOpts
    X0 = cgp._native
    out = []
    for tris, cap in ((16_000, 20000), (args.target_tris, args.gmres_max_iter)):
        case = W.case_cylinder(tris)
        mesh = cgp.Mesh(case.mesh, 1)
        mesh.assemble(case.rho, case.mu, case.dt)
        xy, vd = mesh.export("xy"), mesh.export("vdir")
        g = torch.from_numpy(case.dirichlet(xy, 0.0)).cuda()
        u = torch.from_numpy(case.initial(xy, vd)).cuda()
        n = mesh.info["n_c"]
        pf = torch.zeros(mesh.info["n_f"], dtype=torch.float64, device="cuda")
        pc = torch.zeros(n, dtype=torch.float64, device="cuda")
        o = StepOpts(momentum=SolverOpts(tol=args.mom_tol, max_iter=5000), poisson=SolverOpts(tol=1e-8, max_iter=100000),
                     mass=SolverOpts(tol=args.mass_tol, max_iter=2000))
        for k in range(20):
            mesh.step(g, u, pf, pc, opts=o)
        b = torch.zeros(n, dtype=torch.float64, device="cuda")
        mesh.last_poisson_rhs(b)
        row = dict(coarse_triangles=case.mesh.n_tris, coarse_nodes=n)
        for name, so in (("jacobi_pcg", SolverOpts(tol=1e-8, max_iter=100000, x0_mode=X0.X0_ZERO)),
                         ("ilu0_gmres30", SolverOpts(tol=1e-8, max_iter=cap, x0_mode=X0.X0_ZERO,
                                                     method=X0.METHOD_ILU_GMRES, restart=30)),
                         ("ilu0_gmres60", SolverOpts(tol=1e-8, max_iter=cap, x0_mode=X0.X0_ZERO,
                                                     method=X0.METHOD_ILU_GMRES, restart=60))):
            x = torch.zeros(n, dtype=torch.float64, device="cuda")
            mesh.poisson_solve(b, x, so, allow_noconv=True)  # first solve: factorisation, warm-up
            x.zero_()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = mesh.poisson_solve(b, x, so, allow_noconv=True)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t1)
            row[name] = dict(iterations=st["p_iters"], converged=st["status"] == 0,
                             relres=float(st["p_relres"]), ms=round(ms, 2),
                             ms_per_iteration=round(ms / max(1, st["p_iters"]), 4))
            log(f"Poisson solvers, {case.mesh.n_tris} coarse triangles: {name}: {st['p_iters']} iterations "
                f"({'converged' if st['status'] == 0 else 'capped'}, relres {st['p_relres']:.1e}), {ms:.1f} ms")
        mesh.close()
        out.append(row)
    return dict(workload="Poisson right-hand side of step 20 of plain CGP on cylinder channels (Re 100, l = 1), "
                         "tolerance 1e-8 relative, x0 = 0", points=out)


def run_functionals(args, log):
    """Flow functionals from long runs (Section 3.3, Eq. 42, Table 6, Fig. 13; Section 3.2, Fig. 7):
    drag and lift coefficients (pressure and viscous parts) and the Strouhal number of the cylinder
    flow, and the reattachment length behind the backward-facing step."""
    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts, StepOpts
    X0 = cgp._native
    out = {}
    # cylinder: C = 2 F / (rho U^2 D) with the mean inflow speed U = 1 and D = 0.1
    case = W.case_cylinder(args.target_tris)
    mesh = cgp.Mesh(case.mesh, 1)
    mesh.assemble(case.rho, case.mu, case.dt, args.func_restrict)
    mesh.surface_set(_body_edges(case.mesh))
    xy, vd = mesh.export("xy"), mesh.export("vdir")
    g = torch.from_numpy(case.dirichlet(xy, 0.0)).cuda()
    u = torch.from_numpy(case.initial(xy, vd)).cuda()
    pf = torch.zeros(mesh.info["n_f"], dtype=torch.float64, device="cuda")
    pc = torch.zeros(mesh.info["n_c"], dtype=torch.float64, device="cuda")
    online = cgp.Guess(mesh, n_modes=args.window, hidden=16, seed=5)
    online.set_online(args.window, 1)
    online.attach()
    o = StepOpts(momentum=SolverOpts(tol=args.mom_tol, max_iter=5000, x0_mode=X0.X0_PROJECT),
                 poisson=SolverOpts(tol=1e-8, max_iter=100000, x0_mode=X0.X0_POD_GALERKIN),
                 mass=SolverOpts(tol=args.mass_tol, max_iter=2000))
    hist = []
    t0 = time.perf_counter()
    scale = 2.0 / (case.rho * 1.0 * 1.0 * 0.1)
    for k in range(1, args.func_steps + 1):
        mesh.step(g, u, pf, pc, opts=o)
        if k % args.func_every == 0:
            f = mesh.surface_force(u, pf)
            umax = float(torch.sqrt((u * u).sum(1).max()))
            hist.append([k * case.dt] + [scale * v for v in f] + [umax])
            if k % (50 * args.func_every) == 0:
                log(f"cylinder step {k}: C_D {scale * (f[0] + f[2]):.4f} (pressure {scale * f[0]:.4f}), C_L "
                    f"{scale * (f[1] + f[3]):.4f}, max|u| {umax:.3f}; {time.perf_counter() - t0:.0f}s")
    online.close()
    mesh.close()
    H = np.array(hist)
    tail = H[H[:, 0] >= args.func_steps * case.dt / 2]
    cd, cl = tail[:, 1] + tail[:, 3], tail[:, 2] + tail[:, 4]
    out["cylinder"] = dict(
        workload=f"cylinder channel Re=100, coarse {case.mesh.n_tris} / fine {4 * case.mesh.n_tris} triangles, "
                 f"dt=1e-3, {args.func_steps} steps, restriction {'Galerkin' if args.func_restrict else 'injection'}",
        steps_per_s=round(args.func_steps / (time.perf_counter() - t0), 2),
        second_half=dict(cd_mean=float(cd.mean()), cd_min=float(cd.min()), cd_max=float(cd.max()),
                         cl_min=float(cl.min()), cl_max=float(cl.max()),
                         cl_pressure_max=float(tail[:, 2].max()), cl_viscous_max=float(tail[:, 4].max()),
                         strouhal=strouhal(tail[:, 0], cl), max_abs_u=float(tail[:, 5].max())),
        history_every=args.func_every, history_cd_cl=[[round(r[0], 4), round(r[1] + r[3], 5), round(r[2] + r[4], 5)]
                                                      for r in H[::10]])
    log(f"cylinder: {out['cylinder']['second_half']}")
    # backward-facing step: reattachment point from the floor's viscous traction
    case = W.case_bfs()
    mesh = cgp.Mesh(case.mesh, 1)
    mesh.assemble(case.rho, case.mu, case.dt, args.func_restrict)
    xc, be = case.mesh.xy, case.mesh.bedge
    mesh.surface_set(np.where((xc[be[:, 0], 1] == 0.0) & (xc[be[:, 1], 1] == 0.0))[0])
    xy, vd = mesh.export("xy"), mesh.export("vdir")
    g = torch.from_numpy(case.dirichlet(xy, 0.0)).cuda()
    u = torch.from_numpy(case.initial(xy, vd)).cuda()
    pf = torch.zeros(mesh.info["n_f"], dtype=torch.float64, device="cuda")
    pc = torch.zeros(mesh.info["n_c"], dtype=torch.float64, device="cuda")
    online = cgp.Guess(mesh, n_modes=args.window, hidden=16, seed=5)
    online.set_online(args.window, 1)
    online.attach()
    reat = []
    t0 = time.perf_counter()
    for k in range(1, args.bfs_steps + 1):
        mesh.step(g, u, pf, pc, opts=o)
        if k % 500 == 0:
            rows = mesh.surface_traction(u, pf).cpu().numpy()
            rows = rows[np.argsort(rows[:, 0])]
            tau = rows[:, 5] / rows[:, 2]  # viscous x-traction per unit length on the floor
            r = None
            for q in range(len(tau) - 1):
                if tau[q] < 0.0 <= tau[q + 1] and rows[q, 0] > 0.05:
                    r = float(rows[q, 0] - tau[q] * (rows[q + 1, 0] - rows[q, 0]) / (tau[q + 1] - tau[q]))
                    break
            reat.append([round(k * case.dt, 3), r])
            log(f"backward step step {k}: reattachment x/h {r}; {time.perf_counter() - t0:.0f}s")
    online.close()
    mesh.close()
    out["backward_step"] = dict(
        workload=f"backward-facing step Re=400, coarse {case.mesh.n_tris} / fine {4 * case.mesh.n_tris} triangles, "
                 f"dt=5e-3, {args.bfs_steps} steps", reattachment_x_over_h=reat)
    return out


def run_learned(args, log):
    """The learned initial guess at the shape of the configuration it is specified for: pressure
    snapshots from CGP runs of the cylinder at Re drawn uniformly in [60, 160] (seeded), every
    `learn_stride`-th step after `learn_settle` steps, 64 POD modes, MLPs 64-256-256-64 (GELU, BF16 on
    the matrix cores) trained on the GPU with Adam (lr 1e-3, batch 256); Poisson iterations and solve
    times on held-out Re from x0 = 0, the previous pressure, the POD-Galerkin correction, the absolute
    network and the incremental network (whose basis spans the pressure increments), in FP64 and with
    FP32 inner solves.  The recording runs start each Poisson solve from an online POD basis of the
    run's last 64 solutions (the solutions are the method's to the solver tolerance; only the start
    differs), so that 2000-step runs fit the time budget."""
    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts, StepOpts
    X0 = cgp._native
    n_re, n_test, settle, rec = args.learn_re, args.learn_test_re, args.learn_settle, args.learn_record
    stride, rmode = args.learn_stride, args.learn_restrict
    res = 60.0 + 100.0 * W.uniform01(7, 0, n_re)
    case = W.case_cylinder(args.target_tris)
    mesh = cgp.Mesh(case.mesh, 1)
    n = mesh.info["n_c"]
    xy, vd = mesh.export("xy"), mesh.export("vdir")
    g = torch.from_numpy(case.dirichlet(xy, 0.0)).cuda()
    S = n_re * rec
    B = torch.zeros((S, n), dtype=torch.float64, device="cuda")
    P = torch.zeros_like(B)
    Pp = torch.zeros_like(B)
    window = args.learn_online_window
    o = StepOpts(momentum=SolverOpts(tol=args.mom_tol, max_iter=5000, x0_mode=X0.X0_PROJECT),
                 poisson=SolverOpts(tol=1e-8, max_iter=100000, x0_mode=X0.X0_POD_GALERKIN if window else X0.X0_PREV),
                 mass=SolverOpts(tol=args.mass_tol, max_iter=2000))
    t0 = time.perf_counter()
    max_u = []
    for r, re in enumerate(res):
        mesh.assemble(case.rho, 0.1 / re, case.dt, rmode)
        online = None
        if window:
            online = cgp.Guess(mesh, n_modes=window, hidden=16, seed=5)
            online.set_online(window, 1)
            online.attach()
        u = torch.from_numpy(case.initial(xy, vd)).cuda()
        pf = torch.zeros(mesh.info["n_f"], dtype=torch.float64, device="cuda")
        pc = torch.zeros(n, dtype=torch.float64, device="cuda")
        for k in range(settle + rec * stride):
            j = (k - settle) // stride if k >= settle and (k - settle) % stride == stride - 1 else -1
            if j >= 0:
                Pp[r * rec + j].copy_(pc)
            mesh.step(g, u, pf, pc, opts=o)
            if j >= 0:
                mesh.last_poisson_rhs(B[r * rec + j])
                P[r * rec + j].copy_(pc)
        if online:
            online.detach()
            online.close()
        torch.cuda.synchronize()
        max_u.append(round(float(u.abs().max()), 4))
        log(f"learned study: Re {re:.1f} recorded ({r + 1}/{n_re}), max|u| at the end {max_u[-1]}, "
            f"{time.perf_counter() - t0:.0f}s")
    ntr = (n_re - n_test) * rec
    tr = slice(0, ntr)
    models, train = {}, {}
    for name, incr in (("abs", False), ("incr", True)):
        net = cgp.Guess(mesh, n_modes=64, hidden=256, seed=11)
        snaps = (P[tr] - Pp[tr]).contiguous() if incr else P[tr].contiguous()
        t1 = time.perf_counter()
        net.build_pod(snaps)
        st = net.train(B[tr].contiguous(), P[tr].contiguous(), epochs=args.learn_epochs, batch=256, lr=1e-3,
                       p_prev=Pp[tr].contiguous() if incr else None)
        torch.cuda.synchronize()
        train[name] = dict(loss_first=st["loss_first"], loss_last=st["loss_last"], adam_steps=st["steps"],
                           train_ms=round(st["ms"], 1), pod_and_train_s=round(time.perf_counter() - t1, 2))
        models[name] = net
        log(f"learned study: {name} model loss {st['loss_first']:.3e} -> {st['loss_last']:.3e} in {st['steps']} "
            f"Adam steps ({st['ms']:.0f} ms)")
    # held-out Re: every `learn_eval_every`-th recorded step of each, solved from each initial guess
    test_idx = [i for i in range(ntr, S) if (i - ntr) % args.learn_eval_every == 0]
    modes = {"zero": (X0.X0_ZERO, None, 0), "prev": (X0.X0_PREV, None, 0),
             "pod_galerkin": (X0.X0_POD_GALERKIN, "abs", 0), "learned": (X0.X0_LEARNED, "abs", 0),
             "learned_corr": (X0.X0_LEARNED_CORR, "incr", 0), "mixed+prev": (X0.X0_PREV, None, 1),
             "mixed+learned_corr": (X0.X0_LEARNED_CORR, "incr", 1)}
    mesh.assemble(case.rho, 0.1 / res[ntr // rec], case.dt, rmode)
    out = {}
    for name, (mode, model, prec) in modes.items():
        if model:
            models[model].attach()
        its, ms, errs = [], [], []
        for i in test_idx:
            re_i = res[i // rec]
            if abs(mesh.params["mu"] - 0.1 / re_i) > 0:
                mesh.assemble(case.rho, 0.1 / re_i, case.dt, rmode)  # K does not depend on mu; b is recorded
            x = Pp[i].clone() if mode != X0.X0_ZERO else torch.zeros(n, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st = mesh.poisson_solve(B[i], x, SolverOpts(tol=1e-8, max_iter=100000, x0_mode=mode,
                                                        precision=X0.PREC_FP32_IR if prec else X0.PREC_FP64,
                                                        inner_tol=args.inner_tol))
            ms.append(1e3 * (time.perf_counter() - t1))
            its.append(st["p_iters"])
            errs.append(float(torch.linalg.norm(x - P[i]) / torch.linalg.norm(P[i])))
        if model:
            models[model].detach()
        out[name] = dict(poisson_iters_mean=round(float(np.mean(its)), 1), solve_ms_mean=round(float(np.mean(ms)), 3),
                         rel_err_vs_recorded_max=float(np.max(errs)))
        log(f"learned study, held-out Re: {name}: {np.mean(its):.1f} iterations, {np.mean(ms):.2f} ms per solve, "
            f"max rel diff from the recorded pressure {np.max(errs):.1e}")
    for net in models.values():
        net.close()
    mesh.close()
    return dict(workload=f"cylinder channel, coarse {case.mesh.n_tris} / fine {4 * case.mesh.n_tris} triangles, dt=1e-3, "
                         f"restriction {'Galerkin' if rmode else 'injection'}; {n_re} Re values in [60,160] (seed 7), "
                         f"every {stride}th of steps {settle + 1}-{settle + rec * stride} of each recorded "
                         f"({S} snapshots); the last {n_test} Re held out; Poisson tol 1e-8",
                max_abs_u_end_per_re=max_u,
                train_re=[round(float(v), 2) for v in res[:n_re - n_test]],
                test_re=[round(float(v), 2) for v in res[n_re - n_test:]], samples_evaluated=len(test_idx),
                training=train, guesses=out)


def run_steady(args, log):
    """One continuous run of the online-POD path (not a restart from recorded state): 74 plain steps
    from the impulsive start, then the guess with an empty window that fills as it goes, for each
    Poisson precision; 20-step means of Poisson iterations and steps/s."""
    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts, StepOpts
    X0 = cgp._native
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    case = W.case_cylinder(args.target_tris)
    out = {}
    for name, prec in (("fp64+online_pod", cgp._native.PREC_FP64), ("mixed+online_pod", cgp._native.PREC_FP32_IR)):
        mesh = cgp.Mesh(case.mesh, 1)
        mesh.assemble(case.rho, case.mu, case.dt)
        xy, vdir = mesh.export("xy"), mesh.export("vdir")
        g = torch.from_numpy(case.dirichlet(xy, 0.0)).to(dev)
        u = torch.from_numpy(case.initial(xy, vdir)).to(dev)
        pf = torch.zeros(mesh.info["n_f"], dtype=torch.float64, device=dev)
        pc = torch.zeros(mesh.info["n_c"], dtype=torch.float64, device=dev)

        def opts(x0):
            mx0 = {"prev": X0.X0_PREV, "extrap": X0.X0_EXTRAP, "project": X0.X0_PROJECT}[args.mom_x0]
            return StepOpts(momentum=SolverOpts(tol=args.mom_tol, max_iter=5000, x0_mode=mx0),
                            poisson=SolverOpts(tol=1e-8, max_iter=100000, x0_mode=x0, inner_tol=args.inner_tol,
                                               precision=prec if x0 != X0.X0_PREV else cgp._native.PREC_FP64),
                            mass=SolverOpts(tol=args.mass_tol, max_iter=2000))
        for k in range(74):
            mesh.step(g, u, pf, pc, opts=opts(X0.X0_PREV))
        online = cgp.Guess(mesh, n_modes=args.window, hidden=16, seed=5)
        online.set_online(args.window, args.refresh)
        online.attach()
        torch.cuda.synchronize()
        means = []
        its = []
        t = time.perf_counter()
        for k in range(args.only_steady):
            its.append(mesh.step(g, u, pf, pc, opts=opts(X0.X0_POD_GALERKIN))["p_iters"])
            if (k + 1) % 20 == 0:
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                means.append(dict(steps=[k - 18, k + 1], poisson_iters=float(np.mean(its[-20:])),
                                  max_iters=int(max(its[-20:])), steps_per_s=round(20 / (t1 - t), 1)))
                log(f"steady {name}: steps {k - 18}-{k + 1}: Poisson iterations {np.mean(its[-20:]):.0f} "
                    f"(max {max(its[-20:])}), {20 / (t1 - t):.1f} steps/s")
                t = t1
        out[name] = means
        online.close()
        mesh.close()
    return dict(window=args.window, plain_steps_first=74, blocks=out)


def run_batch_kernel(args, log):
    """Only the batched PCG iteration with every instance active (the sweep's 64 instances, 64 iterations
    from a random right-hand side, three times): the clean dispatches HBM counters are read on."""
    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts
    cases = W.batch_sweep(args.batch)
    meshes = []
    for c in cases:
        m = cgp.Mesh(c.mesh, 1)
        m.assemble(c.rho, c.mu, c.dt)
        meshes.append(m)
    rows = sum(m.info["n_c"] for m in meshes)
    nnz = sum(m.info["nnz_c"] for m in meshes)
    batch = cgp.Batch(meshes)
    TUNING_CACHE.parent.mkdir(exist_ok=True)
    tuned = batch.autotune(TUNING_CACHE)
    rng = np.random.default_rng(0)
    bs = [torch.from_numpy(rng.normal(size=m.info["n_c"])).cuda() for m in meshes]
    xs = [torch.zeros_like(b) for b in bs]
    out = []
    for rep in range(3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        batch.poisson_solve(bs, xs, SolverOpts(tol=1e-300, max_iter=64, x0_mode=0), allow_noconv=True)
        torch.cuda.synchronize()
        out.append(1e6 * (time.perf_counter() - t) / 64)
    kbytes = 12 * nnz + 92 * rows
    log(f"batched PCG kernel, all {len(meshes)} instances active: {out} us per iteration, {kbytes / 1e6:.0f} MB, "
        f"tuning {tuned}")
    batch.close()
    cands = []
    try:
        for key, entry in json.loads(TUNING_CACHE.read_text()).items():
            if key.endswith(f"_inst{len(meshes)}") and "candidates" in entry:
                cands = entry["candidates"]
    except (OSError, ValueError):
        pass
    return dict(rows=rows, nnz=nnz, bytes_per_iteration=kbytes, us_per_iteration=[round(v, 2) for v in out],
                tuning=tuned, autotune_candidates=cands)


def run_batch_long(args, log):
    """The batched sweep as the configuration states it: 64 instances stepped together for
    `batch_long` steps each from the impulsive start, with per-instance online POD guesses and FP32
    inner solves inside FP64 refinement; aggregate steps/s over all the steps, max |u| of every
    instance along the way, and at the end each size-decile instance's one-step error against the FP64
    oracle from the same state (the oracle steps the ten instances on host threads)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import oracle
    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts, StepOpts
    X0 = cgp._native
    t0 = time.perf_counter()
    cases = W.batch_sweep(args.batch)
    meshes, g, u, pf, pc = [], [], [], [], []
    for c in cases:
        m = cgp.Mesh(c.mesh, 1)
        m.assemble(c.rho, c.mu, c.dt)
        xy = m.export("xy")
        meshes.append(m)
        g.append(torch.from_numpy(c.dirichlet(xy, 0.0)).cuda())
        u.append(torch.from_numpy(c.initial(xy, m.export("vdir"))).cuda())
        pf.append(torch.zeros(m.info["n_f"], dtype=torch.float64, device="cuda"))
        pc.append(torch.zeros(m.info["n_c"], dtype=torch.float64, device="cuda"))
    batch = cgp.Batch(meshes)
    TUNING_CACHE.parent.mkdir(exist_ok=True)
    tuned = batch.autotune(TUNING_CACHE)
    guesses = []
    for m in meshes:
        gs = cgp.Guess(m, n_modes=args.batch_window, hidden=16, seed=5)
        gs.set_online(args.batch_window, 1)
        gs.attach()
        guesses.append(gs)
    mom = SolverOpts(tol=args.mom_tol, max_iter=5000, x0_mode=X0.X0_PROJECT)
    opts = StepOpts(momentum=mom, poisson=SolverOpts(tol=1e-8, max_iter=100000, precision=X0.PREC_FP32_IR,
                                                     inner_tol=args.inner_tol, x0_mode=X0.X0_POD_GALERKIN),
                    mass=SolverOpts(tol=args.mass_tol, max_iter=2000))
    log(f"batch long run: {len(meshes)} instances, setup {time.perf_counter() - t0:.1f}s, tuning {tuned}")
    n_steps = args.batch_long
    maxu_hist, iters_hist = [], []
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(n_steps):
        st = batch.step(g, u, pf, pc, opts=opts)
        if (k + 1) % 100 == 0 or k + 1 == n_steps:
            torch.cuda.synchronize()
            mu = [float(x.abs().max()) for x in u]
            maxu_hist.append([k + 1, round(min(mu), 4), round(max(mu), 4)])
            iters_hist.append([k + 1, min(s["p_iters"] for s in st), max(s["p_iters"] for s in st)])
            log(f"batch long run: step {k + 1}, {len(meshes) * (k + 1) / (time.perf_counter() - t1):.1f} "
                f"instance-steps/s so far, max|u| over instances {min(mu):.3f}..{max(mu):.3f}, Poisson inner "
                f"iterations {iters_hist[-1][1]}..{iters_hist[-1][2]}")
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    # one more step of every instance beside the oracle's step from the same state, for the deciles
    idx = W.batch_deciles(args.batch)
    probs = []
    for i in idx:
        o = oracle.Problem(cases[i].mesh, 1)
        o.assemble(cases[i].rho, cases[i].mu, cases[i].dt, 0, 0)
        probs.append(o)
    state = [(u[i].cpu().numpy().copy(), pc[i].cpu().numpy().copy(), g[i].cpu().numpy()) for i in idx]
    batch.step(g, u, pf, pc, opts=opts)
    torch.cuda.synchronize()

    def oracle_step(j):
        uu, pcc, gd = state[j]
        return probs[j].step(gd, uu, pcc, tol_mom=1e-13, tol_p=1e-13, tol_mass=1e-13)

    with ThreadPoolExecutor(max_workers=len(idx)) as pool:
        res = list(pool.map(oracle_step, range(len(idx))))
    errs = []
    for j, i in enumerate(idx):
        ur, pfr, _, code, _ = res[j]
        errs.append(dict(instance=i, coarse_triangles=cases[i].mesh.n_tris, oracle_code=code,
                         rel_err_u=rel(u[i].cpu().numpy(), ur), rel_err_p=rel(pf[i].cpu().numpy(), pfr)))
    for gs in guesses:
        gs.detach()
        gs.close()
    batch.close()
    worst = max(max(e["rel_err_u"], e["rel_err_p"]) for e in errs)
    log(f"batch long run: {n_steps} steps of {len(meshes)} instances in {el:.1f}s = "
        f"{len(meshes) * n_steps / el:.1f} instance-steps/s; size-decile one-step error against the FP64 oracle "
        f"at step {n_steps + 1}: worst {worst:.1e}")
    return dict(workload=f"{len(meshes)} cylinder instances (coarse 15.8k-228k triangles, Re uniform in [60,160]), "
                         f"impulsive start, {n_steps} steps each, per-instance online POD guesses (window "
                         f"{args.batch_window}), FP32 inner Poisson solves inside FP64 refinement to 1e-8",
                steps=n_steps, seconds=round(el, 2), instance_steps_per_s=round(len(meshes) * n_steps / el, 3),
                max_abs_u_min_max_every_100=maxu_hist, poisson_inner_iters_min_max_every_100=iters_hist,
                decile_one_step_error_vs_oracle=errs, worst_rel_err=worst, tuning=tuned)


def run_batch(args, log):
    """Config-4-style sweep: independent cylinder instances of uneven size stepped together."""
    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts, StepOpts
    t0 = time.perf_counter()
    cases = W.batch_sweep(args.batch)
    meshes, g, u, pf, pc = [], [], [], [], []
    for c in cases:
        m = cgp.Mesh(c.mesh, 1)
        m.assemble(c.rho, c.mu, c.dt)
        xy = m.export("xy")
        meshes.append(m)
        g.append(torch.from_numpy(c.dirichlet(xy, 0.0)).cuda())
        u.append(torch.from_numpy(c.initial(xy, m.export("vdir"))).cuda())
        pf.append(torch.zeros(m.info["n_f"], dtype=torch.float64, device="cuda"))
        pc.append(torch.zeros(m.info["n_c"], dtype=torch.float64, device="cuda"))
    rows = sum(m.info["n_c"] for m in meshes)
    nnz = sum(m.info["nnz_c"] for m in meshes)
    t_fine = sum(m.info["t_f"] for m in meshes)
    batch = cgp.Batch(meshes)
    TUNING_CACHE.parent.mkdir(exist_ok=True)
    tuned = batch.autotune(TUNING_CACHE)
    log(f"batch: {len(meshes)} instances, {t_fine} fine triangles, {rows} coarse rows, {nnz} coarse nonzeros; "
        f"setup {time.perf_counter() - t0:.1f}s; autotuned {tuned}")
    tol = 1e-8
    X0 = cgp._native
    mom = SolverOpts(tol=args.mom_tol, max_iter=5000,
                     x0_mode={"prev": X0.X0_PREV, "extrap": X0.X0_EXTRAP, "project": X0.X0_PROJECT}[args.mom_x0])
    opts = StepOpts(timing=1, momentum=mom, poisson=SolverOpts(tol=tol, max_iter=100000),
                    mass=SolverOpts(tol=args.mass_tol, max_iter=2000))
    for k in range(2):
        batch.step(g, u, pf, pc, opts=opts)
    torch.cuda.synchronize()
    su, spc = [x.clone() for x in u], [x.clone() for x in pc]

    def restore():
        for a, b in zip(u, su):
            a.copy_(b)
        for a, b in zip(pc, spc):
            a.copy_(b)
        torch.cuda.synchronize()

    # the sequential reference: one single-instance step of every instance
    restore()
    t1 = time.perf_counter()
    for i, m in enumerate(meshes):
        m.step(g[i], u[i], pf[i], pc[i], opts=opts)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t1
    ref = [(a.cpu().numpy(), b.cpu().numpy()) for a, b in zip(u, pf)]
    # batched steps
    restore()
    st = batch.step(g, u, pf, pc, opts=opts)
    err = max(max(rel(a.cpu().numpy(), r[0]), rel(b.cpu().numpy(), r[1])) for a, b, r in zip(u, pf, ref))
    restore()
    phases = lambda sts: {k: round(float(np.mean([s[0][k] for s in sts])), 2)
                          for k in ("ms_momentum", "ms_poisson", "ms_correct")}
    t1 = time.perf_counter()
    sts = []
    for k in range(args.batch_steps):
        st = batch.step(g, u, pf, pc, opts=opts)
        sts.append(st)
    torch.cuda.synchronize()
    el = time.perf_counter() - t1
    ph_plain = phases(sts)
    iters = [s["p_iters"] for s in st]
    launches = st[0]["n_dominant"]
    # the batched PCG kernel with every instance active: 64 iterations from a random right-hand side
    rng = np.random.default_rng(0)
    bs = [torch.from_numpy(rng.normal(size=m.info["n_c"])).cuda() for m in meshes]
    xs = [torch.zeros_like(b) for b in bs]
    batch.poisson_solve(bs, xs, SolverOpts(tol=1e-300, max_iter=64, x0_mode=0), allow_noconv=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    batch.poisson_solve(bs, xs, SolverOpts(tol=1e-300, max_iter=64, x0_mode=0), allow_noconv=True)
    torch.cuda.synchronize()
    us_it = 1e6 * (time.perf_counter() - t2) / 64
    kbytes = 12 * nnz + 92 * rows
    # every instance with its own online POD basis (the last `batch_window` solutions), which fills during
    # window + 1 untimed batched steps; then the same timed steps
    guesses = []
    for m in meshes:
        gs = cgp.Guess(m, n_modes=args.batch_window, hidden=16, seed=5)
        gs.set_online(args.batch_window, 1)
        gs.attach()
        guesses.append(gs)
    oopts = StepOpts(timing=1, momentum=mom, poisson=SolverOpts(tol=tol, max_iter=100000, x0_mode=X0.X0_POD_GALERKIN),
                     mass=SolverOpts(tol=args.mass_tol, max_iter=2000))
    restore()
    for k in range(args.batch_window + 1):
        batch.step(g, u, pf, pc, opts=oopts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sts = []
    for k in range(args.batch_steps):
        st_on = batch.step(g, u, pf, pc, opts=oopts)
        sts.append(st_on)
    torch.cuda.synchronize()
    el_on = time.perf_counter() - t1
    ph_on = phases(sts)
    iters_on = [s["p_iters"] for s in st_on]
    # the same with every instance's FP32 inner solves batched inside its FP64 refinement
    mopts = StepOpts(timing=1, momentum=mom, poisson=SolverOpts(tol=tol, max_iter=100000, precision=cgp._native.PREC_FP32_IR,
                                                      inner_tol=args.inner_tol, x0_mode=X0.X0_POD_GALERKIN),
                     mass=SolverOpts(tol=args.mass_tol, max_iter=2000))
    batch.step(g, u, pf, pc, opts=mopts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sts = []
    for k in range(args.batch_steps):
        st_mx = batch.step(g, u, pf, pc, opts=mopts)
        sts.append(st_mx)
    torch.cuda.synchronize()
    el_mx = time.perf_counter() - t1
    ph_mx = phases(sts)
    iters_mx = [s["p_iters"] for s in st_mx]
    for gs in guesses:
        gs.detach()
        gs.close()
    batch.close()
    out = dict(instances=len(meshes), fine_triangles=t_fine, coarse_rows=rows, coarse_nnz=nnz,
               instance_steps_per_s=round(len(meshes) * args.batch_steps / el, 3),
               ms_per_batch_step=round(1e3 * el / args.batch_steps, 2),
               sequential_instance_steps_per_s=round(len(meshes) / seq_s, 3),
               speedup_vs_sequential=round(len(meshes) * args.batch_steps / el / (len(meshes) / seq_s), 3),
               poisson_iters_min_max=[min(iters), max(iters)], batched_launches_per_step=launches,
               phase_ms_mean=ph_plain,
               rel_err_vs_single_instance_gpu=err,
               tuning=tuned, batched_kernel_us_per_iteration_all_active=round(us_it, 2),
               batched_kernel_bytes_per_iteration=kbytes,
               batched_kernel_gbs=round(kbytes / (us_it * 1e-6) / 1e9, 1),
               batched_kernel_frac_of_hbm_peak=round(kbytes / (us_it * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
               online_pod=dict(window=args.batch_window,
                               instance_steps_per_s=round(len(meshes) * args.batch_steps / el_on, 3),
                               ms_per_batch_step=round(1e3 * el_on / args.batch_steps, 2),
                               poisson_iters_min_max=[min(iters_on), max(iters_on)], phase_ms_mean=ph_on),
               mixed_online_pod=dict(instance_steps_per_s=round(len(meshes) * args.batch_steps / el_mx, 3),
                                     ms_per_batch_step=round(1e3 * el_mx / args.batch_steps, 2),
                                     inner_iters_min_max=[min(iters_mx), max(iters_mx)], phase_ms_mean=ph_mx))
    log(f"batch: {out['instance_steps_per_s']} instance-steps/s ({out['ms_per_batch_step']} ms per batch step) vs "
        f"{out['sequential_instance_steps_per_s']} sequential; Poisson iterations {min(iters)}..{max(iters)}; "
        f"batched PCG kernel {us_it:.1f} us/iteration for {kbytes / 1e6:.0f} MB -> {out['batched_kernel_gbs']} GB/s; "
        f"rel err vs single-instance {err:.1e}; phases (ms) {ph_plain}")
    log(f"batch with per-instance online POD guesses (window {args.batch_window}): "
        f"{out['online_pod']['instance_steps_per_s']} instance-steps/s ({out['online_pod']['ms_per_batch_step']} ms "
        f"per batch step); Poisson iterations {min(iters_on)}..{max(iters_on)}; phases (ms) {ph_on}")
    log(f"batch with online POD guesses and batched FP32 refinement: {out['mixed_online_pod']['instance_steps_per_s']} "
        f"instance-steps/s ({out['mixed_online_pod']['ms_per_batch_step']} ms per batch step); inner iterations "
        f"{min(iters_mx)}..{max(iters_mx)}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=64,
                    help="untimed steps of each path before its timed steps (an online window of 64 then holds "
                         "only the path's own solves)")
    ap.add_argument("--target-tris", type=int, default=250_000, help="coarse triangles (fine = 4x)")
    ap.add_argument("--snapshots", type=int, default=64, help="plain-FP64 steps recorded as training data")
    ap.add_argument("--modes", type=int, default=32, help="POD modes of the learned guess")
    ap.add_argument("--hidden", type=int, default=128, help="hidden width of the guess networks")
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--window", type=int, default=64, help="solutions kept for the online POD basis (at most 64)")
    ap.add_argument("--refresh", type=int, default=1, help="Poisson solves between online basis rebuilds")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps timed for the CPU baseline (0: skip)")
    ap.add_argument("--no-instrumented", action="store_true", help="skip the event-timed kernel pass")
    ap.add_argument("--only-batch-long", action="store_true",
                    help="run only the long batched run (64 instances, --batch-long steps each) with the oracle check")
    ap.add_argument("--batch-long", type=int, default=500, help="steps of the long batched run")
    ap.add_argument("--only-gmres", action="store_true",
                    help="run only the ILU(0)-GMRES against Jacobi-PCG comparison on the Poisson systems")
    ap.add_argument("--gmres-max-iter", type=int, default=300,
                    help="iteration cap of ILU(0)-GMRES at the full size (each iteration is two level-scheduled "
                         "triangular solves)")
    ap.add_argument("--mass-x0", default="lumped", choices=["lumped", "extrap"],
                    help="mass solve start: the lumped correction, or that plus the last step's consistent-minus-"
                         "lumped difference")
    ap.add_argument("--pcg-graph", type=int, default=0,
                    help="1: fused Poisson PCG iterations launched as captured graphs of 8 (0, one launch each, is "
                         "the library default)")
    ap.add_argument("--launch", choices=["loop", "persistent", "fused"], default="fused",
                    help="Poisson Krylov launch strategy")
    ap.add_argument("--mom-x0", choices=["prev", "extrap", "project"], default="project",
                    help="momentum initial guess: U^n, the quadratic extrapolation of the three previous solves, or "
                         "the residual-minimising combination of the last eight")
    # the Poisson right-hand side is the divergence of U~, small beside U~ itself: a momentum error of
    # relative size t reaches it amplified ~100-300x, so the momentum solve runs 2.5 decades below the
    # Poisson's (sweep on the online-POD path: 1e-9 -> 90, 3e-10 -> 105, 1e-10 -> 114, 3e-11 -> 118 steps/s)
    ap.add_argument("--mom-tol", type=float, default=3e-11, help="momentum solve tolerance (relative residual)")
    ap.add_argument("--mass-tol", type=float, default=1e-10, help="mass solve tolerance of the correction")
    ap.add_argument("--inner-tol", type=float, default=1e-4, help="FP32 inner solve tolerance of the refinement")
    ap.add_argument("--mass-method", default="pcg", choices=["pcg", "cheb"],
                    help="mass solve of the correction: Jacobi-PCG or the Chebyshev iteration on [1/2, 2]")
    ap.add_argument("--paths", default="all", help="comma-separated subset of the timed paths")
    ap.add_argument("--batch", type=int, default=64, help="instances of the batched sweep (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=5)
    ap.add_argument("--batch-window", type=int, default=64, help="online POD window per batched instance (at most 64)")
    ap.add_argument("--only-batch", action="store_true", help="run only the batched sweep")
    ap.add_argument("--only-batch-kernel", action="store_true",
                    help="run only the batched PCG iteration with every instance active (for HBM counters)")
    ap.add_argument("--levels-sweep", type=int, default=1, help="run the l = 0..3 comparison on one fine mesh (0: skip)")
    ap.add_argument("--bfs", type=int, default=1, help="run the backward-facing step at l = 1 and l = 0 (0: skip)")
    ap.add_argument("--only-levels", action="store_true", help="run only the l = 0..3 comparison")
    ap.add_argument("--only-learned", action="store_true",
                    help="run only the learned-guess study (Re sweep, 64 modes, 64-256-256-64, held-out Re)")
    ap.add_argument("--learn-re", type=int, default=20, help="Re values of the learned-guess study")
    ap.add_argument("--learn-test-re", type=int, default=4, help="of them held out for evaluation")
    ap.add_argument("--learn-settle", type=int, default=1000, help="unrecorded steps per Re")
    ap.add_argument("--learn-record", type=int, default=100, help="recorded steps per Re")
    ap.add_argument("--learn-stride", type=int, default=10, help="steps per recorded step after the settling steps")
    ap.add_argument("--learn-restrict", type=int, default=1, help="restriction of the study's runs (0 injection, 1 Galerkin)")
    ap.add_argument("--learn-online-window", type=int, default=64,
                    help="online POD window of the recording runs' Poisson starts (0: previous pressure)")
    ap.add_argument("--learn-epochs", type=int, default=200, help="training epochs")
    ap.add_argument("--learn-eval-every", type=int, default=5, help="held-out recorded steps between evaluations")
    ap.add_argument("--only-functionals", action="store_true",
                    help="run only the long flow-functional runs (cylinder drag, lift, Strouhal; backward-step reattachment)")
    ap.add_argument("--func-steps", type=int, default=8000, help="cylinder steps of the functional run")
    ap.add_argument("--func-every", type=int, default=10, help="steps between force evaluations")
    ap.add_argument("--func-restrict", type=int, default=1,
                    help="restriction of the functional runs: 0 inject, 1 Galerkin (energy-stable; the default)")
    ap.add_argument("--bfs-steps", type=int, default=10000, help="backward-step steps of the functional run")
    ap.add_argument("--level-warmup", type=int, default=10, help="untimed steps per level / backward-step run")
    ap.add_argument("--level-steps", type=int, default=10, help="timed steps per level / backward-step run")
    ap.add_argument("--only-bfs", action="store_true", help="run only the backward-facing step")
    ap.add_argument("--bfs-nx", type=int, default=612, help="cells along the backward-step channel (42 across at 612)")
    ap.add_argument("--spmv-sweep", type=int, default=1, help="run the SpMV size sweep (0: skip)")
    ap.add_argument("--spmv-large", action="store_true", help="add a 16.8M-row point to the SpMV sweep")
    ap.add_argument("--only-spmv", action="store_true", help="run only the SpMV size sweep")
    ap.add_argument("--cg-sweep", type=int, default=1, help="run the PCG iteration size sweep (0: skip)")
    ap.add_argument("--only-cg", action="store_true", help="run only the PCG iteration size sweep")
    ap.add_argument("--only-steady", type=int, default=0, metavar="STEPS",
                    help="run only a continuous online-POD run of STEPS steps per precision (20-step means)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)  # one elementwise kernel: n * 8 bytes read, n * 8 bytes written
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration} MiB three times ({n * 8} bytes read and written per copy)")
        return

    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts, StepOpts
    X0 = cgp._native
    if args.only_batch:
        print(json.dumps({"batch": run_batch(args, log)}), flush=True)
        return
    if args.only_batch_kernel:
        print(json.dumps({"batch_kernel": run_batch_kernel(args, log)}), flush=True)
        return
    if args.only_spmv:
        print(json.dumps({"spmv_sweep": run_spmv_sweep(args, log)}), flush=True)
        return
    if args.only_levels:
        print(json.dumps({"levels": run_levels(args, log)}), flush=True)
        return
    if args.only_learned:
        print(json.dumps({"learned": run_learned(args, log)}), flush=True)
        return
    if args.only_batch_long:
        print(json.dumps({"batch_long": run_batch_long(args, log)}), flush=True)
        return
    if args.only_gmres:
        print(json.dumps({"poisson_solvers": run_gmres(args, log)}), flush=True)
        return
    if args.only_functionals:
        print(json.dumps({"functionals": run_functionals(args, log)}), flush=True)
        return
    if args.only_bfs:
        print(json.dumps({"backward_step": run_bfs(args, log)}), flush=True)
        return
    if args.only_cg:
        print(json.dumps({"cg_sweep": run_cg_sweep(args, log)}), flush=True)
        return
    if args.only_steady:
        print(json.dumps({"steady": run_steady(args, log)}), flush=True)
        return

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    t0 = time.perf_counter()
    case = W.case_cylinder(args.target_tris)
    mesh = cgp.Mesh(case.mesh, 1)
    mesh.assemble(case.rho, case.mu, case.dt)
    mesh.set_tuning(pcg_graph=args.pcg_graph)
    info = mesh.info
    nnz_c, n_c = info["nnz_c"], info["n_c"]
    log(f"mesh: coarse {info['t_c']} tris / {n_c} nodes, fine {info['t_f']} tris / {info['n_f']} nodes, "
        f"nnz_f {info['nnz_f']}, nnz_c {nnz_c}, colours {info['ncol_f']}; setup {time.perf_counter() - t0:.1f}s")

    xy = mesh.export("xy")
    vdir = mesh.export("vdir")
    g = torch.from_numpy(case.dirichlet(xy, 0.0)).to(dev)  # steady inflow data
    u = torch.from_numpy(case.initial(xy, vdir)).to(dev)
    pf = torch.zeros(info["n_f"], dtype=torch.float64, device=dev)
    pc = torch.zeros(n_c, dtype=torch.float64, device=dev)

    tol = 1e-8
    launch = {"loop": 1, "persistent": 2, "fused": 3}[args.launch]

    mom_x0 = {"prev": X0.X0_PREV, "extrap": X0.X0_EXTRAP, "project": X0.X0_PROJECT}[args.mom_x0]
    mass_x0 = {"lumped": X0.X0_PREV, "extrap": X0.X0_EXTRAP}[args.mass_x0]
    mass_method = {"pcg": X0.METHOD_DEFAULT, "cheb": X0.METHOD_CHEBYSHEV}[args.mass_method]

    F64, F32 = cgp._native.PREC_FP64, cgp._native.PREC_FP32_IR
    MIXED_ALL = 100  # the bench's own code: FP32 inner solves in the momentum and the Poisson solve

    def opts(precision=0, x0=X0.X0_PREV, timing=0):
        pp = F32 if precision in (F32, MIXED_ALL) else F64
        mp = F32 if precision == MIXED_ALL else F64
        return StepOpts(momentum=SolverOpts(tol=args.mom_tol, max_iter=5000, x0_mode=mom_x0, precision=mp),
                        poisson=SolverOpts(tol=tol, max_iter=100000, precision=pp, inner_tol=args.inner_tol,
                                           x0_mode=x0, launch=launch),
                        mass=SolverOpts(tol=args.mass_tol, max_iter=2000, x0_mode=mass_x0, method=mass_method),
                        timing=timing)

    SETTLE = 10  # plain steps from the impulsive start before the training data is recorded
    for k in range(SETTLE):
        st = mesh.step(g, u, pf, pc, opts=opts())
    torch.cuda.synchronize()
    log(f"{SETTLE} plain steps done; last Poisson iterations {st['p_iters']}")

    # training data from the plain path, then the POD bases and networks, all on the GPU
    S = args.snapshots
    rhs = torch.zeros((S, n_c), dtype=torch.float64, device=dev)
    ps = torch.zeros_like(rhs)
    pprev = torch.zeros_like(rhs)
    # each path restarts REPLAY recorded steps before the end and steps them again, so that the
    # momentum guess's history (the last 8 solves) is this trajectory's own when the path starts
    REPLAY = 9
    assert S >= REPLAY, "--snapshots must be at least 9"
    for k in range(S):
        if k == S - REPLAY:
            replay_u, replay_pc = u.clone(), pc.clone()
        pprev[k].copy_(pc)
        mesh.step(g, u, pf, pc, opts=opts())
        mesh.last_poisson_rhs(rhs[k])
        ps[k].copy_(pc)
    torch.cuda.synchronize()
    train = {}
    models = {}
    for name, prev in (("abs", None), ("incr", pprev)):
        net = cgp.Guess(mesh, n_modes=args.modes, hidden=args.hidden, seed=11)
        t1 = time.perf_counter()
        # the incremental model's basis spans the recorded pressure increments, the quantity it predicts
        net.build_pod(ps if prev is None else (ps - prev).contiguous())
        tr = net.train(rhs, ps, epochs=args.epochs, batch=64, lr=2e-3, p_prev=prev)
        torch.cuda.synchronize()
        train[name] = dict(loss_first=tr["loss_first"], loss_last=tr["loss_last"], adam_steps=tr["steps"],
                           train_ms=round(tr["ms"], 1), pod_and_train_s=round(time.perf_counter() - t1, 3))
        models[name] = net
        log(f"{name} model: POD {args.modes} modes of {S} snapshots, training loss {tr['loss_first']:.3e} -> "
            f"{tr['loss_last']:.3e} in {tr['steps']} Adam steps ({tr['ms']:.0f} ms on the GPU)")
    # online basis: rebuilt after every solve from the last `window` solutions (a recycled subspace);
    # restarting a path refills its window from the recorded pressures
    online = cgp.Guess(mesh, n_modes=args.window, hidden=16, seed=5)
    models["online"] = online

    def restore(model=None):
        """Back to the recorded state with `model` attached (None: no guess model): the last REPLAY
        recorded steps are stepped again with plain FP64 Poisson solves and no model, the first with
        the momentum solve started from U^n (which empties the momentum guess's history)."""
        online.detach()
        u.copy_(replay_u)
        pc.copy_(replay_pc)
        pf.zero_()
        for k in range(REPLAY):
            o = opts()
            if k == 0:
                o.momentum.x0_mode = X0.X0_PREV
            mesh.step(g, u, pf, pc, opts=o)
        if model == "online":
            online.set_online(args.window, args.refresh)
            online.attach()
            for k in range(max(0, S - args.window), S):  # the newest recorded solves fill the window
                mesh.poisson_solve(rhs[k], ps[k].clone(), SolverOpts(tol=tol, x0_mode=X0.X0_PREV))
        elif model:
            models[model].attach()
        else:
            online.detach()
        torch.cuda.synchronize()

    paths = {
        "fp64": (F64, X0.X0_PREV, None),
        "fp64+pod_galerkin": (F64, X0.X0_POD_GALERKIN, "abs"),
        "fp64+learned": (F64, X0.X0_LEARNED, "abs"),
        "fp64+learned_corr": (F64, X0.X0_LEARNED_CORR, "incr"),
        "fp64+online_pod": (F64, X0.X0_POD_GALERKIN, "online"),
        "mixed": (F32, X0.X0_PREV, None),
        "mixed+learned_corr": (F32, X0.X0_LEARNED_CORR, "incr"),
        "mixed+online_pod": (F32, X0.X0_POD_GALERKIN, "online"),
        "mixed_all+online_pod": (MIXED_ALL, X0.X0_POD_GALERKIN, "online"),
    }
    if args.paths != "all":
        keep = set(args.paths.split(",")) | {"fp64"}
        paths = {k: v for k, v in paths.items() if k in keep}

    ml = torch.from_numpy(mesh.export("ml_f")).to(dev)

    def flow_stats():
        """max |u| and the kinetic energy (1/2) u^T M_L u of the current velocity"""
        sp = u[:, 0] * u[:, 0] + u[:, 1] * u[:, 1]
        return float(torch.sqrt(sp.max())), float(0.5 * (ml * sp).sum())

    def one_step_error(prec, x0, model):
        """From the current state: one step of the path against one plain FP64 step (state restored
        between them); the path's step is the one kept."""
        su, spc, spf = u.clone(), pc.clone(), pf.clone()
        if model:
            (online if model == "online" else models[model]).detach()
        mesh.step(g, u, pf, pc, opts=opts())
        ref_u, ref_pf = u.clone(), pf.clone()
        u.copy_(su)
        pc.copy_(spc)
        pf.copy_(spf)
        if model:
            (online if model == "online" else models[model]).attach()
        mesh.step(g, u, pf, pc, opts=opts(prec, x0))
        return max(rel(u.cpu().numpy(), ref_u.cpu().numpy()), rel(pf.cpu().numpy(), ref_pf.cpu().numpy()))

    # the plain FP64 trajectory of the timed window, for each path's trajectory difference (reported)
    restore()
    for k in range(args.warmup + args.steps):
        mesh.step(g, u, pf, pc, opts=opts())
    traj_u, traj_pf = u.cpu().numpy(), pf.cpu().numpy()
    results = {}
    phase_keys = ("ms_momentum", "ms_restrict", "ms_poisson", "ms_prolong", "ms_correct")
    for name, (prec, x0, model) in paths.items():
        restore(model)
        err_start = one_step_error(prec, x0, model)
        restore(model)
        for k in range(args.warmup):  # untimed: solver chunk sizes adapt, guess windows turn over
            mesh.step(g, u, pf, pc, opts=opts(prec, x0))
        torch.cuda.synchronize()
        iters, miters, mass_its, phases, flow = [], [], [], {k: 0.0 for k in phase_keys}, []
        t1 = time.perf_counter()
        for k in range(args.steps):
            st = mesh.step(g, u, pf, pc, opts=opts(prec, x0, timing=1))
            iters.append(st["p_iters"])
            miters.append(st["mom_iters"])
            mass_its.append(st["mass_iters"])
            for key in phase_keys:
                phases[key] += st[key]
            if k == 0:
                flow.append(flow_stats())
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        flow.append(flow_stats())
        err_traj = max(rel(u.cpu().numpy(), traj_u), rel(pf.cpu().numpy(), traj_pf))
        err_end = one_step_error(prec, x0, model)
        results[name] = dict(steps_per_s=round(args.steps / el, 3), ms_per_step=round(1e3 * el / args.steps, 3),
                             poisson_iters_mean=float(np.mean(iters)), momentum_iters_mean=float(np.mean(miters)),
                             mass_iters_mean=float(np.mean(mass_its)),
                             rel_err_vs_fp64=max(err_start, err_end), rel_err_vs_fp64_at_restart=err_start,
                             rel_err_vs_fp64_after_timed_steps=err_end,
                             trajectory_diff_vs_fp64=err_traj,
                             max_abs_u_first_last=[round(flow[0][0], 6), round(flow[-1][0], 6)],
                             kinetic_energy_first_last=[round(flow[0][1], 8), round(flow[-1][1], 8)],
                             phase_ms_mean={k: round(v / args.steps, 4) for k, v in phases.items()})
        log(f"{name}: {args.steps / el:.2f} steps/s ({1e3 * el / args.steps:.2f} ms/step), Poisson iterations "
            f"{np.mean(iters):.0f}, momentum iterations {np.mean(miters):.1f}; one-step rel err vs fp64 "
            f"{err_start:.1e} at restart, {err_end:.1e} after the timed steps; trajectory diff {err_traj:.1e}; "
            f"max|u| {flow[0][0]:.3f} -> {flow[-1][0]:.3f}; phases (ms) mom {phases['ms_momentum'] / args.steps:.2f} "
            f"poisson {phases['ms_poisson'] / args.steps:.2f} correct {phases['ms_correct'] / args.steps:.2f}")
    restore()

    eligible = {k: v for k, v in results.items() if v["rel_err_vs_fp64"] <= ERR_BAR}
    best = max(eligible, key=lambda k: eligible[k]["steps_per_s"])
    bprec, bx0, bmodel = paths[best]
    res = results[best]

    # dominant kernel of the best path: every launch bracketed by events that its own dispatch records
    dom = None
    if not args.no_instrumented:
        restore(bmodel)
        tot_ms, cnt, its = 0.0, 0, 0
        for k in range(args.steps):
            s = mesh.step(g, u, pf, pc, opts=opts(bprec, bx0, timing=2))
            tot_ms += s["ms_dominant"]
            cnt += s["n_dominant"]
            its += s["dominant_iters"]
        restore()
        kname, bytes_per_iter = dominant_kernel("f32" if bprec in (F32, MIXED_ALL) else "f64", args.launch, nnz_c,
                                                n_c)
        achieved = bytes_per_iter * its / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
        traffic = None
        tf = ROOT / "profiles" / "traffic_dominant.json"
        if tf.exists():
            tj = json.loads(tf.read_text()).get(kname, {})
            if tj.get("source_hash") == kernel_source_hash() and tj.get("n_c") == n_c:
                traffic = tj.get("bytes_per_launch")
        dom = dict(kernel=kname, launches=cnt, iterations=its, avg_us=1e3 * tot_ms / max(cnt, 1),
                   bytes_per_launch=bytes_per_iter, achieved=achieved, traffic=traffic)
        log(f"dominant kernel {kname}: {cnt} launches, avg {dom['avg_us']:.2f} us, {bytes_per_iter} algorithmic "
            f"bytes per launch, {achieved:.0f} GB/s")

    # CPU baseline: the FP64 oracle from the same state (one thread, and the OpenMP build on every host
    # core, in child processes), and the best path's one-step accuracy against it
    cpu = None
    err_vs_oracle = None
    if args.cpu_steps > 0:
        import os
        import subprocess
        import tempfile

        import oracle
        ref = oracle.Problem(case.mesh, 1)
        ref.assemble(case.rho, case.mu, case.dt)
        gh = g.cpu().numpy()
        restore(bmodel)
        ur, pcr = u.cpu().numpy(), pc.cpu().numpy()
        mesh.step(g, u, pf, pc, opts=opts(bprec, bx0))
        ub, pfb = u.cpu().numpy(), pf.cpu().numpy()
        restore()
        t2 = time.perf_counter()
        ur1, pfr1, _, code, _ = ref.step(gh, ur, pcr, tol_mom=args.mom_tol, tol_p=tol, tol_mass=args.mass_tol)
        el1 = time.perf_counter() - t2
        err_vs_oracle = max(rel(ub, ur1), rel(pfb, pfr1))
        nproc = os.cpu_count() or 1
        try:
            nproc = len(os.sched_getaffinity(0))
        except AttributeError:
            pass
        model_name = "unknown"
        try:
            for ln in open("/proc/cpuinfo"):
                if ln.startswith("model name"):
                    model_name = ln.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
        timed = {}
        with tempfile.TemporaryDirectory() as td:
            state = os.path.join(td, "state.npz")
            np.savez(state, u=ur, pc=pcr, g=gh)
            for label, env_extra in (("single", {"CGP_ORACLE_OPENMP": "0", "OMP_NUM_THREADS": "1"}),
                                     ("openmp", {"CGP_ORACLE_OPENMP": "1", "OMP_NUM_THREADS": str(nproc)})):
                env = dict(os.environ, **env_extra)
                cmd = [sys.executable, "-m", "oracle.timing", state, str(args.target_tris), str(args.cpu_steps),
                       repr(args.mom_tol), repr(tol), repr(args.mass_tol)]
                r = subprocess.run(cmd, cwd=str(ROOT), env=env, capture_output=True, text=True, timeout=900)
                if r.returncode == 0:
                    timed[label] = json.loads(r.stdout.strip().splitlines()[-1])
                else:
                    log(f"oracle timing ({label}) failed: {r.stderr[-400:]}")
        single = timed.get("single", dict(s_per_step=el1, steps=1, threads=1))
        cpu = dict(value=round(1.0 / single["s_per_step"], 5), unit="CGP steps/s", cores=1, kind="oracle",
                   sample=f"{single['steps']} FP64 oracle steps (single thread) of the same cylinder workload "
                          f"from the post-training state; {single['s_per_step']:.2f} s per step",
                   nproc=nproc, cpu_model=model_name)
        if "openmp" in timed:
            om = timed["openmp"]
            cpu["openmp"] = dict(value=round(1.0 / om["s_per_step"], 5), unit="CGP steps/s", cores=om["threads"],
                                 s_per_step=round(om["s_per_step"], 3))
        log(f"oracle: {single['s_per_step']:.2f} s/step on one thread"
            + (f", {timed['openmp']['s_per_step']:.2f} s/step on {timed['openmp']['threads']} threads" if "openmp" in
               timed else "") + f" ({model_name}, {nproc} cores); {best} step vs oracle rel err {err_vs_oracle:.2e}")

    line = {
        "metric": "CGP steps/s (1M-tri fine mesh) vs plain FP64 at <=1e-6 rel err; SpMV HBM GB/s",
        "value": res["steps_per_s"],
        "unit": "CGP steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32-ir" if bprec in (F32, MIXED_ALL) else "f64", "data": "synthetic",
        "config": {"workload": f"cylinder channel Re=100, coarse {info['t_c']} / fine {info['t_f']} P1 triangles, "
                               f"l=1, injection restriction, consistent-mass correction, dt=1e-3, Poisson PCG tol 1e-8 "
                               f"(momentum {args.mom_tol:g}, mass {args.mass_tol:g}), momentum x0 {args.mom_x0}, "
                               f"path {best}",
                   "path": best, "fine_nodes": info["n_f"], "coarse_nodes": n_c, "nnz_f": info["nnz_f"],
                   "nnz_c": nnz_c, "pod_modes": args.modes, "snapshots": S, "parallelism": "single GPU"},
        "fp64_steps_per_s": results["fp64"]["steps_per_s"],
        "speedup_vs_fp64": round(res["steps_per_s"] / results["fp64"]["steps_per_s"], 3),
        "rel_err_vs_fp64_gpu": res["rel_err_vs_fp64"],
        "max_abs_u_first_last": res["max_abs_u_first_last"],
        "kinetic_energy_first_last": res["kinetic_energy_first_last"],
        "rel_err_vs_fp64_oracle": err_vs_oracle,
        "paths": results,
        "training": train,
    }
    if dom:
        line["roofline"] = {"bound": "hbm", "achieved": round(dom["achieved"], 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(dom["achieved"] / HBM_PEAK_GBS, 4),
                            "traffic": dom["traffic"], "kernel": dom["kernel"], "avg_us": round(dom["avg_us"], 3),
                            "launches": dom["launches"], "bytes_per_launch": dom["bytes_per_launch"]}
    if cpu:
        line["cpu_baseline"] = cpu
    for net in models.values():
        net.close()
    if args.levels_sweep:
        try:
            line["levels"] = run_levels(args, log)
        except Exception as e:
            line["levels"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"levels sweep failed: {e}")
    if args.bfs:
        try:
            line["backward_step"] = run_bfs(args, log)
        except Exception as e:
            line["backward_step"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"backward-facing step failed: {e}")
    if args.spmv_sweep:
        try:
            line["spmv_sweep"] = run_spmv_sweep(args, log)
        except Exception as e:
            line["spmv_sweep"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"SpMV sweep failed: {e}")
    if args.cg_sweep:
        try:
            line["cg_sweep"] = run_cg_sweep(args, log)
        except Exception as e:
            line["cg_sweep"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"PCG sweep failed: {e}")
    if args.batch > 0:
        try:
            line["batch"] = run_batch(args, log)
        except Exception as e:  # the sweep is reported beside the headline metric, never instead of it
            line["batch"] = {"error": f"{type(e).__name__}: {e}"}
            log(f"batch sweep failed: {e}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
