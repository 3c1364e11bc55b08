#!/usr/bin/env python3
"""IFE-CGP benchmark on one MI355X.

Workload: flow past a cylinder (radius 0.05 at (0.2, 0.2)) in a 2.2 x 0.41
channel, Re = 100, dt = 1e-3; seeded coarse mesh of ~250k P1 triangles, fine
mesh of ~1M triangles after one 1:4 subdivision (l = 1).  A step is one pass
of the whole CGP path: convective assembly and momentum solve on the fine
mesh, restriction and coarse divergence, coarse pressure Poisson solve,
prolongation, velocity correction.

Warm-up steps develop the flow from an impulsive start with the plain FP64
path; the two paths are then timed from the same state:
  * plain FP64 CGP (Jacobi-PCG to 1e-8, x0 = previous pressure);
  * mixed precision: FP32 Jacobi-PCG inside FP64 iterative refinement to
    the same 1e-8; its per-step output is compared with the FP64 GPU path
    and with the FP64 CPU oracle from the same state.
``value`` is the mixed-precision path's steps/s.  One JSON line goes to stdout.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def rel(a, b):
    import numpy as np
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in sorted((ROOT / "paper_1610_06993_amd" / "csrc").glob("*")):
        h.update(p.read_bytes())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--target-tris", type=int, default=250_000, help="coarse triangles (fine = 4x)")
    ap.add_argument("--cpu-steps", type=int, default=2, help="oracle steps timed for the CPU baseline (0: skip)")
    ap.add_argument("--no-instrumented", action="store_true", help="skip the event-bracketed kernel pass")
    ap.add_argument("--launch", choices=["loop", "persistent", "fused"], default="fused",
                    help="Poisson Krylov launch strategy")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (HBM counter calibration)")
    args = ap.parse_args()
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
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1610_06993_amd as cgp
    import workloads as W
    from paper_1610_06993_amd import SolverOpts, StepOpts

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)

    t0 = time.perf_counter()
    case = W.case_cylinder(args.target_tris)
    mesh = cgp.Mesh(case.mesh, 1)
    mesh.assemble(case.rho, case.mu, case.dt)
    info = mesh.info
    log(f"mesh: coarse {info['t_c']} tris / {info['n_c']} nodes, fine {info['t_f']} tris / {info['n_f']} nodes, "
        f"nnz_f {info['nnz_f']}, nnz_c {info['nnz_c']}, colours {info['ncol_f']}; setup {time.perf_counter() - t0:.1f}s")

    xy = mesh.export("xy")
    vdir = mesh.export("vdir")
    g = torch.from_numpy(case.dirichlet(xy, 0.0)).to(dev)  # steady inflow data
    u = torch.from_numpy(case.initial(xy, vdir)).to(dev)
    pf = torch.zeros(info["n_f"], dtype=torch.float64, device=dev)
    pc = torch.zeros(info["n_c"], dtype=torch.float64, device=dev)

    tol = 1e-8
    launch = {"loop": 1, "persistent": 2, "fused": 3}[args.launch]
    fp64 = StepOpts(momentum=SolverOpts(tol=tol, max_iter=5000),
                    poisson=SolverOpts(tol=tol, max_iter=100000, launch=launch),
                    mass=SolverOpts(tol=1e-10, max_iter=2000))
    mixed = StepOpts(momentum=SolverOpts(tol=tol, max_iter=5000),
                     poisson=SolverOpts(tol=tol, max_iter=100000, precision=cgp._native.PREC_FP32_IR,
                                        inner_tol=1e-4, launch=launch),
                     mass=SolverOpts(tol=1e-10, max_iter=2000))

    for k in range(args.warmup):
        st = mesh.step(g, u, pf, pc, opts=fp64)
    torch.cuda.synchronize()
    log(f"warm-up {args.warmup} steps done; last: {st}")
    snap_u, snap_pc = u.clone(), pc.clone()

    def restore():
        u.copy_(snap_u)
        pc.copy_(snap_pc)
        pf.zero_()
        torch.cuda.synchronize()

    results = {}
    for name, opts in (("fp64", fp64), ("mixed", mixed)):
        restore()
        mesh.step(g, u, pf, pc, opts=opts)  # one untimed step per path (solver chunk sizes adapt)
        restore()
        iters = []
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(args.steps):
            st = mesh.step(g, u, pf, pc, opts=opts)
            iters.append(st["p_iters"])
        torch.cuda.synchronize()
        el = time.perf_counter() - t1
        results[name] = dict(steps_per_s=args.steps / el, ms_per_step=1e3 * el / args.steps,
                             p_iters_mean=float(np.mean(iters)), last=st)
        log(f"{name}: {args.steps / el:.2f} steps/s ({1e3 * el / args.steps:.2f} ms/step), mean Poisson iters "
            f"{np.mean(iters):.0f}")

    # per-phase breakdown and accuracy from the same state
    restore()
    st64 = mesh.step(g, u, pf, pc, opts=StepOpts(fp64.momentum, fp64.poisson, fp64.mass, timing=1))
    u64, pf64 = u.cpu().numpy(), pf.cpu().numpy()
    restore()
    stmx = mesh.step(g, u, pf, pc, opts=StepOpts(mixed.momentum, mixed.poisson, mixed.mass, timing=1))
    umx, pfmx = u.cpu().numpy(), pf.cpu().numpy()
    err_vs_fp64 = max(rel(umx, u64), rel(pfmx, pf64))
    log(f"phases fp64 (ms): mom {st64['ms_momentum']:.2f} restr {st64['ms_restrict']:.3f} poisson "
        f"{st64['ms_poisson']:.2f} prolong {st64['ms_prolong']:.3f} correct {st64['ms_correct']:.2f}")
    log(f"phases mixed (ms): mom {stmx['ms_momentum']:.2f} poisson {stmx['ms_poisson']:.2f} "
        f"(outer {stmx['p_outer']}, inner iters {stmx['p_iters']}); rel err vs fp64 {err_vs_fp64:.2e}")

    # dominant kernel of the timed (mixed) path, every launch bracketed by HIP events on the mesh stream:
    # the persistent FP32 PCG kernel (one launch per inner solve) or, in the launch-per-phase loop, the
    # fused FP32 p-update + SpMV kernel (one launch per iteration)
    dom = None
    if not args.no_instrumented:
        restore()
        tot_ms, cnt, its = 0.0, 0, 0
        for k in range(args.steps):
            s = mesh.step(g, u, pf, pc, opts=StepOpts(mixed.momentum, mixed.poisson, mixed.mass, timing=2))
            tot_ms += s["ms_dominant"]
            cnt += s["n_dominant"]
            its += s["dominant_iters"]
        nnz_c, n_c = info["nnz_c"], info["n_c"]
        if args.launch == "loop":
            kname = "k_cg_spmv<float>"
            # values 4 B + column 4 B per nonzero; row pointer 4 B, z and p_old 4+4 B read, p_new and q
            # 4+4 B written per row (each vector touched once)
            bytes_per_iter = 8 * nnz_c + 20 * n_c
        elif args.launch == "fused":
            kname = "k_cg1_iter<float>"
            # one whole FP32 iteration: values + columns 8 B per nonzero; row pointer 4 B, D^-1, r, w, s, p, x
            # read (24 B) and x, p, s, r, w written (20 B) per row, each vector touched once
            bytes_per_iter = 8 * nnz_c + 48 * n_c
        else:
            kname = "k_pcg_persistent<float>"
            # one FP32 PCG iteration: the SpMV phase above (8 nnz + 20 n) plus the update phase reading
            # x, p, r, q, D^-1 and writing x, r, z (32 n)
            bytes_per_iter = 8 * nnz_c + 52 * n_c
        total_bytes = bytes_per_iter * its
        achieved = total_bytes / (tot_ms * 1e-3) / 1e9 if tot_ms > 0 else 0.0
        traffic = None
        tf = ROOT / "profiles" / "traffic_dominant.json"
        if tf.exists():
            tj = json.loads(tf.read_text())
            if tj.get("source_hash") == kernel_source_hash() and tj.get("kernel") == kname:
                traffic = tj.get("bytes_per_iteration")
        dom = dict(kernel=kname, launches=cnt, iterations=its, avg_us=1e3 * tot_ms / max(cnt, 1),
                   bytes_per_launch=total_bytes / max(cnt, 1), bytes_per_iteration=bytes_per_iter,
                   achieved=achieved, traffic=traffic, us_per_iteration=1e3 * tot_ms / max(its, 1))
        log(f"dominant kernel {kname}: {cnt} launches, {its} iterations, avg {dom['avg_us']:.1f} us/launch, "
            f"{dom['us_per_iteration']:.2f} us/iteration, {achieved:.0f} GB/s algorithmic")

    # CPU baseline: the FP64 oracle from the same state, and the accuracy of the timed path against it
    cpu = None
    err_vs_oracle = None
    if args.cpu_steps > 0:
        import oracle
        ref = oracle.Problem(case.mesh, 1)
        ref.assemble(case.rho, case.mu, case.dt)
        ur, pcr = snap_u.cpu().numpy(), snap_pc.cpu().numpy()
        gh = g.cpu().numpy()
        t2 = time.perf_counter()
        outs = []
        for k in range(args.cpu_steps):
            ur, pfr, pcr, code, ost = ref.step(gh, ur, pcr, tol_mom=tol, tol_p=tol, tol_mass=1e-10)
            outs.append((ur.copy(), pfr.copy()))
        el = time.perf_counter() - t2
        err_vs_oracle = max(rel(umx, outs[0][0]), rel(pfmx, outs[0][1]))
        cpu = dict(value=args.cpu_steps / el, unit="CGP steps/s", cores=1, kind="oracle",
                   sample=f"{args.cpu_steps} FP64 oracle steps (single thread) of the same cylinder workload "
                          f"from the post-warm-up state; {el:.1f} s")
        log(f"oracle: {el / args.cpu_steps:.2f} s/step; mixed GPU step vs oracle rel err {err_vs_oracle:.2e}")

    res = results["mixed"]
    line = {
        "metric": "CGP steps/s (1M-tri fine mesh) vs plain FP64 at <=1e-6 rel err; SpMV HBM GB/s",
        "value": round(res["steps_per_s"], 3),
        "unit": "CGP steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64+f32-ir", "data": "synthetic",
        "config": {"workload": f"cylinder channel Re=100, coarse {info['t_c']} / fine {info['t_f']} P1 triangles, "
                               f"l=1, dt=1e-3, PCG tol 1e-8 (FP32 inner in FP64 refinement)",
                   "fine_nodes": info["n_f"], "coarse_nodes": info["n_c"], "nnz_f": info["nnz_f"],
                   "nnz_c": info["nnz_c"], "parallelism": "single GPU"},
        "fp64_steps_per_s": round(results["fp64"]["steps_per_s"], 3),
        "speedup_vs_fp64": round(res["steps_per_s"] / results["fp64"]["steps_per_s"], 3),
        "rel_err_vs_fp64_gpu": err_vs_fp64,
        "rel_err_vs_fp64_oracle": err_vs_oracle,
        "poisson_iters_mean": {"fp64": results["fp64"]["p_iters_mean"], "mixed_inner": res["p_iters_mean"]},
        "phase_ms_fp64": {k: round(st64[k], 4) for k in ("ms_momentum", "ms_restrict", "ms_poisson", "ms_prolong",
                                                         "ms_correct")},
        "phase_ms_mixed": {k: round(stmx[k], 4) for k in ("ms_momentum", "ms_restrict", "ms_poisson", "ms_prolong",
                                                          "ms_correct")},
    }
    if dom:
        line["roofline"] = {"bound": "hbm", "achieved": round(dom["achieved"], 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(dom["achieved"] / HBM_PEAK_GBS, 4),
                            "traffic": dom["traffic"], "kernel": dom["kernel"], "avg_us": round(dom["avg_us"], 3),
                            "launches": dom["launches"], "iterations": dom["iterations"],
                            "bytes_per_iteration": dom["bytes_per_iteration"],
                            "us_per_iteration": round(dom["us_per_iteration"], 3)}
    if cpu:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
