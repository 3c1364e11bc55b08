"""Batched multi-instance solves (one PCG launch per iteration for all instances)
against the oracle and against the single-instance path; graph replay against
eager launches; the autotuner's cache."""
import json

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TIGHT = 1e-13


def _say(*a):
    print("[gpu-test]", *a, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch

    import oracle
    import paper_1610_06993_amd as cgp
    cgp.lib()
    oracle.lib()
    return torch, cgp, oracle


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


# uneven instances: cylinders of different sizes and seeds, a backward-facing step, and a pure-Neumann
# Taylor-Green square (no pressure-Dirichlet node)
CASES = [lambda: W.case_cylinder(2500, seed=11), lambda: W.case_cylinder(9000, seed=12),
         lambda: W.case_bfs(nx=50, ny=8), lambda: W.case_tg(n=12), lambda: W.case_cylinder(4000, seed=13)]


@pytest.fixture(scope="module")
def instances(env):
    torch, cgp, oracle = env
    out = []
    for make in CASES:
        case = make()
        g = cgp.Mesh(case.mesh, 1)
        g.assemble(case.rho, case.mu, case.dt)
        o = oracle.Problem(case.mesh, 1)
        o.assemble(case.rho, case.mu, case.dt, 0, 0)
        out.append((case, g, o))
    _say("instances (coarse nodes):", [g.info["n_c"] for _, g, _ in out])
    return out


def _rhs(instances, seed):
    rng = np.random.default_rng(seed)
    return [rng.normal(size=g.info["n_c"]) for _, g, _ in instances]


def test_batch_poisson_matches_oracle(env, instances):
    torch, cgp, oracle = env
    batch = cgp.Batch([g for _, g, _ in instances])
    bs = _rhs(instances, 1)
    xs = [torch.zeros(len(b), dtype=torch.float64, device="cuda") for b in bs]
    st = batch.poisson_solve([dev(torch, b) for b in bs], xs, cgp.SolverOpts(tol=TIGHT, max_iter=100000,
                                                                             x0_mode=cgp._native.X0_ZERO))
    for (case, g, o), b, x, s in zip(instances, bs, xs, st):
        ref, code, its, rr = o.poisson_solve(b, tol=1e-14)
        err = rel(x.cpu().numpy(), ref)
        _say(f"  n_c {len(b)}: batch iterations {s['p_iters']}, oracle {its}, rel err {err:.2e}")
        assert code == 0 and s["p_iters"] > 0 and s["p_relres"] <= TIGHT * 1.0001
        assert err <= 1e-10
    batch.close()


def test_batch_equals_single_instance_solves(env, instances):
    """Same kernels' arithmetic per instance: the batch and the single-mesh solver agree to rounding."""
    torch, cgp, oracle = env
    batch = cgp.Batch([g for _, g, _ in instances])
    bs = _rhs(instances, 2)
    opts = cgp.SolverOpts(tol=1e-10, max_iter=100000, x0_mode=cgp._native.X0_ZERO)
    xs = [torch.zeros(len(b), dtype=torch.float64, device="cuda") for b in bs]
    st = batch.poisson_solve([dev(torch, b) for b in bs], xs, opts)
    for (case, g, o), b, x, s in zip(instances, bs, xs, st):
        y = torch.zeros_like(x)
        s1 = g.poisson_solve(dev(torch, b), y, opts)
        assert abs(s1["p_iters"] - s["p_iters"]) <= 2, (s1["p_iters"], s["p_iters"])
        assert rel(x.cpu().numpy(), y.cpu().numpy()) <= 1e-8
    batch.close()


def test_batch_fp32_refinement(env, instances):
    """Every instance's FP32 inner solves batched inside its own FP64 refinement: each solution within
    1e-6 of the oracle, refinement counts close to the single-instance refinement."""
    torch, cgp, oracle = env
    batch = cgp.Batch([g for _, g, _ in instances])
    bs = _rhs(instances, 5)
    opts = cgp.SolverOpts(tol=1e-10, max_iter=100000, precision=cgp._native.PREC_FP32_IR,
                          x0_mode=cgp._native.X0_ZERO)
    xs = [torch.zeros(len(b), dtype=torch.float64, device="cuda") for b in bs]
    st = batch.poisson_solve([dev(torch, b) for b in bs], xs, opts)
    for (case, g, o), b, x, s in zip(instances, bs, xs, st):
        ref, code, its, rr = o.poisson_solve(b, tol=1e-14)
        y = torch.zeros_like(x)
        s1 = g.poisson_solve(dev(torch, b), y, opts)
        err = rel(x.cpu().numpy(), ref)
        _say(f"  n_c {len(b)}: batched refinement {s['p_outer']} checks / {s['p_iters']} inner iterations, "
             f"single {s1['p_outer']} / {s1['p_iters']}; rel err vs oracle {err:.2e}")
        assert code == 0 and s["p_relres"] <= 1e-10 and err <= 1e-6
        assert abs(s["p_outer"] - s1["p_outer"]) <= 1
    batch.close()


@pytest.mark.parametrize("lanes,block,passes,ahead", [(4, 512, 2, 0), (2, 512, 2, 0), (4, 512, 2, 1), (8, 256, 4, 1),
                                                      (4, 1024, 1, 1), (4, 256, 4, 2), (8, 512, 2, 2),
                                                      (8, 256, 8, 1), (8, 1024, 8, 2)])
def test_batch_kernel_forms(env, instances, lanes, block, passes, ahead):
    """Both forms of the batched iteration (the row loop and the loads-ahead kernel) at several launch
    shapes: per-instance solutions <= 1e-10 from the oracle in FP64, <= 1e-6 with the FP32 inner solves."""
    torch, cgp, oracle = env
    X0 = cgp._native
    batch = cgp.Batch([g for _, g, _ in instances])
    batch.set_tuning(lanes=lanes, block=block, passes=passes, ahead=ahead)
    bs = _rhs(instances, 9)
    for prec, tol, bar in ((X0.PREC_FP64, TIGHT, 1e-10), (X0.PREC_FP32_IR, 1e-10, 1e-6)):
        xs = [torch.zeros(len(b), dtype=torch.float64, device="cuda") for b in bs]
        st = batch.poisson_solve([dev(torch, b) for b in bs], xs, cgp.SolverOpts(tol=tol, max_iter=100000, precision=prec,
                                                                                 x0_mode=X0.X0_ZERO))
        errs = []
        for (case, g, o), b, x, s in zip(instances, bs, xs, st):
            ref, code, its, rr = o.poisson_solve(b, tol=1e-14)
            errs.append(rel(x.cpu().numpy(), ref))
            assert code == 0
        _say(f"  shape {lanes}/{block}/{passes} ahead {ahead} precision {prec}: worst rel err {max(errs):.2e}, "
             f"iterations {[s['p_iters'] for s in st]}")
        assert max(errs) <= bar
    batch.close()


def test_graph_replays_equal_eager(env, instances):
    torch, cgp, oracle = env
    batch = cgp.Batch([g for _, g, _ in instances])
    bs = [dev(torch, b) for b in _rhs(instances, 3)]
    opts = cgp.SolverOpts(tol=1e-11, max_iter=100000, x0_mode=cgp._native.X0_ZERO)

    def run():
        xs = [torch.zeros(b.shape[0], dtype=torch.float64, device="cuda") for b in bs]
        st = batch.poisson_solve(bs, xs, opts)
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in xs], [s["p_iters"] for s in st]

    batch.set_tuning(use_graph=0)
    ref, its = run()
    batch.set_tuning(use_graph=1)
    for rep in range(3):
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work between the replays
        got, its2 = run()
        assert its2 == its
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), rep
    batch.close()


def test_batch_step_matches_single_steps(env, instances):
    torch, cgp, oracle = env
    sub = [instances[0], instances[2], instances[4]]
    opts = cgp.StepOpts(momentum=cgp.SolverOpts(tol=TIGHT, max_iter=100000),
                        poisson=cgp.SolverOpts(tol=1e-14, max_iter=100000),
                        mass=cgp.SolverOpts(tol=TIGHT, max_iter=100000))
    states = {}
    for mode in ("batch", "single"):
        us, pfs, pcs, gds = [], [], [], []
        for case, g, o in sub:
            xy = g.export("xy")
            us.append(dev(torch, case.initial(xy, g.export("vdir"))))
            pfs.append(torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda"))
            pcs.append(torch.zeros(g.info["n_c"], dtype=torch.float64, device="cuda"))
        batch = cgp.Batch([g for _, g, _ in sub]) if mode == "batch" else None
        for k in range(3):
            gds = [dev(torch, case.dirichlet(g.export("xy"), (k + 1) * case.dt)) for case, g, _ in sub]
            if batch:
                batch.step(gds, us, pfs, pcs, opts=opts)
            else:
                for (case, g, o), gd, u, pf, pc in zip(sub, gds, us, pfs, pcs):
                    g.step(gd, u, pf, pc, opts=opts)
        if batch:
            batch.close()
        states[mode] = [(u.cpu().numpy(), pf.cpu().numpy()) for u, pf in zip(us, pfs)]
    for (ub, pb), (us_, ps) in zip(states["batch"], states["single"]):
        assert rel(ub, us_) <= 1e-10 and rel(pb, ps) <= 1e-10


def test_batch_step_solver_options_match_single_steps(env, instances):
    """The per-instance phases of a batch step honour the momentum and mass options as a single step
    does: FP32 inner BiCGStab inside FP64 refinement for the momentum solve and the extrapolated mass
    start, three steps, batched against single-instance steps (the batched Poisson solve differs only
    in its reduction order)."""
    torch, cgp, oracle = env
    X0 = cgp._native
    sub = [instances[0], instances[2], instances[4]]
    opts = cgp.StepOpts(momentum=cgp.SolverOpts(tol=TIGHT, max_iter=100000, precision=X0.PREC_FP32_IR),
                        poisson=cgp.SolverOpts(tol=1e-13, max_iter=100000),
                        mass=cgp.SolverOpts(tol=TIGHT, max_iter=100000, x0_mode=X0.X0_EXTRAP))
    states = {}
    for mode in ("batch", "single"):
        us, pfs, pcs = [], [], []
        for case, g, o in sub:
            us.append(dev(torch, case.initial(g.export("xy"), g.export("vdir"))))
            pfs.append(torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda"))
            pcs.append(torch.zeros(g.info["n_c"], dtype=torch.float64, device="cuda"))
        batch = cgp.Batch([g for _, g, _ in sub]) if mode == "batch" else None
        try:
            for k in range(3):
                gds = [dev(torch, case.dirichlet(g.export("xy"), (k + 1) * case.dt)) for case, g, _ in sub]
                if batch:
                    batch.step(gds, us, pfs, pcs, opts=opts)
                else:
                    for (case, g, o), gd, u, pf, pc in zip(sub, gds, us, pfs, pcs):
                        g.step(gd, u, pf, pc, opts=opts)
        finally:
            if batch:
                batch.close()
        states[mode] = [(u.cpu().numpy(), pf.cpu().numpy()) for u, pf in zip(us, pfs)]
    errs = [max(rel(ub, us_), rel(pb, ps)) for (ub, pb), (us_, ps) in zip(states["batch"], states["single"])]
    _say(f"  FP32-refined momentum, extrapolated mass start: batch vs single worst rel err {max(errs):.1e}")
    assert max(errs) <= 1e-9


def test_batch_step_online_guess_matches_single_steps(env, instances):
    """Every instance keeps its own online POD basis (window 4); inside the batched solve each instance's
    initial guess comes from it exactly as in its single solve.  After the windows fill, the batched
    steps agree with single-instance steps, and the guess cuts the Poisson iterations."""
    torch, cgp, oracle = env
    sub = [instances[0], instances[2], instances[4]]
    X0 = cgp._native

    def opts(x0):
        return cgp.StepOpts(momentum=cgp.SolverOpts(tol=TIGHT, max_iter=100000),
                            poisson=cgp.SolverOpts(tol=1e-12, max_iter=100000, x0_mode=x0),
                            mass=cgp.SolverOpts(tol=TIGHT, max_iter=100000))

    states, iters = {}, {}
    for mode in ("batch", "single", "batch_prev"):
        guesses, us, pfs, pcs = [], [], [], []
        for case, g, o in sub:
            gs = cgp.Guess(g, n_modes=4, hidden=16, seed=3)
            gs.set_online(4, 1)
            gs.attach()
            guesses.append(gs)
            us.append(dev(torch, case.initial(g.export("xy"), g.export("vdir"))))
            pfs.append(torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda"))
            pcs.append(torch.zeros(g.info["n_c"], dtype=torch.float64, device="cuda"))
        x0 = X0.X0_PREV if mode == "batch_prev" else X0.X0_POD_GALERKIN
        batch = cgp.Batch([g for _, g, _ in sub]) if mode != "single" else None
        last = []
        try:
            for k in range(9):
                gds = [dev(torch, case.dirichlet(g.export("xy"), (k + 1) * case.dt)) for case, g, _ in sub]
                if batch:
                    st = batch.step(gds, us, pfs, pcs, opts=opts(x0))
                else:
                    st = [g.step(gd, u, pf, pc, opts=opts(x0)) for (case, g, o), gd, u, pf, pc in
                          zip(sub, gds, us, pfs, pcs)]
                if k >= 6:
                    last.append([s["p_iters"] for s in st])
        finally:
            if batch:
                batch.close()
            for gs in guesses:
                gs.detach()
                gs.close()
        states[mode] = [(u.cpu().numpy(), pf.cpu().numpy()) for u, pf in zip(us, pfs)]
        iters[mode] = np.sum(last, axis=0)
    _say("  Poisson iterations of the last 3 steps: batch+online", iters["batch"], "single+online",
         iters["single"], "batch, previous pressure", iters["batch_prev"])
    for (ub, pb), (us_, ps) in zip(states["batch"], states["single"]):
        assert rel(ub, us_) <= 1e-9 and rel(pb, ps) <= 1e-9
    assert np.all(np.abs(iters["batch"] - iters["single"]) <= 6)
    assert iters["batch"].sum() < iters["batch_prev"].sum()


def test_batch_step_learned_guess_per_instance_matches_single_steps(env, instances):
    """Every instance with its own trained network (a POD basis of its own recorded pressures and an
    MLP trained on the GPU from its recorded right-hand sides): inside the batched solve each instance
    forms its initial guess from its own model (CGP_X0_LEARNED) as in its single step; three batched
    steps agree with three single-instance steps, and the guess changes where the solves start (the
    Poisson counts differ from the previous-pressure start)."""
    torch, cgp, oracle = env
    X0 = cgp._native
    sub = [instances[0], instances[4]]
    rec_opts = cgp.StepOpts(momentum=cgp.SolverOpts(tol=TIGHT, max_iter=100000),
                            poisson=cgp.SolverOpts(tol=1e-12, max_iter=100000),
                            mass=cgp.SolverOpts(tol=TIGHT, max_iter=100000))
    models, starts = [], []
    for case, g, o in sub:
        xy = g.export("xy")
        u = dev(torch, case.initial(xy, g.export("vdir")))
        pf = torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda")
        pc = torch.zeros(g.info["n_c"], dtype=torch.float64, device="cuda")
        n = g.info["n_c"]
        B = torch.zeros((24, n), dtype=torch.float64, device="cuda")
        P = torch.zeros_like(B)
        for k in range(24):
            g.step(dev(torch, case.dirichlet(xy, (k + 1) * case.dt)), u, pf, pc, opts=rec_opts)
            g.last_poisson_rhs(B[k])
            P[k].copy_(pc)
        net = cgp.Guess(g, n_modes=8, hidden=32, seed=7)
        net.build_pod(P.contiguous())
        net.train(B.contiguous(), P.contiguous(), epochs=40, batch=8)
        models.append(net)
        starts.append((u.clone(), pc.clone()))
    opts = {x0: cgp.StepOpts(momentum=cgp.SolverOpts(tol=TIGHT, max_iter=100000),
                             poisson=cgp.SolverOpts(tol=1e-12, max_iter=100000, x0_mode=x0),
                             mass=cgp.SolverOpts(tol=TIGHT, max_iter=100000)) for x0 in (X0.X0_LEARNED, X0.X0_PREV)}
    states, iters = {}, {}
    try:
        for mode, x0 in (("batch", X0.X0_LEARNED), ("single", X0.X0_LEARNED), ("batch_prev", X0.X0_PREV)):
            for net in models:
                net.attach()
            us = [st[0].clone() for st in starts]
            pcs = [st[1].clone() for st in starts]
            pfs = [torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda") for _, g, _ in sub]
            batch = cgp.Batch([g for _, g, _ in sub]) if mode != "single" else None
            its = []
            try:
                for k in range(24, 27):
                    gds = [dev(torch, case.dirichlet(g.export("xy"), (k + 1) * case.dt)) for case, g, _ in sub]
                    if batch:
                        st = batch.step(gds, us, pfs, pcs, opts=opts[x0])
                    else:
                        st = [g.step(gd, u, pf, pc, opts=opts[x0]) for (case, g, o), gd, u, pf, pc in
                              zip(sub, gds, us, pfs, pcs)]
                    its.append([s_["p_iters"] for s_ in st])
            finally:
                if batch:
                    batch.close()
                for net in models:
                    net.detach()
            states[mode] = [(u.cpu().numpy(), pf.cpu().numpy()) for u, pf in zip(us, pfs)]
            iters[mode] = its
    finally:
        for net in models:
            net.close()
    _say(f"  Poisson iterations, learned start batch {iters['batch']}, single {iters['single']}, previous "
         f"pressure {iters['batch_prev']}")
    for (ub, pb), (us_, ps) in zip(states["batch"], states["single"]):
        assert rel(ub, us_) <= 1e-9 and rel(pb, ps) <= 1e-9
    assert np.all(np.abs(np.array(iters["batch"]) - np.array(iters["single"])) <= 6)
    assert iters["batch"] != iters["batch_prev"]


def test_autotune_cache(env, instances, tmp_path):
    torch, cgp, oracle = env
    batch = cgp.Batch([g for _, g, _ in instances])
    cache = tmp_path / "tune.json"
    chosen = batch.autotune(cache)
    _say("  autotuned:", chosen)
    data = json.loads(cache.read_text())
    assert len(data) == 1
    entry = next(iter(data.values()))
    assert {"lanes", "block", "passes", "ahead", "candidates"} <= set(entry) and len(entry["candidates"]) == 69
    assert (entry["lanes"], entry["block"], entry["passes"], entry["ahead"]) == (chosen["lanes"], chosen["block"], chosen["passes"], chosen["ahead"])
    batch.set_tuning(lanes=16, block=64, passes=3, ahead=0)
    again = batch.autotune(cache)   # from the cache: same choice, no timing
    assert (again["lanes"], again["block"], again["passes"], again["ahead"]) == \
        (chosen["lanes"], chosen["block"], chosen["passes"], chosen["ahead"])
    # the tuned batch still solves correctly
    bs = _rhs(instances, 4)
    xs = [torch.zeros(len(b), dtype=torch.float64, device="cuda") for b in bs]
    batch.poisson_solve([dev(torch, b) for b in bs], xs, cgp.SolverOpts(tol=TIGHT, max_iter=100000,
                                                                        x0_mode=cgp._native.X0_ZERO))
    for (case, g, o), b, x in zip(instances, bs, xs):
        ref, code, its, rr = o.poisson_solve(b, tol=1e-14)
        assert rel(x.cpu().numpy(), ref) <= 1e-10
    batch.close()


DECILE_STEPS = 6


@pytest.fixture(scope="module")
def deciles(env):
    """One instance per size decile of the 64-instance sweep (coarse 19k to 201k triangles, Re in
    [60, 160]) and the oracle's trajectory of each over the first steps, computed once on host threads
    (one per instance) and shared by the batched paths."""
    from concurrent.futures import ThreadPoolExecutor

    torch, cgp, oracle = env
    idx = W.batch_deciles()
    cases = [W.batch_instance(i) for i in idx]
    meshes, probs = [], []
    for case in cases:
        g = cgp.Mesh(case.mesh, 1)
        g.assemble(case.rho, case.mu, case.dt)
        o = oracle.Problem(case.mesh, 1)
        o.assemble(case.rho, case.mu, case.dt, 0, 0)
        meshes.append(g)
        probs.append(o)
    _say(f"batch deciles: instances {idx}, coarse nodes {[g.info['n_c'] for g in meshes]}; oracle trajectories")
    xys = [g.export("xy") for g in meshes]

    def trajectory(j):
        case, o, xy = cases[j], probs[j], xys[j]
        u, pc, out = case.initial(xy, meshes[j].export("vdir")), None, []
        for k in range(DECILE_STEPS):
            gd = case.dirichlet(xy, (k + 1) * case.dt)
            un, pf, pcn, code, _ = o.step(gd, u, pc, tol_mom=1e-13, tol_p=1e-14, tol_mass=1e-13)
            assert code == 0
            out.append(dict(gd=gd, u=u, pc=pc, u_next=un, pf_next=pf))
            u, pc = un, pcn
        return out

    with ThreadPoolExecutor(max_workers=len(cases)) as pool:
        trajs = list(pool.map(trajectory, range(len(cases))))
    return cases, meshes, trajs


@pytest.mark.parametrize("path", ["online", "mixed+online"])
def test_batch_size_deciles_against_oracle(env, deciles, path):
    """The ten decile instances stepped together in one batch with per-instance online POD guesses
    (window 4), FP64 or with the batched FP32 inner solves inside each instance's FP64 refinement.
    Every step starts all instances from the oracle's state of the step before, so each comparison is
    one step's local error: <= 1e-10 for FP64, <= 1e-6 for the FP32 refinement (its tolerance 1e-10
    times the condition of the coarse Laplacian)."""
    torch, cgp, oracle = env
    X0 = cgp._native
    cases, meshes, trajs = deciles
    mixed = path.startswith("mixed")
    poisson = cgp.SolverOpts(tol=1e-10 if mixed else 1e-13, max_iter=100000, x0_mode=X0.X0_POD_GALERKIN,
                             precision=X0.PREC_FP32_IR if mixed else X0.PREC_FP64)
    tight = cgp.SolverOpts(tol=1e-13, max_iter=100000)
    opts = cgp.StepOpts(momentum=tight, poisson=poisson, mass=tight)
    bar = 1e-6 if mixed else 1e-10
    guesses = []
    for g in meshes:
        gs = cgp.Guess(g, n_modes=4, hidden=16, seed=3)
        gs.set_online(4, 1)
        gs.attach()
        guesses.append(gs)
    batch = cgp.Batch(meshes)
    try:
        for k in range(DECILE_STEPS):
            rows = [t[k] for t in trajs]
            us = [dev(torch, r["u"].copy()) for r in rows]
            pcs = [dev(torch, r["pc"].copy()) if r["pc"] is not None else
                   torch.zeros(g.info["n_c"], dtype=torch.float64, device="cuda") for r, g in zip(rows, meshes)]
            pfs = [torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda") for g in meshes]
            st = batch.step([dev(torch, r["gd"]) for r in rows], us, pfs, pcs, opts=opts)
            errs = [max(rel(u.cpu().numpy(), r["u_next"]), rel(pf.cpu().numpy(), r["pf_next"]))
                    for u, pf, r in zip(us, pfs, rows)]
            _say(f"  {path} step {k + 1}: worst rel err {max(errs):.2e}, Poisson iterations "
                 f"{[s['p_iters'] for s in st]}")
            assert max(errs) <= bar
    finally:
        batch.close()
        for gs in guesses:
            gs.detach()
            gs.close()
