"""The paper's solver on the GPU: ILU(0)-preconditioned GMRES(m) for the coarse Poisson equation
(Eq. 21; Section 2.3), through cgp_poisson_solve with CGP_METHOD_ILU_GMRES: the device's level-scheduled
ILU(0) factors against the oracle's (<= 1e-12), the solution against the oracle's Poisson solution
(<= 1e-10 at tolerance 1e-13), and the iteration count against the oracle's ILU(0)-GMRES with the same
orthogonalisation (classical Gram-Schmidt done twice; restarted GMRES on these stagnating systems is
sensitive to rounding, so the counts are compared within 10 %); pure Neumann and outflow pressure; two
restart lengths; a re-assembled mesh is re-factorised; a whole CGP step with it matches the oracle."""
import numpy as np
import pytest

import workloads as W
from parity_cases import CYLINDER_CASE, make

pytestmark = pytest.mark.gpu


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
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


# restarted GMRES on the graded cylinder is chaotic in its iteration count at short restarts (the oracle's
# own count moves between 827 and 1338 at restart 30 under 1e-15 relative perturbations of b), so counts
# are compared where they are stable (measured over five perturbations: Taylor-Green at 30 and 8,
# the cylinder at 60) and only the solution where they are not
@pytest.mark.parametrize("which,restart,count", [("neumann", 30, True), ("neumann", 8, True),
                                                 ("dirichlet", 60, True), ("dirichlet", 8, False)])
def test_ilu_gmres_poisson(env, which, restart, count):
    torch, cgp, oracle = env
    mesh = W.unit_square_tg(16, seed=3) if which == "neumann" else W.cylinder_channel(3000, seed=2)
    _say("ILU(0)-GMRES", which, "restart", restart)
    g = cgp.Mesh(mesh, 1)
    g.assemble(1.0, 1e-3, 1e-3)
    o = oracle.Problem(mesh, 1)
    o.assemble(1.0, 1e-3, 1e-3)
    n = g.info["n_c"]
    b = np.random.default_rng(7).normal(size=n)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    X0 = cgp._native
    st = g.poisson_solve(torch.from_numpy(b).cuda(), x, cgp.SolverOpts(tol=1e-13, max_iter=100000, x0_mode=X0.X0_ZERO,
                                                                       method=X0.METHOD_ILU_GMRES, restart=restart))
    ref, code, it, rr = o.poisson_solve(b, tol=1e-14)
    assert code == 0
    e = rel(x.cpu().numpy(), ref)
    # the factors, and the oracle's ILU(0)-GMRES on the same eliminated system
    rp, col, K = o.export("rowptr_c"), o.export("col_c"), o.values("K_c_bc")
    lu_ref = oracle.ilu0(rp, col, K)
    lu = g.export("ilu_c")
    e_lu = float(np.abs(lu - lu_ref).max() / np.abs(lu_ref).max())
    pdir = o.export("pdir").astype(bool)
    bb = b.copy()
    if pdir.any():
        bb[pdir] = 0.0
    else:
        bb -= bb.mean()
    _, ocode, oit, _ = oracle.gmres(rp, col, K, bb, m=restart, tol=1e-13, orth="cgs2")
    _, _, oit_mgs, _ = oracle.gmres(rp, col, K, bb, m=restart, tol=1e-13, orth="mgs")
    _say(f"  rel err {e:.2e}, factors {e_lu:.1e}; iterations GPU {st['p_iters']}, oracle GMRES {oit} (modified "
         f"Gram-Schmidt {oit_mgs}), oracle PCG {it}")
    assert e_lu <= 1e-12
    assert e <= 1e-10 and st["p_relres"] <= 1e-13
    assert ocode == 0
    if count:
        assert abs(st["p_iters"] - oit) <= max(2, 0.10 * oit)


def test_ilu_gmres_refactorised_after_assembly_and_in_a_step(env):
    torch, cgp, oracle = env
    case = make(CYLINDER_CASE)
    X0 = cgp._native
    g = cgp.Mesh(case.mesh, 1)
    o = oracle.Problem(case.mesh, 1)
    # a first assembly with another viscosity and dt (another Kbar scaling does not change Kbar, but the
    # factorisation must be redone from the new operators anyway), then the real one
    g.assemble(case.rho, 10 * case.mu, 2 * case.dt)
    n = g.info["n_c"]
    b = torch.from_numpy(np.random.default_rng(2).normal(size=n)).cuda()
    g.poisson_solve(b, torch.zeros_like(b), cgp.SolverOpts(tol=1e-10, method=X0.METHOD_ILU_GMRES))
    g.assemble(case.rho, case.mu, case.dt)
    o.assemble(case.rho, case.mu, case.dt)
    xy = g.export("xy")
    u0 = case.initial(xy, g.export("vdir"))
    u = torch.from_numpy(u0.copy()).cuda()
    pf = torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda")
    pc = torch.zeros(n, dtype=torch.float64, device="cuda")
    s = cgp.SolverOpts(tol=1e-13, max_iter=100000)
    # GMRES stops on the true residual ||b - A x||, which on this right-hand side cannot go much below
    # 1e-16 ||A|| ||x|| / ||b|| ~ 1e-11 (the ratio is about 1.3e5 at the first step: restarted GMRES
    # stagnates at a true relative residual of 3e-13); 1e-12 is reached and puts the pressure within
    # 2e-13 of the oracle's PCG solution
    opts = cgp.StepOpts(momentum=s, poisson=cgp.SolverOpts(tol=1e-12, max_iter=20000, method=X0.METHOD_ILU_GMRES,
                                                           restart=60), mass=s)
    ur, pcr = u0.copy(), None
    for k in range(3):
        gd = case.dirichlet(xy, (k + 1) * case.dt)
        g.step(torch.from_numpy(gd).cuda(), u, pf, pc, opts=opts)
        ur, pfr, pcr, code, _ = o.step(gd, ur, pcr, tol_mom=1e-13, tol_p=1e-14, tol_mass=1e-13)
        assert code == 0
        eu, ep = rel(u.cpu().numpy(), ur), rel(pf.cpu().numpy(), pfr)
        _say(f"  step {k + 1}: rel err u {eu:.2e}, p {ep:.2e}")
        assert eu <= 1e-10 and ep <= 1e-10


def test_ilu_gmres_arguments(env):
    torch, cgp, oracle = env
    X0 = cgp._native
    g = cgp.Mesh(W.unit_square_tg(6), 1)
    g.assemble(1.0, 0.01, 1e-3)
    b = torch.ones(g.info["n_c"], dtype=torch.float64, device="cuda")
    for o in (cgp.SolverOpts(method=X0.METHOD_ILU_GMRES, precision=X0.PREC_FP32_IR),
              cgp.SolverOpts(method=X0.METHOD_ILU_GMRES, restart=201), cgp.SolverOpts(method=7)):
        with pytest.raises(cgp.CGPError):
            g.poisson_solve(b, torch.zeros_like(b), o)
    with pytest.raises(cgp.CGPError):  # the momentum solve has no GMRES
        u = torch.zeros((g.info["n_f"], 2), dtype=torch.float64, device="cuda")
        g.momentum(u, u, torch.zeros_like(u), opts=cgp.SolverOpts(method=X0.METHOD_ILU_GMRES))
