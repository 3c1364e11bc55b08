"""Flow functionals on the GPU (drag and lift on the cylinder with their pressure and viscous parts;
wall traction along the floor behind the backward-facing step) against the oracle's surface forces
on the same velocity and pressure fields, after a few GPU steps; per edge and in total, <= 1e-12
relative (one pass over the edges: only the summation order differs)."""
import numpy as np
import pytest

import workloads as W
from parity_cases import CYLINDER_CASE, STEP_VARIANT_CASE, make

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


def _run(env, case, levels, steps, ids):
    torch, cgp, oracle = env
    g = cgp.Mesh(case.mesh, levels)
    g.assemble(case.rho, case.mu, case.dt)
    o = oracle.Problem(case.mesh, levels)
    o.assemble(case.rho, case.mu, case.dt)
    xy = g.export("xy")
    u = torch.from_numpy(case.initial(xy, g.export("vdir"))).cuda()
    pf = torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda")
    pc = torch.zeros(g.info["n_c"], dtype=torch.float64, device="cuda")
    gd = torch.from_numpy(case.dirichlet(xy, case.dt)).cuda()
    for _ in range(steps):
        g.step(gd, u, pf, pc)
    g.surface_set(ids)
    rows = g.surface_traction(u, pf).cpu().numpy()
    tot = g.surface_force(u, pf)
    mark = np.zeros(case.mesh.bedge.shape[0], np.int32)
    mark[ids] = 1
    un, pn = u.cpu().numpy(), pf.cpu().numpy()
    ref_rows = o.surface_traction(mark, un, pn)
    ref_tot = o.surface_force(mark, un, pn)
    return rows, tot, ref_rows, ref_tot


def test_cylinder_drag_and_lift(env):
    case = make(CYLINDER_CASE)
    xy, be = case.mesh.xy, case.mesh.bedge
    mid = 0.5 * (xy[be[:, 0]] + xy[be[:, 1]])
    ids = np.where(np.hypot(mid[:, 0] - 0.2, mid[:, 1] - 0.2) < 0.06)[0]
    _say("cylinder surface forces,", ids.size, "coarse body edges")
    rows, tot, ref_rows, ref_tot = _run(env, case, 1, 4, ids)
    assert rows.shape == ref_rows.shape == (2 * ids.size, 8)
    np.testing.assert_allclose(rows, ref_rows, rtol=1e-12, atol=1e-15 * np.abs(ref_rows).max())
    np.testing.assert_allclose(tot, ref_tot, rtol=1e-12, atol=1e-14 * np.abs(ref_tot).max())
    _say("  forces (pressure x, y, viscous x, y):", tot)
    assert tot[0] > 0 and tot[2] > 0  # drag: both parts push the body downstream


def test_floor_traction_behind_the_step(env):
    case = make(STEP_VARIANT_CASE)
    xy, be = case.mesh.xy, case.mesh.bedge
    ids = np.where((xy[be[:, 0], 1] == 0.0) & (xy[be[:, 1], 1] == 0.0))[0]
    _say("backward-facing step floor traction,", ids.size, "coarse edges, l = 2")
    rows, tot, ref_rows, ref_tot = _run(env, case, 2, 3, ids)
    assert rows.shape[0] == 4 * ids.size
    np.testing.assert_allclose(rows, ref_rows, rtol=1e-12, atol=1e-15 * np.abs(ref_rows).max())
    np.testing.assert_allclose(tot, ref_tot, rtol=1e-12, atol=1e-14 * np.abs(ref_tot).max())


def test_surface_arguments(env):
    torch, cgp, oracle = env
    g = cgp.Mesh(W.unit_square_tg(4), 1)
    g.assemble(1.0, 0.01, 1e-3)
    with pytest.raises(cgp.CGPError):
        g.surface_set([10_000])
    u = torch.zeros((g.info["n_f"], 2), dtype=torch.float64, device="cuda")
    p = torch.zeros(g.info["n_f"], dtype=torch.float64, device="cuda")
    assert not g.surface_force(u, p).any()  # nothing marked
    g.surface_set(np.arange(g.export("bedge", 0).shape[0]))
    p.fill_(2.0)
    assert np.abs(g.surface_force(u, p)).max() < 1e-14  # closed surface, constant pressure
