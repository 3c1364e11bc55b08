"""Pins of the oracle's incremental pressure-correction schemes (the extension Remark 3.1 and the
paper's conclusions point to: standard and rotational incremental forms inside CGP).

* Taylor-Green (Eqs. 34-36, all-Dirichlet velocity): with the transpose-of-prolongation restriction
  the l = 1 velocity/pressure pair is the inf-sup stable P1-iso-P2/P1 pair, and the incremental
  scheme removes the first-order splitting error of the non-incremental one: at dt = 1e-2 its
  velocity error is well below the non-incremental error and no longer depends on dt, while the
  non-incremental error still falls as dt is refined (Remark 3.1: its time error dominates with
  Dirichlet boundaries).
* The rotational update subtracts mu times the lumped L2 projection of div U~: for a linear field
  (a x, b y) that is mu (a + b) at coarse nodes away from the boundary, whichever restriction.
* l = 0 with zero pressure history: the first incremental step equals the non-incremental step.
"""
import numpy as np
import pytest

import workloads as W


def _tg_error(orc, dt, pmode, n=16, T=0.1):
    case = W.case_tg(n, levels=1, dt=dt)
    P = orc.Problem(case.mesh, 1)
    P.assemble(case.rho, case.mu, dt, 1, 0, pmode)
    xy, xc = P.export("xy"), P.export("xy", 0)
    u = W.tg_velocity(xy, 0.0, case.mu)
    pc = W.tg_pressure(xc, 0.0, case.mu) if pmode else np.zeros(P.info["n_c"])
    for k in range(1, int(round(T / dt)) + 1):
        u, pf, pc, code, _ = P.step(W.tg_velocity(xy, k * dt, case.mu), u, pc, tol_mom=1e-12, tol_p=1e-12,
                                    tol_mass=1e-12)
        assert code == 0
    l2, _ = P.error_norms(u, lambda q: W.tg_velocity(q, T, case.mu))
    return l2


def test_incremental_removes_the_splitting_error_on_taylor_green(orc):
    e0 = {dt: _tg_error(orc, dt, 0) for dt in (1e-2, 2.5e-3)}
    e1 = {dt: _tg_error(orc, dt, 1) for dt in (1e-2, 2.5e-3)}
    e2 = _tg_error(orc, 1e-2, 2)
    assert e1[1e-2] < 0.6 * e0[1e-2], (e0, e1)
    assert e2 < 0.6 * e0[1e-2], (e0, e2)
    # non-incremental: the error still falls with dt; incremental: at the spatial floor already
    assert e0[1e-2] > 1.5 * e0[2.5e-3], e0
    assert abs(e1[1e-2] - e1[2.5e-3]) < 0.1 * e1[2.5e-3], e1


@pytest.mark.parametrize("rmode", [0, 1])
def test_rotational_update_subtracts_mu_div(orc, rmode):
    case = W.case_bfs(30, 6, levels=1)
    rho, mu, dt = 1.0, 0.37, 0.01
    P = orc.Problem(case.mesh, 1)
    P.assemble(rho, mu, dt, rmode, 0, 2)
    xy = P.export("xy")
    a, b = 0.8, -2.1
    ut = np.stack([a * xy[:, 0], b * xy[:, 1]], 1)
    bc = P.restrict(ut, rmode)
    pc0 = np.random.default_rng(2).normal(size=P.info["n_c"])
    phi = np.zeros_like(pc0)
    pc1 = P.pressure_update(bc, phi, pc0)
    # coarse nodes whose coarse triangles all lie inside: their test function sees the constant divergence
    tri_c = P.export("tri", 0)
    onb = np.zeros(P.info["n_c"], bool)
    onb[P.export("bedge", 0).ravel()] = True
    near = np.zeros_like(onb)
    for t in tri_c:
        if onb[t].any():
            near[t] = True
    inner = ~near
    assert inner.sum() > 50
    np.testing.assert_allclose(pc1[inner] - pc0[inner], -mu * (a + b), rtol=1e-11)
    pdir = P.export("pdir").astype(bool)
    assert not pc1[pdir].any()
    # the standard form leaves the previous pressure plus the increment
    P.assemble(rho, mu, dt, rmode, 0, 1)
    inc = np.random.default_rng(3).normal(size=pc0.size)
    pc2 = P.pressure_update(bc, inc, pc0)
    np.testing.assert_array_equal(pc2[~pdir], (pc0 + inc)[~pdir])


def test_first_incremental_step_from_zero_pressure_is_the_plain_step(orc):
    case = W.case_cylinder(1500, seed=5, levels=1)
    outs = []
    for pmode in (0, 1):
        P = orc.Problem(case.mesh, 1)
        P.assemble(case.rho, case.mu, case.dt, 1, 0, pmode)
        xy, vd = P.export("xy"), P.export("vdir")
        u0 = case.initial(xy, vd)
        u, pf, pc, code, _ = P.step(case.dirichlet(xy, case.dt), u0, np.zeros(P.info["n_c"]), tol_mom=1e-13,
                                    tol_p=1e-13, tol_mass=1e-13)
        assert code == 0
        outs.append((u, pf))
    assert np.linalg.norm(outs[0][0] - outs[1][0]) <= 1e-11 * np.linalg.norm(outs[0][0])
    assert np.linalg.norm(outs[0][1] - outs[1][1]) <= 1e-9 * np.linalg.norm(outs[0][1])
