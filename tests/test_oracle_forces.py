"""Pins of the oracle's surface forces (drag and lift on the body of Section 3.3, Table 6 and
Fig. 13; wall shear for the reattachment point of Section 3.2, Fig. 7) against closed forms that
hold exactly for P1 fields:

* a constant pressure and zero velocity give no force on a closed body (the polygon's normals sum
  to zero);
* a linear pressure a + b x + c y and zero velocity give -(b, c) times the area the body's polygon
  encloses (divergence theorem, exact for the polygon and the linear field);
* a linear velocity has a constant stress, so no viscous force on a closed body either;
* simple shear u = (g y, 0) over a wall at y = 0 gives a viscous force mu g L along the wall,
  per fine edge and in total;
* the body's surface is found from coarse boundary-edge marks at any level."""
import math

import numpy as np
import pytest

import workloads as W


def _cyl_mark(mesh):
    xy, be = mesh.xy, mesh.bedge
    mid = 0.5 * (xy[be[:, 0]] + xy[be[:, 1]])
    return (np.hypot(mid[:, 0] - 0.2, mid[:, 1] - 0.2) < 0.06).astype(np.int32)


@pytest.mark.parametrize("levels", [0, 1, 2])
def test_pressure_force_on_the_cylinder(orc, levels):
    case = W.case_cylinder(2000, seed=5, levels=levels)
    P = orc.Problem(case.mesh, levels)
    P.assemble(1.0, 0.01, 1e-3)
    xy = P.export("xy")
    mark = _cyl_mark(case.mesh)
    assert mark.sum() > 8
    u0 = np.zeros((xy.shape[0], 2))
    f = P.surface_force(mark, u0, np.full(xy.shape[0], 3.7))
    assert np.abs(f).max() < 1e-14
    # the inscribed polygon of the circle: its area from the marked fine edges' vertices
    be = P.export("bedge")
    fine_mark = mark[np.arange(be.shape[0]) >> levels].astype(bool)
    pts = xy[be[fine_mark]].reshape(-1, 2)
    ang = np.arctan2(pts[:, 1] - 0.2, pts[:, 0] - 0.2)
    ring = np.unique(np.round(ang, 12), return_index=True)[1]
    q = pts[ring][np.argsort(ang[ring])]
    area = 0.5 * abs(np.sum(q[:, 0] * np.roll(q[:, 1], -1) - np.roll(q[:, 0], -1) * q[:, 1]))
    assert abs(area - math.pi * 0.05 ** 2) < 0.02 * math.pi * 0.05 ** 2
    a, b, c = 0.3, -2.0, 5.0
    f = P.surface_force(mark, u0, a + b * xy[:, 0] + c * xy[:, 1])
    np.testing.assert_allclose(f[:2], [-b * area, -c * area], rtol=1e-10)
    assert np.abs(f[2:]).max() == 0.0
    # any linear velocity: constant stress, no net viscous force on the closed body
    u = np.stack([0.4 + 1.3 * xy[:, 0] - 0.7 * xy[:, 1], -0.2 + 2.2 * xy[:, 0] - 1.3 * xy[:, 1]], 1)
    f = P.surface_force(mark, u, np.zeros(xy.shape[0]))
    assert np.abs(f).max() < 1e-13


def test_wall_shear_of_simple_shear(orc):
    case = W.case_bfs(40, 6, levels=1)
    mu, gam = 0.37, 1.9
    P = orc.Problem(case.mesh, 1)
    P.assemble(1.0, mu, 1e-3)
    xy = P.export("xy")
    xc, be = case.mesh.xy, case.mesh.bedge
    floor = ((xc[be[:, 0], 1] == 0.0) & (xc[be[:, 1], 1] == 0.0)).astype(np.int32)
    u = np.stack([gam * xy[:, 1], np.zeros(xy.shape[0])], 1)
    tr = P.surface_traction(floor, u, np.zeros(xy.shape[0]))
    assert tr.shape[0] == 2 * floor.sum()
    np.testing.assert_allclose(tr[:, 5], mu * gam * tr[:, 2], rtol=1e-12)
    np.testing.assert_allclose(tr[:, 6], 0.0, atol=1e-14)
    np.testing.assert_allclose(tr[:, 1], 0.0, atol=0)
    f = P.surface_force(floor, u, np.zeros(xy.shape[0]))
    np.testing.assert_allclose(f[2], mu * gam * 30.0, rtol=1e-12)
