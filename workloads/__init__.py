"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module produces *inputs only*: coarse P1 triangle meshes, boundary-edge
tags, Dirichlet data and initial states shaped like the paper's three test
cases (Taylor-Green vortex, backward-facing step, flow past a cylinder;
Section 3).  It holds none of the method's arithmetic (no element matrices,
no subdivision, no solvers), so that the oracle and the HIP path can both
consume it without sharing code.

Random numbers come from a SplitMix64 stream (Steele, Lea & Flood, 2014):
output k of stream ``seed`` is mix(seed + (k+1)*GAMMA); a uniform double is
(z >> 11) * 2**-53.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

VEL_DIRICHLET = 1
OUTFLOW = 2

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start..start+count-1 of the SplitMix64 stream seeded with ``seed``."""
    k = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, start: int, count: int) -> np.ndarray:
    return (splitmix64(seed, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclass
class CoarseMesh:
    """A coarse P1 mesh: nodes, CCW triangles and tagged boundary edges."""

    xy: np.ndarray  # float64 [N, 2]
    tri: np.ndarray  # int32 [T, 3], counter-clockwise
    bedge: np.ndarray  # int32 [NB, 2]
    bkind: np.ndarray  # int32 [NB]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_tris(self) -> int:
        return int(self.tri.shape[0])


def _signed_area2(xy, tri):
    p0, p1, p2 = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    return (p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1]) - (p2[:, 0] - p0[:, 0]) * (p1[:, 1] - p0[:, 1])


def _orient_ccw(xy, tri):
    a2 = _signed_area2(xy, tri)
    flip = a2 < 0
    tri = tri.copy()
    tri[flip, 1], tri[flip, 2] = tri[flip, 2].copy(), tri[flip, 1].copy()
    return tri


def _boundary_edges(tri):
    """Edges used by exactly one triangle, oriented as in that triangle."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    key = np.sort(e, axis=1)
    kk = key[:, 0].astype(np.int64) * (1 << 32) + key[:, 1]
    uniq, inv, cnt = np.unique(kk, return_inverse=True, return_counts=True)
    once = cnt[inv] == 1
    return e[once].astype(np.int32)


def _jitter(xy, tri, interior, seed, frac=0.2):
    """Move interior nodes by U(-frac*h, frac*h) per coordinate, h = shortest incident edge."""
    n = xy.shape[0]
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    ln = np.hypot(*(xy[e[:, 0]] - xy[e[:, 1]]).T)
    h = np.full(n, np.inf)
    np.minimum.at(h, e[:, 0], ln)
    np.minimum.at(h, e[:, 1], ln)
    u = uniform01(seed, 0, 2 * n).reshape(n, 2)
    d = (2.0 * u - 1.0) * frac * h[:, None]
    d[~interior] = 0.0
    scale = np.ones(n)
    a_ref = np.abs(_signed_area2(xy, tri))
    for _ in range(30):
        out = xy + d * scale[:, None]
        a2 = _signed_area2(out, tri)
        bad = a2 < 0.1 * a_ref
        if not bad.any():
            return out
        scale[np.unique(tri[bad])] *= 0.5
    raise RuntimeError("jitter could not keep every triangle valid")


def _split_quads(q, bits):
    """Split quads (a,b,c,d in CCW order) into two triangles along a-c (bit 0) or b-d (bit 1)."""
    a, b, c, d = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    t0 = np.where(bits[:, None] == 0, np.stack([a, b, c], 1), np.stack([a, b, d], 1))
    t1 = np.where(bits[:, None] == 0, np.stack([a, c, d], 1), np.stack([b, c, d], 1))
    return np.concatenate([t0, t1]).astype(np.int32)


def _finish(xy, tri, seed, outflow_x=None, name="", meta=None):
    tri = _orient_ccw(xy, tri.astype(np.int32))
    be = _boundary_edges(tri)
    bnode = np.zeros(xy.shape[0], bool)
    bnode[be.ravel()] = True
    xy = _jitter(xy, tri, ~bnode, seed)
    kind = np.full(be.shape[0], VEL_DIRICHLET, np.int32)
    if outflow_x is not None:
        on = (xy[be[:, 0], 0] == outflow_x) & (xy[be[:, 1], 0] == outflow_x)
        kind[on] = OUTFLOW
    return CoarseMesh(np.ascontiguousarray(xy, dtype=np.float64), np.ascontiguousarray(tri, dtype=np.int32),
                      np.ascontiguousarray(be, dtype=np.int32), kind, name=name, meta=meta or {})


def _grid_nodes(xs, ys):
    X, Y = np.meshgrid(xs, ys)  # [ny+1, nx+1]
    return np.stack([X.ravel(), Y.ravel()], 1)


def unit_square_tg(n: int = 32, seed: int = 1) -> CoarseMesh:
    """Unit square, n x n cells each split by the (i,j)-(i+1,j+1) diagonal, interior jitter 0.2h.

    Every boundary edge is velocity-Dirichlet (Taylor-Green data, Section 3.1).
    """
    xs = np.linspace(0.0, 1.0, n + 1)
    xy = _grid_nodes(xs, xs)
    i, j = np.meshgrid(np.arange(n), np.arange(n))
    i, j = i.ravel(), j.ravel()
    v00 = j * (n + 1) + i
    q = np.stack([v00, v00 + 1, v00 + n + 2, v00 + n + 1], 1)
    tri = _split_quads(q, np.zeros(len(q), np.int64))
    return _finish(xy, tri, seed, None, name=f"tg_square_{n}")


def bfs_channel(nx: int = 612, ny: int = 42, length: float = 30.0, height: float = 2.0, seed: int = 2) -> CoarseMesh:
    """Backward-facing step channel [0,L]x[0,H]: inlet at x=0, y in [H/2,H]; step face below it.

    Random diagonal per cell, interior jitter 0.2h, outflow (zero traction) at x=L.
    """
    assert ny % 2 == 0
    xs = np.linspace(0.0, length, nx + 1)
    ys = np.linspace(0.0, height, ny + 1)
    xy = _grid_nodes(xs, ys)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny))
    i, j = i.ravel(), j.ravel()
    v00 = j * (nx + 1) + i
    q = np.stack([v00, v00 + 1, v00 + nx + 2, v00 + nx + 1], 1)
    bits = (splitmix64(seed ^ 0x5DEECE66D, 0, len(q)) >> np.uint64(63)).astype(np.int64)
    tri = _split_quads(q, bits)
    m = _finish(xy, tri, seed, outflow_x=xs[-1], name=f"bfs_{nx}x{ny}")
    m.meta.update(length=length, height=height)
    return m


def _cyl_lines(ns):
    hs = 0.2 / ns
    m1 = max(2, int(round(0.1 / hs)))
    m3 = max(4, int(round(1.9 * math.log(2.0) / hs)))
    mb = max(2, int(round(0.1 / hs)))
    mt = max(2, int(round(0.11 / hs)))
    xs = np.concatenate([np.linspace(0.0, 0.1, m1 + 1)[:-1], np.linspace(0.1, 0.3, ns + 1)[:-1],
                         0.3 + 1.9 * (2.0 ** (np.arange(m3 + 1) / m3) - 1.0)])
    xs[-1] = 2.2
    ys = np.concatenate([np.linspace(0.0, 0.1, mb + 1)[:-1], np.linspace(0.1, 0.3, ns + 1)[:-1],
                         np.linspace(0.3, 0.41, mt + 1)])
    nr = max(4, int(round(0.05 / hs * 0.55)))
    return xs, ys, m1, mb, nr


def _cyl_count(ns):
    xs, ys, m1, mb, nr = _cyl_lines(ns)
    nx, ny = len(xs) - 1, len(ys) - 1
    return 2 * (nx * ny - ns * ns) + 2 * (4 * ns) * nr


def cylinder_channel(target_tris: int = 250_000, seed: int = 3) -> CoarseMesh:
    """Channel [0,2.2]x[0,0.41] with a cylinder of radius 0.05 at (0.2,0.2).

    Multi-block mesh: a tensor grid (graded downstream) outside the square
    [0.1,0.3]^2 and an O-grid ring between that square and the circle, random
    diagonals, interior jitter 0.2h.  Inlet, walls and cylinder are
    velocity-Dirichlet; x=2.2 is the zero-traction outflow.
    """
    ns = max(4, int(round(math.sqrt(target_tris / 33.3))))
    best = min(range(max(4, ns - 6), ns + 7), key=lambda s: abs(_cyl_count(s) - target_tris))
    ns = best
    xs, ys, m1, mb, nr = _cyl_lines(ns)
    nx, ny = len(xs) - 1, len(ys) - 1
    ia, ib, ja, jb = m1, m1 + ns, mb, mb + ns  # square occupies grid lines ia..ib, ja..jb
    I, J = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
    I, J = I.ravel(), J.ravel()
    inside = (I > ia) & (I < ib) & (J > ja) & (J < jb)
    gid = -np.ones((ny + 1) * (nx + 1), np.int64)
    gid[~inside] = np.arange((~inside).sum())
    xy_grid = np.stack([xs[I[~inside]], ys[J[~inside]]], 1)

    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny))
    ci, cj = ci.ravel(), cj.ravel()
    keep = ~((ci >= ia) & (ci < ib) & (cj >= ja) & (cj < jb))
    ci, cj = ci[keep], cj[keep]
    g = lambda i, j: gid[j * (nx + 1) + i]
    q = np.stack([g(ci, cj), g(ci + 1, cj), g(ci + 1, cj + 1), g(ci, cj + 1)], 1)

    # square perimeter, counter-clockwise from corner (ia, ja)
    per = [(i, ja) for i in range(ia, ib)] + [(ib, j) for j in range(ja, jb)] + \
          [(i, jb) for i in range(ib, ia, -1)] + [(ia, j) for j in range(jb, ja, -1)]
    nth = len(per)
    per_id = np.array([g(i, j) for i, j in per], np.int64)
    per_xy = xy_grid[per_id]
    theta = -0.75 * math.pi + 2.0 * math.pi * np.arange(nth) / nth
    circ = np.stack([0.2 + 0.05 * np.cos(theta), 0.2 + 0.05 * np.sin(theta)], 1)
    gr = 1.04
    t = (gr ** np.arange(nr + 1) - 1.0) / (gr ** nr - 1.0)
    ring_ids = [None] * (nr + 1)
    ring_ids[nr] = per_id
    extra = []
    base = xy_grid.shape[0]
    for k in range(nr):
        pts = (1.0 - t[k]) * circ + t[k] * per_xy
        ring_ids[k] = base + np.arange(nth)
        base += nth
        extra.append(pts)
    xy = np.concatenate([xy_grid] + extra)
    oq = []
    for k in range(nr):
        a = ring_ids[k]
        b = np.roll(ring_ids[k], -1)
        c = np.roll(ring_ids[k + 1], -1)
        d = ring_ids[k + 1]
        oq.append(np.stack([a, d, c, b], 1))
    q = np.concatenate([q] + oq)
    bits = (splitmix64(seed ^ 0x5DEECE66D, 0, len(q)) >> np.uint64(63)).astype(np.int64)
    tri = _split_quads(q, bits)
    m = _finish(xy, tri, seed, outflow_x=2.2, name=f"cylinder_{len(tri)}")
    m.meta.update(ns=ns, nr=nr)
    return m


# ---------------------------------------------------------------- data on nodes

def tg_velocity(xy, t, mu=0.01, rho=1.0):
    """Taylor-Green velocity, Eqs. (34)-(35) (nu = mu/rho)."""
    nu = mu / rho
    x, y = xy[:, 0], xy[:, 1]
    e = math.exp(-8.0 * math.pi ** 2 * nu * t)
    u = -np.cos(2 * math.pi * x) * np.sin(2 * math.pi * y) * e
    v = np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y) * e
    return np.ascontiguousarray(np.stack([u, v], 1))


def tg_pressure(xy, t, mu=0.01, rho=1.0):
    """Taylor-Green pressure, Eq. (36)."""
    nu = mu / rho
    x, y = xy[:, 0], xy[:, 1]
    return -(np.cos(4 * math.pi * x) + np.cos(4 * math.pi * y)) / 4.0 * math.exp(-16.0 * math.pi ** 2 * nu * t)


def bfs_inflow(xy, height=2.0):
    """Parabolic inlet on x=0, y in [H/2, H] with unit mean (the analogue of Eq. 37)."""
    y = xy[:, 1]
    lo = 0.5 * height
    hh = height - lo
    u = np.where((xy[:, 0] == 0.0) & (y >= lo), 6.0 * (y - lo) * (height - y) / (hh * hh), 0.0)
    return np.ascontiguousarray(np.stack([u, np.zeros_like(u)], 1))


def cylinder_inflow(xy, um=1.5, height=0.41):
    """Parabolic inlet u = 4 Um y (H-y)/H^2 on x=0 (mean velocity 2Um/3)."""
    y = xy[:, 1]
    u = np.where(xy[:, 0] == 0.0, 4.0 * um * y * (height - y) / (height * height), 0.0)
    return np.ascontiguousarray(np.stack([u, np.zeros_like(u)], 1))


# ---------------------------------------------------------------- configurations

@dataclass
class Case:
    """One workload: coarse mesh, levels, physics and solver tolerances."""

    name: str
    mesh: CoarseMesh
    levels: int
    rho: float
    mu: float
    dt: float
    steps: int
    tol_p: float
    tol_mom: float
    tol_mass: float
    kind: str  # "tg" | "bfs" | "cyl"

    def dirichlet(self, xy_f: np.ndarray, t: float) -> np.ndarray:
        """Velocity data g(t) at every fine node (only Dirichlet nodes are read)."""
        if self.kind == "tg":
            return tg_velocity(xy_f, t, self.mu, self.rho)
        if self.kind == "bfs":
            return bfs_inflow(xy_f, self.mesh.meta.get("height", 2.0))
        return cylinder_inflow(xy_f)

    def initial(self, xy_f: np.ndarray, dirichlet_mask: np.ndarray) -> np.ndarray:
        """U^0: Taylor-Green exact state, else impulsive start (g on Gamma_D, 0 elsewhere)."""
        if self.kind == "tg":
            return tg_velocity(xy_f, 0.0, self.mu, self.rho)
        u = self.dirichlet(xy_f, 0.0)
        u[~dirichlet_mask.astype(bool)] = 0.0
        return np.ascontiguousarray(u)


def case_tg(n=32, seed=1, levels=1, dt=1e-3, steps=100) -> Case:
    return Case("taylor_green", unit_square_tg(n, seed), levels, 1.0, 0.01, dt, steps, 1e-12, 1e-12, 1e-12, "tg")


def case_bfs(nx=612, ny=42, seed=2, levels=1) -> Case:
    # H = 2, mean inlet speed 1, Re = rho*H*ubar/mu = 400 -> mu = 0.005
    return Case("backward_step", bfs_channel(nx, ny, seed=seed), levels, 1.0, 0.005, 5e-3, 500, 1e-8, 1e-8, 1e-10, "bfs")


def case_cylinder(target_tris=250_000, seed=3, levels=1, mu=1e-3) -> Case:
    # D = 0.1, mean inlet speed 1, Re = 100 -> mu = 1e-3
    return Case("cylinder", cylinder_channel(target_tris, seed), levels, 1.0, mu, 1e-3, 2000, 1e-8, 1e-8, 1e-10, "cyl")


def batch_sweep(n: int = 64, lo: int = 16_000, hi: int = 250_000, seed: int = 4, levels: int = 1) -> list:
    """Independent cylinder-flow instances for a batched run: coarse sizes log-uniform in [lo, hi]
    triangles, Re uniform in [60, 160] (mu = 0.1 / Re with rho = 1, mean inlet speed 1, D = 0.1), mesh
    seeds 1000 + i."""
    return [batch_instance(i, n, lo, hi, seed, levels) for i in range(n)]


def batch_sweep_sizes(n: int = 64, lo: int = 16_000, hi: int = 250_000, seed: int = 4) -> list:
    """Target coarse triangle counts and Reynolds numbers of batch_sweep's instances, without building
    the meshes."""
    u = uniform01(seed, 0, 2 * n).reshape(n, 2)
    return [(int(round(math.exp(math.log(lo) + u[i, 0] * (math.log(hi) - math.log(lo))))), 60.0 + 100.0 * u[i, 1])
            for i in range(n)]


def batch_instance(i: int, n: int = 64, lo: int = 16_000, hi: int = 250_000, seed: int = 4, levels: int = 1) -> Case:
    """Instance i of batch_sweep(n, lo, hi, seed, levels) alone."""
    tris, re = batch_sweep_sizes(n, lo, hi, seed)[i]
    return case_cylinder(tris, seed=1000 + i, levels=levels, mu=0.1 / re)


def batch_deciles(n: int = 64, lo: int = 16_000, hi: int = 250_000, seed: int = 4) -> list:
    """Indices of one batch_sweep instance per size decile: the instance at the middle of each tenth of
    the instances sorted by size."""
    sizes = batch_sweep_sizes(n, lo, hi, seed)
    order = sorted(range(n), key=lambda i: sizes[i][0])
    return [order[min(n - 1, int((d + 0.5) * n / 10))] for d in range(10)]
