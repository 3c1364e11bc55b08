"""More pins of the FP64 oracle against facts that do not come from the oracle
itself:

* the lumped-mass velocity correction (Eq. 23 with a row-sum mass) on a linear
  pressure, where D_x x equals the lumped mass at interior nodes, so the
  correction is the exact gradient times dt/rho;
* the oracle's own mesh validation rejecting each kind of invalid mesh;
* the POD of pressure snapshots (method of snapshots, own Jacobi eigensolver):
  a closed-form 2x2 eigenproblem, orthonormality, exact reconstruction at
  rank <= m, the Eckart-Young residual identity and a library eigensolver;
* the paper's error norms (Eqs. 31-33): zero for linear fields, the 1/M
  factor on a constant error, and an independent quadrature of the
  interpolation error of a quadratic;
* energy stability of the projection part of the step (Eqs. 20-23), built
  column by column from the oracle's own restriction, Poisson solve,
  prolongation and correction: an orthogonal projection (norm 1 in the
  consistent-mass energy) for the transpose-of-prolongation restriction and
  for l = 0, an oblique one (norm about 3) for injection at l = 1.
"""
import numpy as np
import pytest

import workloads as W


# ---------------------------------------------------------------- lumped correction

@pytest.mark.parametrize("which", ["bfs", "cyl"])
def test_lumped_correction_of_a_linear_pressure(orc, which):
    case = W.case_bfs(40, 6, levels=1) if which == "bfs" else W.case_cylinder(2000, seed=5, levels=1)
    rho, dt = 1.3, 0.01
    P = orc.Problem(case.mesh, 1)
    P.assemble(rho, case.mu, dt, 0, 1)
    xy = P.export("xy")
    xc = P.export("xy", 0)
    a, b, c = 0.4, -1.7, 2.9
    pf = P.prolong(a + b * xc[:, 0] + c * xc[:, 1])
    np.testing.assert_allclose(pf, a + b * xy[:, 0] + c * xy[:, 1], rtol=0, atol=1e-13)
    rng = np.random.default_rng(1)
    ut = rng.normal(size=(xy.shape[0], 2))
    g = rng.normal(size=(xy.shape[0], 2))
    u, code, st = P.correct(g, ut, pf)
    assert code == 0 and st["mass_iters"] == [0, 0]
    # interior nodes: not on any boundary edge of the fine mesh
    onb = np.zeros(xy.shape[0], bool)
    onb[P.export("bedge").ravel()] = True
    vd = P.export("vdir").astype(bool)
    inner = ~onb
    assert inner.sum() > 100
    want = np.array([-(dt / rho) * b, -(dt / rho) * c])
    np.testing.assert_allclose(u[inner] - ut[inner], np.broadcast_to(want, (inner.sum(), 2)), rtol=1e-12, atol=1e-14)
    # velocity data re-imposed on the Dirichlet nodes
    assert np.array_equal(u[vd], g[vd])


# ---------------------------------------------------------------- mesh validation

def test_oracle_rejects_invalid_meshes(orc):
    base = W.unit_square_tg(4)

    def clone(**kw):
        m = W.CoarseMesh(base.xy.copy(), base.tri.copy(), base.bedge.copy(), base.bkind.copy())
        for k, v in kw.items():
            setattr(m, k, v)
        return m

    assert orc.check_mesh(base) == 0
    cw = clone()
    cw.tri[0, [1, 2]] = cw.tri[0, [2, 1]]
    untagged = clone(bedge=base.bedge[1:].copy(), bkind=base.bkind[1:].copy())
    nonman = clone(tri=np.concatenate([base.tri, base.tri[:1]]))
    badkind = clone()
    badkind.bkind[0] = 7
    oob = clone()
    oob.tri[3, 0] = 10_000
    flat = clone()
    flat.xy[flat.tri[5, 2]] = 0.5 * (flat.xy[flat.tri[5, 0]] + flat.xy[flat.tri[5, 1]])
    for bad in (cw, untagged, nonman, badkind, oob, flat):
        assert orc.check_mesh(bad) == 2
        with pytest.raises(ValueError, match="invalid mesh"):
            orc.Problem(bad, 1)
    with pytest.raises(ValueError, match="bad argument"):
        orc.Problem(base, 9)


# ---------------------------------------------------------------- POD

def test_jacobi_eigen_closed_form_2x2(orc):
    for a, b, d in ((2.0, 1.0, -3.0), (1.0, 1e-9, 1.0), (5.0, -4.0, 5.0)):
        lam, V = orc.jacobi_eigen([[a, b], [b, d]])
        mid, rad = 0.5 * (a + d), np.hypot(0.5 * (a - d), b)
        np.testing.assert_allclose(np.sort(lam), [mid - rad, mid + rad], rtol=1e-14, atol=1e-15)
        np.testing.assert_allclose(V.T @ V, np.eye(2), atol=1e-15)


def test_jacobi_eigen_invariants_and_library(orc):
    rng = np.random.default_rng(3)
    X = rng.normal(size=(40, 40))
    A = X + X.T
    lam, V = orc.jacobi_eigen(A)
    np.testing.assert_allclose(V.T @ V, np.eye(40), atol=1e-13)
    np.testing.assert_allclose(A @ V, V * lam, atol=1e-12 * np.abs(lam).max())
    np.testing.assert_allclose(np.sort(lam), np.linalg.eigvalsh(A), rtol=0, atol=1e-12 * np.abs(lam).max())


def _snaps(rng, S, n, r):
    # amplitudes decay to ~0.02: the method of snapshots squares the condition of the snapshot matrix,
    # so a mode of relative energy e is orthonormal only to about 1e-16 / e
    return (rng.normal(size=(S, r)) * 0.85 ** np.arange(r)) @ rng.normal(size=(r, n))


@pytest.mark.parametrize("S,r,m", [(30, 8, 12), (24, 24, 24), (50, 60, 16)])
def test_pod_properties(orc, S, r, m):
    rng = np.random.default_rng(S + r + m)
    n = 300
    w = rng.uniform(0.5, 2.0, n)
    snaps = _snaps(rng, S, n, r)
    phi, energy, rank = orc.pod(snaps, w, m)
    rk = min(S, r, m)
    # eigenvalues at the rounding level of a rank-deficient Gram matrix (~1e-16 of the largest) lie
    # above the 1e-20 cut-off and are kept, as in the library; the resolved modes are checked
    assert rank >= rk
    # orthonormal in the w-weighted inner product, to the rounding the Gram matrix leaves in each pair of
    # modes (its error ~1e-16 lambda_0 divided by sqrt(lambda_i lambda_j))
    G = phi.T @ (w[:, None] * phi)
    lam = energy[:rk]
    bound = 1e-14 * lam[0] / np.sqrt(np.outer(lam, lam))
    assert np.all(np.abs(G[:rk, :rk] - np.eye(rk)) <= bound)
    # energies: non-increasing, and the total captures the snapshots' weighted norm when m >= rank
    assert np.all(np.diff(energy[:rk]) <= 1e-12 * energy[0])
    total = np.sum(w * snaps * snaps)
    if rk == min(S, r):
        np.testing.assert_allclose(energy.sum(), total, rtol=1e-12)
        rec = (phi @ (phi.T @ (w[:, None] * snaps.T))).T
        np.testing.assert_allclose(rec, snaps, atol=1e-10 * np.abs(snaps).max())
    # Eckart-Young: the energy left outside the first k modes is the sum of the remaining eigenvalues
    lam_all = np.sort(np.linalg.eigvalsh(snaps @ (w[:, None] * snaps.T)))[::-1]
    for k in (1, rk // 2, rk):
        Pk = phi[:, :k]
        resid = snaps.T - Pk @ (Pk.T @ (w[:, None] * snaps.T))
        left = np.sum(w[:, None] * resid * resid)
        np.testing.assert_allclose(left, lam_all[k:].sum(), rtol=1e-8, atol=1e-12 * total)
    # same eigenvalues as a library eigensolver of the same Gram matrix
    np.testing.assert_allclose(energy[:rk], lam_all[:rk], rtol=0, atol=1e-13 * lam_all[0])


def test_pod_drops_modes_without_energy(orc):
    rng = np.random.default_rng(9)
    snaps = np.zeros((20, 100))
    snaps[:3] = rng.normal(size=(3, 100))   # zero snapshots add exact zero eigenvalues
    phi, energy, rank = orc.pod(snaps, np.ones(100), 6)
    assert rank == 3 and not phi[:, 3:].any() and not energy[3:].any()
    np.testing.assert_allclose(phi[:, :3].T @ phi[:, :3], np.eye(3), atol=1e-13)


# ---------------------------------------------------------------- error norms, Eqs. (31)-(33)

def _collapsed_gauss(xy3, f, k=8):
    """Integral of f over a triangle by a Duffy-collapsed k x k Gauss-Legendre rule (exact to degree 2k-2)."""
    t, wt = np.polynomial.legendre.leggauss(k)
    t, wt = 0.5 * (t + 1), 0.5 * wt
    p0, p1, p2 = xy3
    area2 = abs((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]))
    acc = 0.0
    for s, ws in zip(t, wt):
        for r, wr in zip(t, wt):
            l1, l2 = s, r * (1 - s)
            x = p0 + l1 * (p1 - p0) + l2 * (p2 - p0)
            acc += ws * wr * (1 - s) * f(x, (1 - l1 - l2, l1, l2))
    return acc * area2


def test_error_norms(orc):
    case = W.case_tg(6, levels=1)
    P = orc.Problem(case.mesh, 1)
    xy = P.export("xy")
    tri = P.export("tri")
    M = tri.shape[0]
    lin = lambda q: 0.3 - 1.1 * q[:, 0] + 2.0 * q[:, 1]
    l2, linf = P.error_norms(lin(xy), lin)
    assert l2 < 1e-15 and linf < 1e-15
    # a constant error c: ||e||_L2 = c sqrt(|V| / M) (the 1/M of Eq. 32; |V| = 1), ||e||_inf = c
    l2, linf = P.error_norms(lin(xy) + 0.25, lin)
    np.testing.assert_allclose([l2, linf], [0.25 / np.sqrt(M), 0.25], rtol=1e-13)
    # vector field: Euclidean length of the error vector
    vec = lambda q: np.stack([lin(q), 2 * lin(q)], 1)
    l2, linf = P.error_norms(vec(xy) + np.array([0.3, 0.4]), vec)
    np.testing.assert_allclose([l2, linf], [0.5 / np.sqrt(M), 0.5], rtol=1e-13)
    # interpolation error of x^2 + x y (degree 4 integrand, integrated exactly by the degree-4 rule)
    quad = lambda q: q[:, 0] ** 2 + q[:, 0] * q[:, 1]
    A = quad(xy)
    l2, linf = P.error_norms(A, quad)
    ref = 0.0
    for t in tri:
        p3 = xy[t]
        e2 = lambda x, lam: (sum(lam[j] * A[t[j]] for j in range(3)) - (x[0] ** 2 + x[0] * x[1])) ** 2
        ref += _collapsed_gauss(p3, e2)
    np.testing.assert_allclose(l2, np.sqrt(ref / M), rtol=1e-12)
    assert 0 < linf < 0.1


# ---------------------------------------------------------------- energy stability of the projection

def _projection_map(orc, case, levels, rmode, mmode):
    """Columns: the velocity after restriction, Poisson solve, prolongation and correction (Eqs. 20-23)
    of each unit perturbation of a free velocity value, zero velocity data."""
    P = orc.Problem(case.mesh, levels)
    P.assemble(case.rho, case.mu, case.dt, rmode, mmode)
    nf = P.info["n_f"]
    free = np.where(P.export("vdir") == 0)[0]
    g = np.zeros((nf, 2))
    cols = []
    for comp in (0, 1):
        for i in free:
            ut = np.zeros((nf, 2))
            ut[i, comp] = 1.0
            b = P.restrict(ut, rmode)
            pc, code, _, _ = P.poisson_solve(b, tol=1e-14)
            assert code == 0
            u, code, _ = P.correct(g, ut, P.prolong(pc), tol=1e-14)
            assert code == 0
            cols.append(np.concatenate([u[free, 0], u[free, 1]]))
    T = np.array(cols).T
    import scipy.sparse as sp
    Mf = sp.csr_matrix((P.values("M_f"), P.export("col_f"), P.export("rowptr_f")), shape=(nf, nf)).toarray()
    Mff = Mf[np.ix_(free, free)]
    Z = np.zeros_like(Mff)
    Wm = np.block([[Mff, Z], [Z, Mff]])
    L = np.linalg.cholesky(Wm)
    return np.linalg.norm(L.T @ T @ np.linalg.inv(L.T), 2)


@pytest.mark.parametrize("which", ["tg", "bfs"])
def test_projection_energy_norm(orc, which):
    case = W.case_tg(6, levels=1) if which == "tg" else W.case_bfs(24, 4, levels=1)
    gal = _projection_map(orc, case, 1, 1, 0)
    inj = _projection_map(orc, case, 1, 0, 0)
    std = _projection_map(orc, W.Case(case.name, case.mesh, 0, case.rho, case.mu, case.dt, 1, 0, 0, 0, case.kind),
                          0, 0, 0)
    # an M-orthogonal projection: the transpose of prolongation pairs the divergence with the
    # prolonged gradient, as the standard method (l = 0) pairs D with G
    assert abs(gal - 1.0) < 1e-9, gal
    assert abs(std - 1.0) < 1e-9, std
    # injection leaves the midpoint velocities out of the divergence: an oblique projection that can
    # multiply a perturbation's kinetic energy several times in one step
    assert inj > 2.0, inj


def _max_speed_history(orc, case, rmode, mmode, steps, stop_above):
    P = orc.Problem(case.mesh, case.levels)
    P.assemble(case.rho, case.mu, case.dt, rmode, mmode)
    xy, vd = P.export("xy"), P.export("vdir")
    u, g = case.initial(xy, vd), case.dirichlet(xy, case.dt)
    pc = np.zeros(P.info["n_c"])
    hist = []
    for k in range(steps):
        u, pf, pc, code, _ = P.step(g, u, pc, tol_mom=1e-10, tol_p=1e-10, tol_mass=1e-10, maxit=3000)
        hist.append(float(np.max(np.hypot(u[:, 0], u[:, 1]))))
        if code or hist[-1] > stop_above:
            break
    return hist


def test_injection_trajectory_grows_galerkin_stays_bounded(orc):
    """The consequence of the oblique projection on a cylinder flow from an impulsive start (l = 1,
    dt = 1e-3, 1500 coarse triangles): with injection a fine-scale velocity grows past 20 (10x the
    inflow peak) within 200 steps, with the consistent and with the lumped mass; with the transpose of
    prolongation the same flow stays below 3.5 for 300 steps (2.5 after the first 100)."""
    case = W.case_cylinder(1500, levels=1)
    for mmode in (0, 1):
        h = _max_speed_history(orc, case, 0, mmode, 600 if mmode else 200, 20.0)
        assert max(h) > 20.0, (mmode, len(h), max(h))
    h = _max_speed_history(orc, case, 1, 0, 300, 20.0)
    assert len(h) == 300 and max(h) < 3.5 and max(h[100:]) < 2.5, (max(h), max(h[100:]))
