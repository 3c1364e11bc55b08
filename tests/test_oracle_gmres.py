"""Pins of the oracle's ILU(0)-GMRES(m), the paper's solver (Section 2.3):

* ILU(0) reproduces the matrix on its pattern, (L U)_ij = a_ij, which is its definition, on the coarse
  Poisson matrix and on a nonsymmetric momentum matrix (dense products, not the oracle's arithmetic);
* a matrix whose pattern admits no fill (tridiagonal) is factored exactly: L U = A everywhere, and the
  preconditioned GMRES converges in one iteration;
* unpreconditioned full GMRES (m >= n) on a small system converges within n iterations;
* the converged solutions agree with a dense solve (SPD Poisson matrix, nonsymmetric momentum
  matrix), with and without restarts."""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W


def _dense(rp, col, val, n):
    return sp.csr_matrix((val, col, rp), shape=(n, n)).toarray()


def _split(rp, col, lu, n):
    F = _dense(rp, col, lu, n)
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    return L, U


def _systems(orc):
    case = W.case_bfs(16, 4, levels=1)
    P = orc.Problem(case.mesh, 1)
    P.assemble(1.0, 0.005, 5e-3)
    rpc, colc = P.export("rowptr_c"), P.export("col_c")
    K = P.values("K_c_bc")
    rpf, colf = P.export("rowptr_f"), P.export("col_f")
    xy = P.export("xy")
    u = np.stack([1.0 + xy[:, 1], 0.3 * xy[:, 0]], 1)
    A = P.values("M_f") + 5e-3 * 0.005 * P.values("K_f") + 5e-3 * P.convection(u)  # nonsymmetric
    return [("poisson", rpc, colc, K), ("momentum", rpf, colf, A)]


def test_ilu0_reproduces_the_matrix_on_its_pattern(orc):
    for name, rp, col, val in _systems(orc):
        n = len(rp) - 1
        lu = orc.ilu0(rp, col, val)
        L, U = _split(rp, col, lu, n)
        LU = L @ U
        Ad = _dense(rp, col, val, n)
        mask = _dense(rp, col, np.ones_like(val), n) > 0
        np.testing.assert_allclose(LU[mask], Ad[mask], rtol=0, atol=1e-12 * np.abs(Ad).max(), err_msg=name)
        # and it is incomplete: L U has entries outside the pattern
        assert np.abs(LU[~mask]).max() > 1e-8 * np.abs(Ad).max(), name


def test_tridiagonal_is_factored_exactly(orc):
    n = 40
    rng = np.random.default_rng(0)
    main = 4.0 + rng.uniform(size=n)
    lo, up = rng.uniform(-1, 1, n - 1), rng.uniform(-1, 1, n - 1)
    T = sp.diags([lo, main, up], [-1, 0, 1], format="csr")
    T.sort_indices()
    lu = orc.ilu0(T.indptr, T.indices, T.data)
    L, U = _split(T.indptr, T.indices, lu, n)
    np.testing.assert_allclose(L @ U, T.toarray(), atol=1e-14)
    b = rng.normal(size=n)
    x, st, it, rr = orc.gmres(T.indptr, T.indices, T.data, b, m=10, tol=1e-13)
    assert st == 0 and it == 1
    np.testing.assert_allclose(x, np.linalg.solve(T.toarray(), b), rtol=1e-12)


def test_full_gmres_converges_within_n(orc):
    rng = np.random.default_rng(1)
    n = 30
    A = sp.random(n, n, density=0.3, random_state=2, format="csr") + sp.eye(n) * 3.0
    A = A.tocsr()
    A.sort_indices()
    b = rng.normal(size=n)
    x, st, it, rr = orc.gmres(A.indptr, A.indices, A.data, b, m=n, tol=1e-12, ilu=False)
    assert st == 0 and it <= n
    np.testing.assert_allclose(x, np.linalg.solve(A.toarray(), b), rtol=1e-9)


@pytest.mark.parametrize("m,orth", [(5, "mgs"), (30, "mgs"), (5, "cgs2"), (30, "cgs2")])
def test_gmres_matches_dense_solve(orc, m, orth):
    rng = np.random.default_rng(3)
    for name, rp, col, val in _systems(orc):
        n = len(rp) - 1
        b = rng.normal(size=n)
        x, st, it, rr = orc.gmres(rp, col, val, b, m=m, tol=1e-13, orth=orth)
        assert st == 0 and rr <= 1e-13, (name, st, rr)
        ref = orc.dense_solve(_dense(rp, col, val, n), b)
        np.testing.assert_allclose(x, ref, rtol=0, atol=1e-10 * np.abs(ref).max(), err_msg=name)
        # ILU(0) helps: fewer iterations than without it
        _, st0, it0, _ = orc.gmres(rp, col, val, b, m=m, tol=1e-13, ilu=False, orth=orth)
        assert it < it0, (name, it, it0)
