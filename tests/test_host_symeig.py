"""The host eigen-decomposition behind the POD basis (csrc/symeig.h: Householder tridiagonalisation and
implicit shifted QR, Golub & Van Loan Algorithms 8.3.1-8.3.3), compiled with the system C++ compiler
into a small driver and checked against LAPACK's symmetric solver through numpy: eigenvalues, the
residual A Z - Z diag(lambda), and orthonormal vectors, on random symmetric, SPD, and nearly rank-
deficient snapshot Gram matrices like the ones the online basis decomposes."""
import shutil
import subprocess
from pathlib import Path

import numpy as np
import pytest

HEADER_DIR = Path(__file__).resolve().parents[1] / "paper_1610_06993_amd" / "csrc"
DRIVER = r"""
#include <cstdio>
#include <vector>
#include "symeig.h"
int main() {
  int n;
  if (scanf("%d", &n) != 1) return 1;
  std::vector<double> A((size_t)n * n), Z;
  for (auto &x : A) if (scanf("%lf", &x) != 1) return 1;
  const bool ok = cgp::sym_eigen(n, A, Z);
  printf("%d\n", ok ? 1 : 0);
  for (int i = 0; i < n; i++) printf("%.17g\n", A[(size_t)i * n + i]);
  for (double x : Z) printf("%.17g\n", x);
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    d = tmp_path_factory.mktemp("symeig")
    (d / "drv.cpp").write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([cxx, "-O2", "-std=c++17", f"-I{HEADER_DIR}", str(d / "drv.cpp"), "-o", str(exe)], check=True)
    return exe


def decompose(exe, A):
    n = A.shape[0]
    text = f"{n}\n" + "\n".join(" ".join(repr(float(x)) for x in row) for row in A)
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout.split()
    ok = out[0] == "1"
    vals = np.array([float(x) for x in out[1:]])
    return ok, vals[:n], vals[n:].reshape(n, n)


def snapshot_gram(rng, S=64, n=3000):
    """Gram matrix of S slowly drifting snapshots: a few smooth modes over a common base, plus noise at
    1e-9, so the spectrum spans some twenty orders of magnitude."""
    x = np.arange(n) / n
    base = rng.normal(size=n)
    snaps = []
    for s in range(S):
        v = base.copy()
        for d in range(6):
            v += 0.1 ** (d + 1) * np.sin(0.05 * s * (d + 1)) * np.cos(2 * np.pi * (d + 1) * x)
        snaps.append(v + 1e-9 * rng.normal(size=n))
    S_ = np.array(snaps)
    return S_ @ S_.T


CASES = ["sym64", "spd64", "gram64", "sym1", "sym2", "diag5", "spd100", "repeated"]


@pytest.mark.parametrize("case", CASES)
def test_sym_eigen_against_lapack(driver, case):
    rng = np.random.default_rng(CASES.index(case))
    if case == "sym64":
        X = rng.normal(size=(64, 64)); A = X + X.T
    elif case == "spd64":
        X = rng.normal(size=(64, 64)); A = X @ X.T
    elif case == "gram64":
        A = snapshot_gram(rng)
    elif case == "sym1":
        A = np.array([[3.5]])
    elif case == "sym2":
        A = np.array([[2.0, 1.0], [1.0, -1.0]])
    elif case == "diag5":
        A = np.diag([5.0, -1.0, 3.0, 0.0, 2.0])
    elif case == "spd100":
        X = rng.normal(size=(100, 100)); A = X @ X.T
    else:  # a repeated eigenvalue: Q diag(1, 1, 1, 2, 3) Q^T
        Q, _ = np.linalg.qr(rng.normal(size=(5, 5)))
        A = Q @ np.diag([1.0, 1.0, 1.0, 2.0, 3.0]) @ Q.T
    A = 0.5 * (A + A.T)
    ok, lam, Z = decompose(driver, A)
    assert ok
    n = A.shape[0]
    scale = np.max(np.abs(np.linalg.eigvalsh(A)))
    assert np.max(np.abs(np.sort(lam) - np.linalg.eigvalsh(A))) <= 1e-13 * scale
    assert np.max(np.abs(A @ Z - Z * lam)) <= 1e-13 * scale
    assert np.max(np.abs(Z.T @ Z - np.eye(n))) <= 1e-13
    if case == "gram64":
        # the resolved (large) eigenvalues to high relative accuracy as well
        ref = np.sort(np.linalg.eigvalsh(A))[::-1]
        got = np.sort(lam)[::-1]
        big = ref > 1e-8 * ref[0]
        assert np.max(np.abs(got[big] - ref[big]) / ref[big]) < 1e-6


INV_DRIVER = r"""
#include <cstdio>
#include <vector>
#include "symeig.h"
int main() {
  int nm, rank;
  if (scanf("%d %d", &nm, &rank) != 2) return 1;
  std::vector<double> K((size_t)nm * nm), inv((size_t)nm * nm, -1.0);
  for (auto &x : K) if (scanf("%lf", &x) != 1) return 1;
  const bool ok = cgp::independent_inverse(nm, rank, K.data(), inv);
  printf("%d\n", ok ? 1 : 0);
  for (double x : inv) printf("%.17g\n", x);
  return 0;
}
"""


@pytest.fixture(scope="module")
def inv_driver(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no C++ compiler")
    d = tmp_path_factory.mktemp("indinv")
    (d / "drv.cpp").write_text(INV_DRIVER)
    exe = d / "drv"
    subprocess.run([cxx, "-O2", "-std=c++17", f"-I{HEADER_DIR}", str(d / "drv.cpp"), "-o", str(exe)], check=True)
    return exe


def independent_inverse(exe, K, rank):
    nm = K.shape[0]
    text = f"{nm} {rank}\n" + "\n".join(" ".join(repr(float(x)) for x in row) for row in K)
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout.split()
    return out[0] == "1", np.array([float(x) for x in out[1:]]).reshape(nm, nm)


def _spd(rng, n):
    X = rng.normal(size=(n, n))
    return X @ X.T + n * np.eye(n)


def test_independent_inverse_of_a_definite_matrix(inv_driver):
    """Positive definite Phi^T K Phi: every mode is kept and the result is the inverse of the leading
    rank x rank block (numpy's), the rows and columns beyond the rank zero."""
    rng = np.random.default_rng(11)
    n, nm, rank = 200, 12, 10
    K = _spd(rng, n)
    Phi = rng.normal(size=(n, nm))
    G = Phi.T @ K @ Phi
    ok, inv = independent_inverse(inv_driver, G, rank)
    assert ok
    ref = np.linalg.inv(G[:rank, :rank])
    assert np.max(np.abs(inv[:rank, :rank] - ref)) <= 1e-10 * np.max(np.abs(ref))
    assert np.all(inv[rank:, :] == 0.0) and np.all(inv[:, rank:] == 0.0)


def test_independent_inverse_leaves_out_dependent_modes(inv_driver):
    """Modes 3 and 6 are combinations of the modes before them and mode 5 is zero: those three are left
    out (zero rows and columns), the others are inverted as a block; the Galerkin solution x = Phi c,
    c = inv Phi^T K s, recovers any s in the span of the modes, which is what the guess needs."""
    rng = np.random.default_rng(12)
    n, nm = 300, 8
    K = _spd(rng, n)
    P = rng.normal(size=(n, nm))
    P[:, 3] = 0.7 * P[:, 0] - 1.3 * P[:, 2]
    P[:, 5] = 0.0
    P[:, 6] = P[:, 1] + 0.25 * P[:, 4]
    G = P.T @ K @ P
    G = 0.5 * (G + G.T)
    ok, inv = independent_inverse(inv_driver, G, nm)
    assert ok
    kept = [0, 1, 2, 4, 7]
    out = [3, 5, 6]
    assert np.all(inv[out, :] == 0.0) and np.all(inv[:, out] == 0.0)
    ref = np.linalg.inv(G[np.ix_(kept, kept)])
    assert np.max(np.abs(inv[np.ix_(kept, kept)] - ref)) <= 1e-9 * np.max(np.abs(ref))
    s = P @ rng.normal(size=nm)
    x = P @ (inv @ (P.T @ (K @ s)))
    assert np.linalg.norm(x - s) <= 1e-9 * np.linalg.norm(s)


def test_independent_inverse_of_a_rank_one_matrix(inv_driver):
    """All modes along one direction (snapshots that repeat): only the first is kept; no mode at all (a
    zero matrix) is reported as a failure."""
    rng = np.random.default_rng(13)
    n, nm = 100, 6
    K = _spd(rng, n)
    v = rng.normal(size=n)
    P = np.outer(v, rng.uniform(0.5, 2.0, size=nm))
    G = P.T @ K @ P
    ok, inv = independent_inverse(inv_driver, G, nm)
    assert ok
    assert inv[0, 0] == pytest.approx(1.0 / G[0, 0], rel=1e-12)
    assert np.count_nonzero(inv) == 1
    ok0, _ = independent_inverse(inv_driver, np.zeros((nm, nm)), nm)
    assert not ok0
