// Dense symmetric eigen-decomposition on the host (the POD basis builds up to a few hundred modes), and
// the inverse of the POD-Galerkin matrix over its independent modes.
//
// Householder reduction to tridiagonal form T = Q^T A Q, then implicit symmetric QR steps with the
// Wilkinson shift on T, the Givens rotations accumulated into Q (Golub & Van Loan, Matrix
// Computations, 4th ed., Algorithms 8.3.1-8.3.3).  About 9 n^3 flops, against roughly 40 n^3 for
// the nine or so cyclic Jacobi sweeps a 64 x 64 snapshot Gram matrix needs.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

namespace cgp {

// A: n x n row-major symmetric (only its values are read; it is overwritten).  On return A[c*n + c]
// is eigenvalue c (unordered) and Z[j*n + c] component j of its unit eigenvector.  Returns false if
// the QR iteration did not converge within 30 n steps (then A and Z hold the partial result).
inline bool sym_eigen(int n, std::vector<double> &A, std::vector<double> &Z) {
  Z.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; i++) Z[(size_t)i * n + i] = 1.0;
  if (n == 0) return true;
  auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
  auto z = [&](int i, int j) -> double & { return Z[(size_t)i * n + j]; };
  std::vector<double> v(n), p(n), w(n);
  // 1. Householder: column j below the subdiagonal is zeroed by H = I - beta v v^T on rows j+1..n-1
  for (int j = 0; j + 2 < n; j++) {
    const int L = n - j - 1;  // length of the reflected part
    double xn = 0.0;
    for (int k = 0; k < L; k++) xn += a(j + 1 + k, j) * a(j + 1 + k, j);
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const double x0 = a(j + 1, j);
    const double alpha = x0 >= 0.0 ? -xn : xn;
    for (int k = 0; k < L; k++) v[k] = a(j + 1 + k, j);
    v[0] -= alpha;
    double vn2 = 0.0;
    for (int k = 0; k < L; k++) vn2 += v[k] * v[k];
    if (vn2 == 0.0) continue;
    const double beta = 2.0 / vn2;
    // the trailing block B (rows/columns j+1..n-1): B <- H B H = B - v w^T - w v^T with p = beta B v,
    // K = beta/2 v^T p, w = p - K v
    for (int r = 0; r < L; r++) {
      double s = 0.0;
      for (int k = 0; k < L; k++) s += a(j + 1 + r, j + 1 + k) * v[k];
      p[r] = beta * s;
    }
    double K = 0.0;
    for (int k = 0; k < L; k++) K += v[k] * p[k];
    K *= 0.5 * beta;
    for (int k = 0; k < L; k++) w[k] = p[k] - K * v[k];
    for (int r = 0; r < L; r++)
      for (int k = 0; k < L; k++) a(j + 1 + r, j + 1 + k) -= v[r] * w[k] + w[r] * v[k];
    a(j + 1, j) = a(j, j + 1) = alpha;
    for (int k = 1; k < L; k++) a(j + 1 + k, j) = a(j, j + 1 + k) = 0.0;
    // Q <- Q H on columns j+1..n-1
    for (int r = 0; r < n; r++) {
      double s = 0.0;
      for (int k = 0; k < L; k++) s += z(r, j + 1 + k) * v[k];
      s *= beta;
      for (int k = 0; k < L; k++) z(r, j + 1 + k) -= s * v[k];
    }
  }
  std::vector<double> d(n), e(n, 0.0);  // e[i] = T(i+1, i)
  for (int i = 0; i < n; i++) d[i] = a(i, i);
  for (int i = 0; i + 1 < n; i++) e[i] = a(i + 1, i);
  // 2. implicit symmetric QR: deflate negligible subdiagonal entries, then one Wilkinson-shifted
  //    step on the lowest unreduced block [l, m], the bulge chased down by Givens rotations
  const double eps = 2.220446049250313e-16;
  int m = n - 1, steps = 0;
  while (m > 0) {
    if (std::fabs(e[m - 1]) <= eps * (std::fabs(d[m - 1]) + std::fabs(d[m]))) {
      e[m - 1] = 0.0;
      m--;
      continue;
    }
    int l = m - 1;
    while (l > 0 && std::fabs(e[l - 1]) > eps * (std::fabs(d[l - 1]) + std::fabs(d[l]))) l--;
    if (l > 0) e[l - 1] = 0.0;
    if (++steps > 30 * n) break;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block closer to its last diagonal entry
    const double del = 0.5 * (d[m - 1] - d[m]), b = e[m - 1];
    const double mu = d[m] - b * b / (del + (del >= 0.0 ? 1.0 : -1.0) * std::hypot(del, b));
    double x = d[l] - mu, y = e[l];
    for (int k = l; k < m; k++) {
      const double r = std::hypot(x, y);
      const double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : y / r;
      if (k > l) e[k - 1] = r;
      // rotation R = [c s; -s c] on rows/columns k, k+1: T <- R T R^T
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk1 - dk) + (c * c - s * s) * ek;
      if (k + 1 < m) {  // the bulge at (k+2, k)
        x = e[k];
        y = s * e[k + 1];
        e[k + 1] *= c;
      }
      for (int r2 = 0; r2 < n; r2++) {  // Z <- Z R^T
        const double zk = z(r2, k), zk1 = z(r2, k + 1);
        z(r2, k) = c * zk + s * zk1;
        z(r2, k + 1) = -s * zk + c * zk1;
      }
    }
  }
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) a(i, j) = i == j ? d[i] : 0.0;
  return m == 0;
}


// Inverse of Phi^T K Phi (symmetric positive semi-definite, leading rank x rank block of the nm x nm
// row-major Kc) over the modes that are independent of the ones before them: symmetric elimination in
// mode order (most energetic first) keeps a mode when its diagonal entry, reduced by the modes kept
// before it, is above 1e-12 of its own (the sine of its angle to their span, in the K inner product,
// above 1e-6); the kept block is inverted by Gauss-Jordan without exchanges (positive definite) and
// the rows and columns of the other modes are zero.  False when no mode is kept.
inline bool independent_inverse(int nm, int rank, const double *Kc, std::vector<double> &inv) {
  std::vector<double> A(Kc, Kc + (size_t)nm * nm);
  std::vector<int> keep;
  for (int j = 0; j < rank; j++) {
    const double d = A[(size_t)j * nm + j], d0 = Kc[(size_t)j * nm + j];
    if (!(d0 > 0.0) || !(d > 1e-12 * d0)) continue;
    keep.push_back(j);
    for (int r = j + 1; r < rank; r++) {
      const double f = A[(size_t)r * nm + j] / d;
      if (f == 0.0) continue;
      for (int c = j + 1; c < rank; c++) A[(size_t)r * nm + c] -= f * A[(size_t)j * nm + c];
    }
  }
  const int k = (int)keep.size();
  std::fill(inv.begin(), inv.end(), 0.0);
  if (k == 0) return false;
  std::vector<double> B((size_t)k * k), I((size_t)k * k, 0.0);
  for (int a = 0; a < k; a++) {
    I[(size_t)a * k + a] = 1.0;
    for (int b = 0; b < k; b++) B[(size_t)a * k + b] = Kc[(size_t)keep[a] * nm + keep[b]];
  }
  for (int col = 0; col < k; col++) {
    const double d = B[(size_t)col * k + col];
    for (int c = 0; c < k; c++) {
      B[(size_t)col * k + c] /= d;
      I[(size_t)col * k + c] /= d;
    }
    for (int r = 0; r < k; r++) {
      if (r == col) continue;
      const double f = B[(size_t)r * k + col];
      if (f == 0.0) continue;
      for (int c = 0; c < k; c++) {
        B[(size_t)r * k + c] -= f * B[(size_t)col * k + c];
        I[(size_t)r * k + c] -= f * I[(size_t)col * k + c];
      }
    }
  }
  for (int a = 0; a < k; a++)
    for (int b = 0; b < k; b++) inv[(size_t)keep[a] * nm + keep[b]] = I[(size_t)a * k + b];
  return true;
}

}  // namespace cgp
