/*
 * Oracle, linear-algebra part: CSR matrix-vector product (the paper's storage
 * format, Section 2.3), Jacobi-preconditioned conjugate gradients,
 * Jacobi-preconditioned BiCGStab and a dense LU solve with partial pivoting.
 * TEST INFRASTRUCTURE ONLY.
 *
 * The loop pragmas are read only by the OpenMP build of the oracle (liboracle_omp.so, -fopenmp), which
 * serves the multi-core CPU baseline; the single-thread build, which judges the GPU path, ignores them.
 *
 * Stopping rule for both Krylov methods: the (recursively updated,
 * unpreconditioned) residual satisfies ||r||_2 <= tol * ||b||_2; a zero right
 * hand side gives x = 0.  The textbook iterations are written out in full.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

void orc_spmv(const orc_csr *A, const double *val, const double *x, double *y) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < A->n; i++) {
    double s = 0.0;
    for (int k = A->rp[i]; k < A->rp[i + 1]; k++) s += val[k] * x[A->col[k]];
    y[i] = s;
  }
}

static double dot(int n, const double *a, const double *b) {
  double s = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : s)
  for (int i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

static void diag_inverse(const orc_csr *A, const double *val, double *dinv) {
  for (int i = 0; i < A->n; i++) {
    double d = 0.0;
    for (int k = A->rp[i]; k < A->rp[i + 1]; k++)
      if (A->col[k] == i) d = val[k];
    dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
  }
}

/* Jacobi-preconditioned CG (Hestenes-Stiefel with preconditioner M = diag(A)) */
int orc_pcg(const orc_csr *A, const double *val, const double *b, double *x, double tol, int maxit,
            int *iters, double *relres) {
  int n = A->n;
  double bn = sqrt(dot(n, b, b));
  *iters = 0;
  if (!isfinite(bn)) { *relres = NAN; return ORC_E_NONFINITE; }
  if (bn == 0.0) {
    memset(x, 0, sizeof(double) * (size_t)n);
    *relres = 0.0;
    return ORC_OK;
  }
  double *r = (double *)malloc(sizeof(double) * (size_t)n), *z = (double *)malloc(sizeof(double) * (size_t)n);
  double *pv = (double *)malloc(sizeof(double) * (size_t)n), *q = (double *)malloc(sizeof(double) * (size_t)n);
  double *dinv = (double *)malloc(sizeof(double) * (size_t)n);
  diag_inverse(A, val, dinv);
  orc_spmv(A, val, x, q);
  for (int i = 0; i < n; i++) { r[i] = b[i] - q[i]; z[i] = dinv[i] * r[i]; pv[i] = z[i]; }
  double rz = dot(n, r, z), rn = sqrt(dot(n, r, r));
  int k = 0, st = ORC_OK;
  while (rn > tol * bn) {
    if (k >= maxit) { st = ORC_E_NOCONV; break; }
    orc_spmv(A, val, pv, q);
    double alpha = rz / dot(n, pv, q);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) { x[i] += alpha * pv[i]; r[i] -= alpha * q[i]; z[i] = dinv[i] * r[i]; }
    double rz_new = dot(n, r, z);
    double beta = rz_new / rz;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) pv[i] = z[i] + beta * pv[i];
    rz = rz_new;
    rn = sqrt(dot(n, r, r));
    k++;
    if (!isfinite(rn)) { st = ORC_E_NONFINITE; break; }
  }
  *iters = k;
  *relres = rn / bn;
  free(r); free(z); free(pv); free(q); free(dinv);
  return st;
}

/* Jacobi right-preconditioned BiCGStab (van der Vorst 1992) */
int orc_bicgstab(const orc_csr *A, const double *val, const double *b, double *x, double tol, int maxit,
                 int *iters, double *relres) {
  int n = A->n;
  double bn = sqrt(dot(n, b, b));
  *iters = 0;
  if (!isfinite(bn)) { *relres = NAN; return ORC_E_NONFINITE; }
  if (bn == 0.0) {
    memset(x, 0, sizeof(double) * (size_t)n);
    *relres = 0.0;
    return ORC_OK;
  }
  size_t sz = sizeof(double) * (size_t)n;
  double *r = malloc(sz), *rh = malloc(sz), *pv = malloc(sz), *v = malloc(sz), *s = malloc(sz);
  double *t = malloc(sz), *ph = malloc(sz), *sh = malloc(sz), *dinv = malloc(sz);
  diag_inverse(A, val, dinv);
  orc_spmv(A, val, x, v);
  for (int i = 0; i < n; i++) { r[i] = b[i] - v[i]; rh[i] = r[i]; pv[i] = 0.0; v[i] = 0.0; }
  double rho = 1.0, alpha = 1.0, omega = 1.0, rn = sqrt(dot(n, r, r));
  int k = 0, st = ORC_OK;
  while (rn > tol * bn) {
    if (k >= maxit) { st = ORC_E_NOCONV; break; }
    double rho_new = dot(n, rh, r);
    double beta = (rho_new / rho) * (alpha / omega);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) { pv[i] = r[i] + beta * (pv[i] - omega * v[i]); ph[i] = dinv[i] * pv[i]; }
    orc_spmv(A, val, ph, v);
    alpha = rho_new / dot(n, rh, v);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) { s[i] = r[i] - alpha * v[i]; sh[i] = dinv[i] * s[i]; }
    orc_spmv(A, val, sh, t);
    double tt = dot(n, t, t);
    omega = tt > 0.0 ? dot(n, t, s) / tt : 0.0;
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; i++) { x[i] += alpha * ph[i] + omega * sh[i]; r[i] = s[i] - omega * t[i]; }
    rho = rho_new;
    rn = sqrt(dot(n, r, r));
    k++;
    if (!isfinite(rn)) { st = ORC_E_NONFINITE; break; }
    if (omega == 0.0 && rn > tol * bn) { st = ORC_E_NOCONV; break; }
  }
  *iters = k;
  *relres = rn / bn;
  free(r); free(rh); free(pv); free(v); free(s); free(t); free(ph); free(sh); free(dinv);
  return st;
}

/* Dense Gaussian elimination with partial pivoting; A (row-major n x n) and b are overwritten. */
int orc_dense_solve(int n, double *A, double *b, double *x) {
  for (int k = 0; k < n; k++) {
    int piv = k;
    for (int i = k + 1; i < n; i++)
      if (fabs(A[(size_t)i * n + k]) > fabs(A[(size_t)piv * n + k])) piv = i;
    if (A[(size_t)piv * n + k] == 0.0) return ORC_E_ARG;
    if (piv != k) {
      for (int j = 0; j < n; j++) {
        double tmp = A[(size_t)k * n + j];
        A[(size_t)k * n + j] = A[(size_t)piv * n + j];
        A[(size_t)piv * n + j] = tmp;
      }
      double tb = b[k]; b[k] = b[piv]; b[piv] = tb;
    }
    for (int i = k + 1; i < n; i++) {
      double f = A[(size_t)i * n + k] / A[(size_t)k * n + k];
      if (f == 0.0) continue;
      for (int j = k; j < n; j++) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; i--) {
    double s = b[i];
    for (int j = i + 1; j < n; j++) s -= A[(size_t)i * n + j] * x[j];
    x[i] = s / A[(size_t)i * n + i];
  }
  return ORC_OK;
}
