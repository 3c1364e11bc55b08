/*
 * Oracle, the paper's linear solver (Section 2.3, "Computational implementation"):
 * GMRES(m) preconditioned with the incomplete LU factorisation without fill,
 * ILU(0), on the CSR storage of the matrix.  TEST INFRASTRUCTURE ONLY.
 *
 * ILU(0) (Saad, Iterative Methods for Sparse Linear Systems, the IKJ form of
 * Gaussian elimination restricted to the pattern): for each row i in order, for
 * each column k < i of row i in increasing order, l_ik = a_ik / u_kk, then every
 * entry (i, j) of row i with j > k that also exists in row k is reduced by
 * l_ik u_kj.  L (unit diagonal, strictly lower part) and U (upper part with the
 * diagonal) share the matrix's value array.  By construction (L U)_ij = a_ij on
 * the pattern.
 *
 * GMRES(m) with right preconditioning (x = x0 + M^-1 V y): Arnoldi on A M^-1
 * with modified Gram-Schmidt (orth = 0) or classical Gram-Schmidt applied twice
 * (orth = 1), Givens rotations on the Hessenberg matrix, a restart after m
 * inner steps.  The two orthogonalisations agree in exact arithmetic; in
 * floating point the second keeps the basis closer to orthogonal, which on
 * stagnating restarted cycles changes the iteration count.  Stop when ||b - A x||_2 <= tol ||b||_2; the
 * rotated right-hand side estimates that residual inside a cycle and the true
 * residual is computed at every restart and at the end.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static int find_col(const orc_csr *A, int row, int col) {
  int lo = A->rp[row], hi = A->rp[row + 1] - 1;
  while (lo <= hi) {
    int mid = (lo + hi) / 2;
    if (A->col[mid] == col) return mid;
    if (A->col[mid] < col) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

int orc_ilu0(const orc_csr *A, const double *val, double *lu) {
  memcpy(lu, val, sizeof(double) * (size_t)A->nnz);
  for (int i = 0; i < A->n; i++) {
    for (int kk = A->rp[i]; kk < A->rp[i + 1]; kk++) {
      int k = A->col[kk];
      if (k >= i) break; /* columns sorted: the strictly lower part comes first */
      int dk = find_col(A, k, k);
      if (dk < 0 || lu[dk] == 0.0) return ORC_E_ARG;
      double lik = lu[kk] / lu[dk];
      lu[kk] = lik;
      for (int jj = kk + 1; jj < A->rp[i + 1]; jj++) {
        int j = A->col[jj];
        int kj = find_col(A, k, j);
        if (kj >= 0) lu[jj] -= lik * lu[kj];
      }
    }
  }
  return ORC_OK;
}

/* z = (L U)^-1 r: forward substitution with unit L, then backward substitution with U */
void orc_ilu0_apply(const orc_csr *A, const double *lu, const double *r, double *z) {
  int n = A->n;
  for (int i = 0; i < n; i++) {
    double s = r[i];
    for (int k = A->rp[i]; k < A->rp[i + 1] && A->col[k] < i; k++) s -= lu[k] * z[A->col[k]];
    z[i] = s;
  }
  for (int i = n - 1; i >= 0; i--) {
    double s = z[i], d = 1.0;
    for (int k = A->rp[i]; k < A->rp[i + 1]; k++) {
      int j = A->col[k];
      if (j > i) s -= lu[k] * z[j];
      else if (j == i) d = lu[k];
    }
    z[i] = s / d;
  }
}

static double dot(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

int orc_gmres(const orc_csr *A, const double *val, const double *lu, const double *b, double *x, int m, double tol,
              int maxit, int orth, int *iters, double *relres) {
  int n = A->n;
  *iters = 0;
  if (m < 1) return ORC_E_ARG;
  double bn = sqrt(dot(n, b, b));
  if (!isfinite(bn)) { *relres = NAN; return ORC_E_NONFINITE; }
  if (bn == 0.0) {
    memset(x, 0, sizeof(double) * (size_t)n);
    *relres = 0.0;
    return ORC_OK;
  }
  double *V = (double *)calloc((size_t)(m + 1) * n, sizeof(double));
  double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double)); /* H[i][j], i <= j + 1 */
  double *cs = (double *)calloc((size_t)m, sizeof(double)), *sn = (double *)calloc((size_t)m, sizeof(double));
  double *gv = (double *)calloc((size_t)m + 1, sizeof(double)), *y = (double *)calloc((size_t)m, sizeof(double));
  double *w = (double *)malloc(sizeof(double) * (size_t)n), *z = (double *)malloc(sizeof(double) * (size_t)n);
  int k = 0, st = ORC_OK;
  double rn;
  for (;;) {
    /* true residual r = b - A x into V[0] */
    orc_spmv(A, val, x, w);
    for (int i = 0; i < n; i++) V[i] = b[i] - w[i];
    rn = sqrt(dot(n, V, V));
    if (!isfinite(rn)) { st = ORC_E_NONFINITE; break; }
    if (rn <= tol * bn) break;
    if (k >= maxit) { st = ORC_E_NOCONV; break; }
    for (int i = 0; i < n; i++) V[i] /= rn;
    memset(gv, 0, sizeof(double) * ((size_t)m + 1));
    gv[0] = rn;
    int j = 0;
    for (; j < m && k < maxit; j++, k++) {
      double *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
      if (lu) orc_ilu0_apply(A, lu, vj, z); else memcpy(z, vj, sizeof(double) * (size_t)n);
      orc_spmv(A, val, z, w);
      if (orth == 0) {
        for (int i = 0; i <= j; i++) { /* modified Gram-Schmidt */
          double h = dot(n, w, V + (size_t)i * n);
          H[(size_t)i * m + j] = h;
          for (int q = 0; q < n; q++) w[q] -= h * V[(size_t)i * n + q];
        }
      } else {
        for (int i = 0; i <= j; i++) H[(size_t)i * m + j] = 0.0;
        for (int pass = 0; pass < 2; pass++) { /* classical Gram-Schmidt, twice */
          double *hh = (double *)malloc(sizeof(double) * ((size_t)j + 1));
          for (int i = 0; i <= j; i++) hh[i] = dot(n, w, V + (size_t)i * n);
          for (int i = 0; i <= j; i++) {
            for (int q = 0; q < n; q++) w[q] -= hh[i] * V[(size_t)i * n + q];
            H[(size_t)i * m + j] += hh[i];
          }
          free(hh);
        }
      }
      double hn = sqrt(dot(n, w, w));
      H[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0.0)
        for (int q = 0; q < n; q++) vn[q] = w[q] / hn;
      /* earlier rotations, then the one that zeroes H[j+1][j] */
      for (int i = 0; i < j; i++) {
        double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
      double r = hypot(a, c);
      cs[j] = r > 0.0 ? a / r : 1.0;
      sn[j] = r > 0.0 ? c / r : 0.0;
      H[(size_t)j * m + j] = r;
      H[(size_t)(j + 1) * m + j] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      if (fabs(gv[j + 1]) <= tol * bn || hn == 0.0) { j++; k++; break; }
    }
    /* y = H^-1 g (upper triangular j x j), x += M^-1 V y */
    for (int i = j - 1; i >= 0; i--) {
      double s = gv[i];
      for (int q = i + 1; q < j; q++) s -= H[(size_t)i * m + q] * y[q];
      y[i] = s / H[(size_t)i * m + i];
    }
    memset(w, 0, sizeof(double) * (size_t)n);
    for (int i = 0; i < j; i++)
      for (int q = 0; q < n; q++) w[q] += y[i] * V[(size_t)i * n + q];
    if (lu) orc_ilu0_apply(A, lu, w, z); else memcpy(z, w, sizeof(double) * (size_t)n);
    for (int q = 0; q < n; q++) x[q] += z[q];
  }
  *iters = k;
  *relres = rn / bn;
  free(V); free(H); free(cs); free(sn); free(gv); free(y); free(w); free(z);
  return st;
}
