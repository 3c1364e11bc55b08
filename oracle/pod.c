/*
 * Oracle, basis part of the learned initial guess: the proper orthogonal
 * decomposition (POD) of pressure snapshots by the method of snapshots
 * (Sirovich 1987).  The paper has no such step; it belongs to the learned
 * initial-guess extension of the coarse Poisson solve (Eq. 21), whose
 * correctness never depends on the guess.  TEST INFRASTRUCTURE ONLY.
 *
 * With snapshots s_1..s_S (rows of snaps[S][n]) and a positive weight w (the
 * coarse lumped mass, so that the modes are orthonormal in the discrete L2
 * inner product of the pressure space):
 *   1. Gram matrix G_ab = sum_i s_a[i] w[i] s_b[i];
 *   2. all eigenpairs of G by the cyclic Jacobi method (plane rotations that
 *      zero one off-diagonal pair at a time, swept row by row until the
 *      off-diagonal mass is at rounding level; Golub & Van Loan, Matrix
 *      Computations, the symmetric Jacobi method);
 *   3. eigenvalues in decreasing order; mode k = sum_a s_a V_ak / sqrt(lambda_k).
 * Modes whose eigenvalue is not above 1e-20 of the largest are left out: zero
 * column, energy 0 (the same rule as the library's basis).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* Eigen-decomposition of the symmetric q x q matrix A (overwritten: its diagonal
 * ends up holding the eigenvalues); V receives the eigenvectors as columns. */
void orc_jacobi_eigen(int q, double *A, double *V) {
  memset(V, 0, sizeof(double) * (size_t)q * q);
  for (int i = 0; i < q; i++) V[(size_t)i * q + i] = 1.0;
  double total = 0.0;
  for (size_t k = 0; k < (size_t)q * q; k++) total += A[k] * A[k];
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0;
    for (int i = 0; i < q; i++)
      for (int j = 0; j < q; j++)
        if (i != j) off += A[(size_t)i * q + j] * A[(size_t)i * q + j];
    if (off <= 1e-32 * total) break;
    for (int p = 0; p < q - 1; p++)
      for (int r = p + 1; r < q; r++) {
        double apr = A[(size_t)p * q + r];
        if (apr == 0.0) continue;
        double app = A[(size_t)p * q + p], arr = A[(size_t)r * q + r];
        /* rotation angle that zeroes A[p][r]: t = tan(angle) is the smaller root of t^2 + 2 theta t - 1 */
        double theta = (arr - app) / (2.0 * apr);
        double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < q; k++) { /* A <- A J (columns p, r) */
          double akp = A[(size_t)k * q + p], akr = A[(size_t)k * q + r];
          A[(size_t)k * q + p] = c * akp - s * akr;
          A[(size_t)k * q + r] = s * akp + c * akr;
        }
        for (int k = 0; k < q; k++) { /* A <- J^T A (rows p, r) */
          double apk = A[(size_t)p * q + k], ark = A[(size_t)r * q + k];
          A[(size_t)p * q + k] = c * apk - s * ark;
          A[(size_t)r * q + k] = s * apk + c * ark;
        }
        for (int k = 0; k < q; k++) { /* V <- V J */
          double vkp = V[(size_t)k * q + p], vkr = V[(size_t)k * q + r];
          V[(size_t)k * q + p] = c * vkp - s * vkr;
          V[(size_t)k * q + r] = s * vkp + c * vkr;
        }
      }
  }
}

/* Returns the number of modes kept (<= m), or -1 on a bad argument.
 * phi: [n][m] row-major, energy: [m] (may be NULL). */
int orc_pod(int S, int n, const double *snaps, const double *w, int m, double *phi, double *energy) {
  if (S < 1 || n < 1 || m < 1 || m > S || !snaps || !w || !phi) return -1;
  double *G = (double *)calloc((size_t)S * S, sizeof(double));
  double *V = (double *)calloc((size_t)S * S, sizeof(double));
  int *order = (int *)malloc(sizeof(int) * (size_t)S);
  for (int a = 0; a < S; a++)
    for (int b = 0; b < S; b++) {
      double acc = 0.0;
      for (int i = 0; i < n; i++) acc += snaps[(size_t)a * n + i] * w[i] * snaps[(size_t)b * n + i];
      G[(size_t)a * S + b] = acc;
    }
  orc_jacobi_eigen(S, G, V);
  for (int a = 0; a < S; a++) order[a] = a;
  for (int a = 1; a < S; a++) { /* insertion sort, decreasing eigenvalue */
    int k = order[a], b = a - 1;
    double lk = G[(size_t)k * S + k];
    while (b >= 0 && G[(size_t)order[b] * S + order[b]] < lk) { order[b + 1] = order[b]; b--; }
    order[b + 1] = k;
  }
  double lam0 = G[(size_t)order[0] * S + order[0]];
  memset(phi, 0, sizeof(double) * (size_t)n * m);
  if (energy) memset(energy, 0, sizeof(double) * (size_t)m);
  int rank = 0;
  for (int k = 0; k < m; k++) {
    int c = order[k];
    double lam = G[(size_t)c * S + c];
    if (!(lam0 > 0.0) || !(lam > 1e-20 * lam0)) break;
    rank = k + 1;
    if (energy) energy[k] = lam;
    for (int i = 0; i < n; i++) {
      double acc = 0.0;
      for (int a = 0; a < S; a++) acc += snaps[(size_t)a * n + i] * V[(size_t)a * S + c];
      phi[(size_t)i * m + k] = acc / sqrt(lam);
    }
  }
  free(G); free(V); free(order);
  return rank;
}
