/*
 * Oracle, reporting part: the paper's discrete error norms (Section 3,
 * Eqs. 31-33) of a P1 field A against an exact field a on a mesh of M
 * triangles E_i:
 *   e = A - a                                  (Eq. 31)
 *   ||e||_L2(V)   = sqrt( (1/M) sum_i ||e||^2_L2(E_i) )   (Eq. 32, with the 1/M as printed)
 *   ||e||_Linf(V) = max_i ||e||_Linf(E_i)                 (Eq. 33)
 * For a vector field |e| is the Euclidean length of the error vector.  The
 * element integral uses the symmetric 6-point rule of degree 4 (Dunavant
 * 1985); the element maximum is taken over those points and the vertices.
 * Used to report Taylor-Green errors; never for parity.  TEST
 * INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <stdlib.h>

#include "oracle.h"

#define NQ 6
/* barycentric points (l1, l2, l3) and weights (summing to 1) of the degree-4 rule */
static const double QA[2] = {0.445948490915965, 0.091576213509771};
static const double QB[2] = {0.108103018168070, 0.816847572980459};
static const double QW[2] = {0.223381589678011, 0.109951743655322};

static void bary(int k, double *l) {
  int g = k / 3, r = k % 3;
  l[0] = l[1] = l[2] = QA[g];
  l[r] = QB[g];
}

int orc_quad_npts(void) { return NQ; }

/* Quadrature points of every triangle of `level`: xyq[t][NQ][2]. */
int orc_quad_points(const orc_problem *p, int level, double *xyq) {
  if (!p || level < 0 || level > p->levels || !xyq) return ORC_E_ARG;
  const orc_level *L = &p->lev[level];
  for (int t = 0; t < L->t; t++) {
    const int *v = L->tri + 3 * t;
    for (int k = 0; k < NQ; k++) {
      double l[3];
      bary(k, l);
      double x = 0.0, y = 0.0;
      for (int j = 0; j < 3; j++) { x += l[j] * L->xy[2 * v[j]]; y += l[j] * L->xy[2 * v[j] + 1]; }
      xyq[((size_t)t * NQ + k) * 2] = x;
      xyq[((size_t)t * NQ + k) * 2 + 1] = y;
    }
  }
  return ORC_OK;
}

/* Nodal field A[n][nc] (nc = 1 or 2 components) on `level`, exact values at the
 * quadrature points aq[t][NQ][nc] and at the nodes an[n][nc]. */
int orc_error_norms(const orc_problem *p, int level, int nc, const double *A, const double *aq,
                    const double *an, double *l2, double *linf) {
  if (!p || level < 0 || level > p->levels || (nc != 1 && nc != 2) || !A || !aq || !an) return ORC_E_ARG;
  const orc_level *L = &p->lev[level];
  double sum = 0.0, mx = 0.0;
  for (int t = 0; t < L->t; t++) {
    const int *v = L->tri + 3 * t;
    const double *p0 = L->xy + 2 * v[0], *p1 = L->xy + 2 * v[1], *p2 = L->xy + 2 * v[2];
    double area = 0.5 * fabs((p1[0] - p0[0]) * (p2[1] - p0[1]) - (p2[0] - p0[0]) * (p1[1] - p0[1]));
    double el2 = 0.0, emax = 0.0;
    for (int k = 0; k < NQ; k++) {
      double l[3], e2 = 0.0;
      bary(k, l);
      for (int c = 0; c < nc; c++) {
        double Ah = 0.0;
        for (int j = 0; j < 3; j++) Ah += l[j] * A[(size_t)v[j] * nc + c];
        double e = Ah - aq[((size_t)t * NQ + k) * nc + c];
        e2 += e * e;
      }
      el2 += QW[k / 3] * area * e2;
      if (sqrt(e2) > emax) emax = sqrt(e2);
    }
    for (int j = 0; j < 3; j++) {
      double e2 = 0.0;
      for (int c = 0; c < nc; c++) {
        double e = A[(size_t)v[j] * nc + c] - an[(size_t)v[j] * nc + c];
        e2 += e * e;
      }
      if (sqrt(e2) > emax) emax = sqrt(e2);
    }
    sum += el2;
    if (emax > mx) mx = emax;
  }
  *l2 = sqrt(sum / L->t);
  *linf = mx;
  return ORC_OK;
}
