/*
 * Oracle, flow-functional part: the force the fluid exerts on a marked part of
 * the boundary (the body of Section 3.3, for drag, lift and their pressure and
 * viscous parts, Table 6 and Fig. 13; or a wall, whose shear stress locates
 * the reattachment point of Section 3.2, Fig. 7).  TEST INFRASTRUCTURE ONLY.
 *
 * A fine boundary edge e = (a, b) of a marked coarse boundary edge (fine edge j
 * descends from coarse edge j >> l, since every subdivision splits edge k into
 * edges 2k and 2k+1) lies on one fine triangle with third vertex c.  With n the
 * unit normal of e pointing into the fluid (towards c) and the Cauchy stress
 * sigma = -p I + mu (grad u + grad u^T) of the P1 fields (pressure linear along
 * e, velocity gradient constant on the triangle), the edge's share of the force
 * on the body is
 *   pressure part  -|e| (p_a + p_b)/2 n,
 *   viscous part    |e| mu (grad u + grad u^T) n.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

/* third vertex of the fine triangle holding edge (a, b), or -1 */
static int third_vertex(const orc_level *L, int a, int b) {
  for (int t = 0; t < L->t; t++) {
    const int *v = L->tri + 3 * t;
    for (int k = 0; k < 3; k++) {
      int p = v[k], q = v[(k + 1) % 3];
      if ((p == a && q == b) || (p == b && q == a)) return v[(k + 2) % 3];
    }
  }
  return -1;
}

/* Per marked fine edge: x, y of the midpoint, length, pressure force x, y, viscous force x, y, 0.
 * mark: [nb_coarse] 0/1 over the coarse boundary edges.  Returns the number of edges written, or -1.
 * out may be NULL (count only); it holds up to `cap` rows of 8. */
int orc_surface_traction(const orc_problem *p, const int *mark, const double *u, const double *pf, double *out,
                         int cap) {
  if (!p || !mark || !u || !pf) return -1;
  const orc_level *F = &p->lev[p->levels];
  int count = 0;
  for (int j = 0; j < F->nb; j++) {
    if (!mark[j >> p->levels]) continue;
    if (out && count >= cap) return -1;
    int a = F->bedge[2 * j], b = F->bedge[2 * j + 1];
    int c = third_vertex(F, a, b);
    if (c < 0) return -1;
    const double *xa = F->xy + 2 * a, *xb = F->xy + 2 * b, *xc = F->xy + 2 * c;
    double ex = xb[0] - xa[0], ey = xb[1] - xa[1];
    double len = sqrt(ex * ex + ey * ey);
    double nx = -ey / len, ny = ex / len; /* a unit normal of e, turned towards c */
    if (nx * (xc[0] - xa[0]) + ny * (xc[1] - xa[1]) < 0.0) { nx = -nx; ny = -ny; }
    /* P1 gradient on triangle (a, b, c): grad phi_i = (y_j - y_k, x_k - x_j) / (2A) cyclically */
    const double *X[3] = {xa, xb, xc};
    const int V[3] = {a, b, c};
    double A2 = (xb[0] - xa[0]) * (xc[1] - xa[1]) - (xc[0] - xa[0]) * (xb[1] - xa[1]);
    double G[2][2] = {{0.0, 0.0}, {0.0, 0.0}}; /* G[i][j] = d u_i / d x_j */
    for (int k = 0; k < 3; k++) {
      const double *xj = X[(k + 1) % 3], *xk = X[(k + 2) % 3];
      double gx = (xj[1] - xk[1]) / A2, gy = (xk[0] - xj[0]) / A2;
      for (int i = 0; i < 2; i++) {
        G[i][0] += u[2 * V[k] + i] * gx;
        G[i][1] += u[2 * V[k] + i] * gy;
      }
    }
    double pm = 0.5 * (pf[a] + pf[b]);
    double sxx = 2.0 * G[0][0], syy = 2.0 * G[1][1], sxy = G[0][1] + G[1][0];
    if (out) {
      double *o = out + 8 * (size_t)count;
      o[0] = 0.5 * (xa[0] + xb[0]);
      o[1] = 0.5 * (xa[1] + xb[1]);
      o[2] = len;
      o[3] = -len * pm * nx;
      o[4] = -len * pm * ny;
      o[5] = len * p->mu * (sxx * nx + sxy * ny);
      o[6] = len * p->mu * (sxy * nx + syy * ny);
      o[7] = 0.0;
    }
    count++;
  }
  return count;
}

/* Totals over the marked surface: out[4] = pressure force x, y; viscous force x, y. */
int orc_surface_force(const orc_problem *p, const int *mark, const double *u, const double *pf, double *out) {
  int ne = orc_surface_traction(p, mark, u, pf, NULL, 0);
  if (ne < 0) return ORC_E_ARG;
  double *e = (double *)calloc(8 * (size_t)(ne ? ne : 1), sizeof(double));
  orc_surface_traction(p, mark, u, pf, e, ne);
  for (int k = 0; k < 4; k++) out[k] = 0.0;
  for (int i = 0; i < ne; i++)
    for (int k = 0; k < 4; k++) out[k] += e[8 * (size_t)i + 3 + k];
  free(e);
  return ORC_OK;
}
