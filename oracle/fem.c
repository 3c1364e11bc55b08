/*
 * Oracle, finite-element part: P1 element operators and global assembly of
 * the matrices of Eqs. (16)-(18) on the fine mesh and of the coarse-mesh
 * Laplacian and divergence built from coarse shape functions (Section 2.2).
 * TEST INFRASTRUCTURE ONLY.
 *
 * With b = (y2-y3, y3-y1, y1-y2), c = (x3-x2, x1-x3, x2-x1) and A the area,
 * the exact P1 integrals are
 *   mass        M_ij  = int phi_i phi_j            = A/12 (1 + delta_ij)
 *   stiffness   K_ij  = int grad phi_i . grad phi_j = (b_i b_j + c_i c_j) / (4A)
 *   x-derivative Dx_ij = int phi_i d(phi_j)/dx       = b_j / 6
 *   y-derivative Dy_ij = int phi_i d(phi_j)/dy       = c_j / 6
 *   convection  N_ij  = rho int phi_i (u_h . grad phi_j)
 *                     = rho/24 [ (u_i + sum u) b_j + (v_i + sum v) c_j ].
 * The viscous operator of Eq. (16) is mu*K (sign of -mu Laplacian), the pressure
 * Laplacian of Eq. (17) is -K, and the divergence D and gradient G are the same
 * pair (Dx, Dy) (the divergence is integrated without integration by parts).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

int orc_csr_find(const orc_csr *A, int i, int j);

void orc_element(const double *xy3, const double *u3, double rho, double *M, double *K, double *Dx,
                 double *Dy, double *N) {
  double x1 = xy3[0], y1 = xy3[1], x2 = xy3[2], y2 = xy3[3], x3 = xy3[4], y3 = xy3[5];
  double b[3] = {y2 - y3, y3 - y1, y1 - y2};
  double c[3] = {x3 - x2, x1 - x3, x2 - x1};
  double area = 0.5 * ((x2 - x1) * (y3 - y1) - (x3 - x1) * (y2 - y1));
  double su = 0.0, sv = 0.0;
  if (u3) { su = u3[0] + u3[2] + u3[4]; sv = u3[1] + u3[3] + u3[5]; }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      if (M) M[3 * i + j] = area / 12.0 * (i == j ? 2.0 : 1.0);
      if (K) K[3 * i + j] = (b[i] * b[j] + c[i] * c[j]) / (4.0 * area);
      if (Dx) Dx[3 * i + j] = b[j] / 6.0;
      if (Dy) Dy[3 * i + j] = c[j] / 6.0;
      if (N && u3) N[3 * i + j] = rho / 24.0 * ((u3[2 * i] + su) * b[j] + (u3[2 * i + 1] + sv) * c[j]);
    }
}

static void element_xy(const orc_level *L, int e, double *xy3) {
  for (int k = 0; k < 3; k++) {
    xy3[2 * k] = L->xy[2 * L->tri[3 * e + k]];
    xy3[2 * k + 1] = L->xy[2 * L->tri[3 * e + k] + 1];
  }
}

/* add an element matrix into CSR values */
static void scatter(const orc_csr *A, double *val, const int *v, const double *Ae) {
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) val[orc_csr_find(A, v[a], v[b])] += Ae[3 * a + b];
}

int orc_assemble(orc_problem *p, double rho, double mu, double dt, int restrict_mode, int mass_mode) {
  if (!p || !(rho > 0) || !(mu >= 0) || !(dt > 0) || restrict_mode < 0 || restrict_mode > 1 || mass_mode < 0 ||
      mass_mode > 1)
    return ORC_E_ARG;
  p->rho = rho; p->mu = mu; p->dt = dt;
  p->restrict_mode = restrict_mode; p->mass_mode = mass_mode;
  const orc_level *F = &p->lev[p->levels], *C = &p->lev[0];
  size_t nf = (size_t)p->pf.nnz, nc = (size_t)p->pc.nnz;
  free(p->Mf); free(p->Kf); free(p->Dxf); free(p->Dyf); free(p->mlf);
  free(p->Kc); free(p->Kc_bc); free(p->Dxc); free(p->Dyc); free(p->mc);
  p->Mf = (double *)calloc(nf, sizeof(double));
  p->Kf = (double *)calloc(nf, sizeof(double));
  p->Dxf = (double *)calloc(nf, sizeof(double));
  p->Dyf = (double *)calloc(nf, sizeof(double));
  p->mlf = (double *)calloc((size_t)F->n, sizeof(double));
  p->Kc = (double *)calloc(nc, sizeof(double));
  p->Kc_bc = (double *)calloc(nc, sizeof(double));
  p->Dxc = (double *)calloc(nc, sizeof(double));
  p->Dyc = (double *)calloc(nc, sizeof(double));
  p->mc = (double *)calloc((size_t)C->n, sizeof(double));
  double xy3[6], Me[9], Ke[9], Dxe[9], Dye[9];
  for (int e = 0; e < F->t; e++) {
    element_xy(F, e, xy3);
    orc_element(xy3, NULL, rho, Me, Ke, Dxe, Dye, NULL);
    const int *v = F->tri + 3 * e;
    scatter(&p->pf, p->Mf, v, Me);
    scatter(&p->pf, p->Kf, v, Ke);
    scatter(&p->pf, p->Dxf, v, Dxe);
    scatter(&p->pf, p->Dyf, v, Dye);
  }
  /* lumped fine mass: row sums of M */
  for (int i = 0; i < F->n; i++)
    for (int k = p->pf.rp[i]; k < p->pf.rp[i + 1]; k++) p->mlf[i] += p->Mf[k];
  for (int e = 0; e < C->t; e++) {
    element_xy(C, e, xy3);
    orc_element(xy3, NULL, rho, Me, Ke, Dxe, Dye, NULL);
    const int *v = C->tri + 3 * e;
    scatter(&p->pc, p->Kc, v, Ke);
    scatter(&p->pc, p->Dxc, v, Dxe);
    scatter(&p->pc, p->Dyc, v, Dye);
    double area = 0.5 * ((xy3[2] - xy3[0]) * (xy3[5] - xy3[1]) - (xy3[4] - xy3[0]) * (xy3[3] - xy3[1]));
    for (int k = 0; k < 3; k++) p->mc[v[k]] += area / 3.0;
  }
  /* coarse pressure Laplacian with p = 0 imposed at pressure-Dirichlet nodes
   * (Eq. 14): rows and columns of those nodes become identity rows/cols */
  memcpy(p->Kc_bc, p->Kc, sizeof(double) * nc);
  for (int i = 0; i < C->n; i++)
    for (int k = p->pc.rp[i]; k < p->pc.rp[i + 1]; k++) {
      int j = p->pc.col[k];
      if (p->pdir[i] || p->pdir[j]) p->Kc_bc[k] = (i == j) ? 1.0 : 0.0;
    }
  p->assembled = 1;
  return ORC_OK;
}

/* what: 0 Mf, 1 Kf, 2 Dxf, 3 Dyf, 4 lumped fine mass, 5 Kc (no BC), 6 Kc with BC,
 * 7 Dxc, 8 Dyc, 9 coarse lumped mass */
int orc_export_values(const orc_problem *p, int what, double *dst) {
  if (!p->assembled) return ORC_E_ARG;
  size_t nf = (size_t)p->pf.nnz, nc = (size_t)p->pc.nnz;
  const double *src[10] = {p->Mf, p->Kf, p->Dxf, p->Dyf, p->mlf, p->Kc, p->Kc_bc, p->Dxc, p->Dyc, p->mc};
  size_t len[10] = {nf, nf, nf, nf, (size_t)p->lev[p->levels].n, nc, nc, nc, nc, (size_t)p->lev[0].n};
  if (what < 0 || what > 9) return ORC_E_ARG;
  memcpy(dst, src[what], sizeof(double) * len[what]);
  return ORC_OK;
}

/* Convection matrix N(u) of Eq. (16) on the fine pattern (values include rho). */
void orc_convection(const orc_problem *p, const double *u, double *Nval) {
  const orc_level *F = &p->lev[p->levels];
  memset(Nval, 0, sizeof(double) * (size_t)p->pf.nnz);
  double xy3[6], u3[6], Ne[9];
  for (int e = 0; e < F->t; e++) {
    element_xy(F, e, xy3);
    for (int k = 0; k < 3; k++) {
      u3[2 * k] = u[2 * F->tri[3 * e + k]];
      u3[2 * k + 1] = u[2 * F->tri[3 * e + k] + 1];
    }
    orc_element(xy3, u3, p->rho, NULL, NULL, NULL, NULL, Ne);
    scatter(&p->pf, Nval, F->tri + 3 * e, Ne);
  }
}
