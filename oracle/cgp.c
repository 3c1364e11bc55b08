/*
 * Oracle, time-step part: one IFE-CGP step (Section 2.2, Eqs. 19-23) with the
 * non-incremental pressure correction of Section 2.1 (Eqs. 9-15) and the P1
 * matrices of Eqs. (16)-(18).  TEST INFRASTRUCTURE ONLY.
 *
 * Readings taken where the paper is silent (the GPU path follows the same):
 *  - rho is carried as in Eqs. (9), (12), (15): momentum matrix
 *    rho*M + dt*mu*K + dt*N(u^n) (N includes rho), right-hand side
 *    rho*M*U^n + dt*M*F^{n+1}, coarse Poisson K P = -(rho/dt) D U, correction
 *    factor dt/rho.
 *  - "boundary conditions enforced in the discrete operators": symmetric
 *    elimination on the fixed sparsity pattern.  Dirichlet rows/columns are
 *    cleared except for the diagonal, which keeps its value a_ii (so that the
 *    residual norm weighs those rows like the others), the right-hand side
 *    there is a_ii g_i, and the known values g^{n+1} are moved to the
 *    right-hand side of the other rows.
 *  - pressure p = 0 on every node of an outflow edge of the Poisson mesh
 *    (Eq. 14); without such nodes the Poisson problem is pure Neumann
 *    (Eq. 13): the right-hand side is made orthogonal to constants by
 *    subtracting its arithmetic mean, and the solution is shifted to zero
 *    lumped-mass-weighted mean.
 *  - restriction is injection at the shared nodes (Eqs. 20, 30); the
 *    alternative the paper calls feasible, the transpose of prolongation, is
 *    mode 1.  Prolongation is linear interpolation (Eqs. 22, 29), chained over
 *    the levels.
 *  - correction (Eq. 23) solves with the consistent mass matrix (mode 0) or
 *    divides by the lumped mass (mode 1); velocity data are re-imposed last.
 *  - incremental pressure correction (the extension Remark 3.1 and the
 *    conclusions point to; pressure_mode 1 = standard, 2 = rotational form):
 *    the momentum right-hand side gains -dt G P_f^n with P_f^n the prolonged
 *    previous pressure; the coarse Poisson equation of Eq. (21) is solved for
 *    the increment phi with the same right-hand side and boundary conditions;
 *    Eq. (23) corrects with the prolonged increment; the new coarse pressure is
 *    P^n + phi (standard), or P^n + phi - mu q (rotational), where q is the
 *    restricted divergence of U~ divided by the coarse lumped mass (a lumped
 *    L2 projection of div U~ onto the coarse pressure space), zero on the
 *    pressure-Dirichlet nodes, and the result is shifted to zero
 *    lumped-mass-weighted mean when there are none.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

void orc_convection(const orc_problem *p, const double *u, double *Nval);

static double *dalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

/* Symmetric Dirichlet elimination on A (values on pattern P) and rhs for one
 * velocity component c of g: rows j outside D get rhs_j -= sum_{i in D} A_ji g_i,
 * then D rows and columns are cleared except for the diagonal a_ii (kept; 1 if
 * it is not positive) and rhs_i = a_ii g_i. */
static void eliminate(const orc_csr *P, double *val, double *rhs, const unsigned char *dir, const double *g, int c) {
  for (int j = 0; j < P->n; j++) {
    if (dir[j]) continue;
    for (int k = P->rp[j]; k < P->rp[j + 1]; k++)
      if (dir[P->col[k]]) rhs[j] -= val[k] * g[2 * P->col[k] + c];
  }
  for (int j = 0; j < P->n; j++) {
    double d = 1.0;
    if (dir[j])
      for (int k = P->rp[j]; k < P->rp[j + 1]; k++)
        if (P->col[k] == j && val[k] > 0.0) d = val[k];
    for (int k = P->rp[j]; k < P->rp[j + 1]; k++) {
      int i = P->col[k];
      if (dir[j] || dir[i]) val[k] = (i == j) ? d : 0.0;
    }
    if (dir[j]) rhs[j] = d * g[2 * j + c];
  }
}

/* Step 1, Eq. (19): (rho M + dt N(U^n) + dt mu K) U~ = rho M U^n + dt M F, per component;
 * with pn (the incremental schemes) the right-hand side also gets -dt G P_f^n. */
static int momentum(orc_problem *p, const double *g_next, const double *f_next, const double *u, const double *pn,
                    double *ut, double tol, int maxit, orc_stats *st) {
  const orc_csr *P = &p->pf;
  int n = P->n;
  size_t nnz = (size_t)P->nnz;
  double *Nv = dalloc(nnz), *A = dalloc(nnz), *Ac = dalloc(nnz);
  double *uc = dalloc((size_t)n), *tmp = dalloc((size_t)n), *rhs = dalloc((size_t)n), *x = dalloc((size_t)n);
  orc_convection(p, u, Nv);
  for (size_t k = 0; k < nnz; k++) A[k] = p->rho * p->Mf[k] + p->dt * p->mu * p->Kf[k] + p->dt * Nv[k];
  int status = ORC_OK;
  for (int c = 0; c < 2; c++) {
    for (int i = 0; i < n; i++) uc[i] = u[2 * i + c];
    orc_spmv(P, p->Mf, uc, tmp);
    for (int i = 0; i < n; i++) rhs[i] = p->rho * tmp[i];
    if (f_next) {
      for (int i = 0; i < n; i++) uc[i] = f_next[2 * i + c];
      orc_spmv(P, p->Mf, uc, tmp);
      for (int i = 0; i < n; i++) rhs[i] += p->dt * tmp[i];
    }
    if (pn) {
      orc_spmv(P, c == 0 ? p->Dxf : p->Dyf, pn, tmp);
      for (int i = 0; i < n; i++) rhs[i] -= p->dt * tmp[i];
    }
    memcpy(Ac, A, sizeof(double) * nnz);
    eliminate(P, Ac, rhs, p->vdir, g_next, c);
    /* initial guess U^n with the known values g^{n+1} on the Dirichlet rows */
    for (int i = 0; i < n; i++) x[i] = p->vdir[i] ? g_next[2 * i + c] : u[2 * i + c];
    int it; double rr;
    int s = orc_bicgstab(P, Ac, rhs, x, tol, maxit, &it, &rr);
    if (st) { st->mom_iters[c] = it; st->mom_relres[c] = rr; }
    if (s != ORC_OK && status == ORC_OK) status = s;
    for (int i = 0; i < n; i++) ut[2 * i + c] = x[i];
  }
  free(Nv); free(A); free(Ac); free(uc); free(tmp); free(rhs); free(x);
  return status;
}

int orc_momentum(orc_problem *p, const double *g_next, const double *f_next, const double *u, double *ut,
                 double tol, int maxit, orc_stats *st) {
  return momentum(p, g_next, f_next, u, NULL, ut, tol, maxit, st);
}

int orc_set_pressure_mode(orc_problem *p, int mode) {
  if (!p || mode < 0 || mode > 2) return ORC_E_ARG;
  p->pressure_mode = mode;
  return ORC_OK;
}

/* Step 2 (+ right-hand side of step 3), Eqs. (20)-(21):
 *  mode 0: U~_c = U~_f at the shared (prefix) nodes, b_c = -(rho/dt) Dbar U~_c
 *  mode 1: b_f = -(rho/dt) D_f U~_f, then b_c = P^T b_f through every level.
 * Boundary conditions are not applied here. */
int orc_restrict(const orc_problem *p, int mode, const double *ut_f, double *b_c) {
  double s = -p->rho / p->dt;
  if (mode == 0) {
    const orc_csr *P = &p->pc;
    for (int i = 0; i < P->n; i++) {
      double acc = 0.0;
      for (int k = P->rp[i]; k < P->rp[i + 1]; k++) {
        int j = P->col[k]; /* coarse node j is fine node j (Eq. 30) */
        acc += p->Dxc[k] * ut_f[2 * j] + p->Dyc[k] * ut_f[2 * j + 1];
      }
      b_c[i] = s * acc;
    }
    return ORC_OK;
  }
  if (mode != 1) return ORC_E_ARG;
  const orc_csr *P = &p->pf;
  double *b = dalloc((size_t)P->n);
  for (int i = 0; i < P->n; i++) {
    double acc = 0.0;
    for (int k = P->rp[i]; k < P->rp[i + 1]; k++) {
      int j = P->col[k];
      acc += p->Dxf[k] * ut_f[2 * j] + p->Dyf[k] * ut_f[2 * j + 1];
    }
    b[i] = s * acc;
  }
  for (int lv = p->levels; lv >= 1; lv--) {
    int nprev = p->lev[lv - 1].n, nk = p->lev[lv].n;
    double *bp = dalloc((size_t)nprev);
    for (int i = 0; i < nprev; i++) bp[i] = b[i];
    for (int m = nprev; m < nk; m++) {
      const int *par = p->lev[lv].parent + 2 * (m - nprev);
      bp[par[0]] += 0.5 * b[m];
      bp[par[1]] += 0.5 * b[m];
    }
    free(b);
    b = bp;
  }
  memcpy(b_c, b, sizeof(double) * (size_t)p->pc.n);
  free(b);
  return ORC_OK;
}

/* Step 4, Eqs. (22), (29): linear interpolation, level by level. */
void orc_prolong(const orc_problem *p, const double *pc, double *pf) {
  double *cur = dalloc((size_t)p->lev[0].n);
  memcpy(cur, pc, sizeof(double) * (size_t)p->lev[0].n);
  for (int lv = 1; lv <= p->levels; lv++) {
    int nprev = p->lev[lv - 1].n, nk = p->lev[lv].n;
    double *nx = dalloc((size_t)nk);
    for (int i = 0; i < nprev; i++) nx[i] = cur[i];
    for (int m = nprev; m < nk; m++) {
      const int *par = p->lev[lv].parent + 2 * (m - nprev);
      nx[m] = 0.5 * (cur[par[0]] + cur[par[1]]);
    }
    free(cur);
    cur = nx;
  }
  memcpy(pf, cur, sizeof(double) * (size_t)p->lev[p->levels].n);
  free(cur);
}

/* Step 3, Eq. (21) with the boundary conditions of Eqs. (13)-(14):
 * b is the restricted right-hand side; x holds the initial guess on entry. */
int orc_poisson_solve(const orc_problem *p, const double *b, double *x, double tol, int maxit, int *iters,
                      double *relres) {
  const orc_csr *P = &p->pc;
  int n = P->n;
  double *bb = dalloc((size_t)n);
  memcpy(bb, b, sizeof(double) * (size_t)n);
  if (p->n_pdir > 0) {
    for (int i = 0; i < n; i++)
      if (p->pdir[i]) { bb[i] = 0.0; x[i] = 0.0; }
  } else {
    double mean = 0.0;
    for (int i = 0; i < n; i++) mean += bb[i];
    mean /= n;
    for (int i = 0; i < n; i++) bb[i] -= mean;
  }
  int st = orc_pcg(P, p->Kc_bc, bb, x, tol, maxit, iters, relres);
  if (p->n_pdir == 0) {
    double wm = 0.0, ws = 0.0;
    for (int i = 0; i < n; i++) { wm += p->mc[i] * x[i]; ws += p->mc[i]; }
    for (int i = 0; i < n; i++) x[i] -= wm / ws;
  }
  free(bb);
  return st;
}

/* Step 5, Eq. (23): M U = M U~ - (dt/rho) G P_f, velocity data lifted as in step 1. */
int orc_correct(orc_problem *p, const double *g_next, const double *ut, const double *pf, double *u,
                   double tol, int maxit, orc_stats *st) {
  const orc_csr *P = &p->pf;
  int n = P->n;
  size_t nnz = (size_t)P->nnz;
  double *gx = dalloc((size_t)n), *gy = dalloc((size_t)n), *uc = dalloc((size_t)n), *rhs = dalloc((size_t)n);
  double *x = dalloc((size_t)n), *Mc = dalloc(nnz);
  orc_spmv(P, p->Dxf, pf, gx);
  orc_spmv(P, p->Dyf, pf, gy);
  double s = p->dt / p->rho;
  int status = ORC_OK;
  for (int c = 0; c < 2; c++) {
    const double *gp = c == 0 ? gx : gy;
    if (p->mass_mode == 1) {
      for (int i = 0; i < n; i++) u[2 * i + c] = ut[2 * i + c] - s * gp[i] / p->mlf[i];
      if (st) { st->mass_iters[c] = 0; st->mass_relres[c] = 0.0; }
      continue;
    }
    for (int i = 0; i < n; i++) uc[i] = ut[2 * i + c];
    orc_spmv(P, p->Mf, uc, rhs);
    for (int i = 0; i < n; i++) rhs[i] -= s * gp[i];
    memcpy(Mc, p->Mf, sizeof(double) * nnz);
    eliminate(P, Mc, rhs, p->vdir, g_next, c);
    for (int i = 0; i < n; i++) x[i] = p->vdir[i] ? g_next[2 * i + c] : uc[i];
    int it; double rr;
    int q = orc_pcg(P, Mc, rhs, x, tol, maxit, &it, &rr);
    if (st) { st->mass_iters[c] = it; st->mass_relres[c] = rr; }
    if (q != ORC_OK && status == ORC_OK) status = q;
    for (int i = 0; i < n; i++) u[2 * i + c] = x[i];
  }
  for (int i = 0; i < n; i++)
    if (p->vdir[i]) { u[2 * i] = g_next[2 * i]; u[2 * i + 1] = g_next[2 * i + 1]; }
  free(gx); free(gy); free(uc); free(rhs); free(x); free(Mc);
  return status;
}

static int check_finite(const double *v, size_t n) {
  for (size_t i = 0; i < n; i++)
    if (!isfinite(v[i])) return 0;
  return 1;
}

/* New coarse pressure of the incremental schemes from the restricted right-hand side b_c of step 2
 * (before boundary conditions), the increment phi and P^n (in p_c). */
int orc_pressure_update(const orc_problem *p, const double *bc, const double *phi, double *p_c) {
  if (!p || p->pressure_mode < 1) return ORC_E_ARG;
  int nc = p->lev[0].n;
  for (int i = 0; i < nc; i++) {
    double q = 0.0;
    if (p->pressure_mode == 2) /* bc = -(rho/dt) (restricted div U~); q = (restricted div U~) / m_c */
      q = -(p->dt / p->rho) * bc[i] / p->mc[i];
    p_c[i] = (p->n_pdir > 0 && p->pdir[i]) ? 0.0 : p_c[i] + phi[i] - p->mu * q;
  }
  if (p->pressure_mode == 2 && p->n_pdir == 0) {
    double wm = 0.0, ws = 0.0;
    for (int i = 0; i < nc; i++) { wm += p->mc[i] * p_c[i]; ws += p->mc[i]; }
    for (int i = 0; i < nc; i++) p_c[i] -= wm / ws;
  }
  return ORC_OK;
}

int orc_step(orc_problem *p, const double *g_next, const double *f_next, double *u, double *p_f, double *p_c,
             double tol_mom, double tol_p, double tol_mass, int maxit, int x0_prev, orc_stats *st) {
  if (!p || !p->assembled || !g_next || !u || !p_f || !p_c) return ORC_E_ARG;
  int nf = p->lev[p->levels].n, nc = p->lev[0].n;
  if (!check_finite(u, 2 * (size_t)nf) || !check_finite(g_next, 2 * (size_t)nf)) return ORC_E_NONFINITE;
  orc_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof *st);
  double *ut = dalloc(2 * (size_t)nf), *bc = dalloc((size_t)nc);
  int status, s2, s3, s5;
  if (p->pressure_mode == 0) {
    status = orc_momentum(p, g_next, f_next, u, ut, tol_mom, maxit, st);              /* step 1 */
    s2 = orc_restrict(p, p->restrict_mode, ut, bc);                                     /* step 2 */
    if (!x0_prev) memset(p_c, 0, sizeof(double) * (size_t)nc);
    s3 = orc_poisson_solve(p, bc, p_c, tol_p, maxit, &st->p_iters, &st->p_relres);     /* step 3 */
    orc_prolong(p, p_c, p_f);                                                          /* step 4 */
    s5 = orc_correct(p, g_next, ut, p_f, u, tol_mass, maxit, st);                      /* step 5 */
  } else {
    /* incremental schemes: p_c holds P^n on entry */
    double *pn = dalloc((size_t)nf), *phi = dalloc((size_t)nc), *phif = dalloc((size_t)nf);
    orc_prolong(p, p_c, pn);
    status = momentum(p, g_next, f_next, u, pn, ut, tol_mom, maxit, st);              /* step 1 */
    s2 = orc_restrict(p, p->restrict_mode, ut, bc);                                     /* step 2 */
    s3 = orc_poisson_solve(p, bc, phi, tol_p, maxit, &st->p_iters, &st->p_relres);     /* step 3: increment */
    orc_prolong(p, phi, phif);                                                         /* step 4 */
    s5 = orc_correct(p, g_next, ut, phif, u, tol_mass, maxit, st);                     /* step 5 */
    orc_pressure_update(p, bc, phi, p_c);
    orc_prolong(p, p_c, p_f);
    free(pn); free(phi); free(phif);
  }
  if (status == ORC_OK) status = s2;
  if (status == ORC_OK) status = s3;
  if (status == ORC_OK) status = s5;
  if (!check_finite(u, 2 * (size_t)nf)) status = ORC_E_NONFINITE;
  free(ut); free(bc);
  return status;
}

/* The standard (non-CGP) projection step of Eqs. (16)-(18) on the fine mesh
 * alone, written without any grid transfer.  Only meaningful when levels == 0,
 * where CGP reduces to it (Section 3, l = 0). */
int orc_projection_step(orc_problem *p, const double *g_next, const double *f_next, double *u, double *p_f,
                        double tol_mom, double tol_p, double tol_mass, int maxit, orc_stats *st) {
  if (!p || !p->assembled || p->levels != 0) return ORC_E_ARG;
  const orc_csr *P = &p->pf;
  int n = P->n;
  size_t nnz = (size_t)P->nnz;
  orc_stats local;
  if (!st) st = &local;
  memset(st, 0, sizeof *st);
  double *ut = dalloc(2 * (size_t)n), *b = dalloc((size_t)n), *K = dalloc(nnz);
  int status = orc_momentum(p, g_next, f_next, u, ut, tol_mom, maxit, st);
  /* Eq. (17): -K P = (rho/dt) D U~ */
  for (int i = 0; i < n; i++) {
    double acc = 0.0;
    for (int k = P->rp[i]; k < P->rp[i + 1]; k++)
      acc += p->Dxf[k] * ut[2 * P->col[k]] + p->Dyf[k] * ut[2 * P->col[k] + 1];
    b[i] = -p->rho / p->dt * acc;
  }
  memcpy(K, p->Kf, sizeof(double) * nnz);
  if (p->n_pdir > 0) {
    for (int i = 0; i < n; i++)
      for (int k = P->rp[i]; k < P->rp[i + 1]; k++)
        if (p->pdir[i] || p->pdir[P->col[k]]) K[k] = (P->col[k] == i) ? 1.0 : 0.0;
    for (int i = 0; i < n; i++)
      if (p->pdir[i]) b[i] = 0.0;
  } else {
    double mean = 0.0;
    for (int i = 0; i < n; i++) mean += b[i];
    mean /= n;
    for (int i = 0; i < n; i++) b[i] -= mean;
  }
  memset(p_f, 0, sizeof(double) * (size_t)n);
  int s3 = orc_pcg(P, K, b, p_f, tol_p, maxit, &st->p_iters, &st->p_relres);
  if (p->n_pdir == 0) {
    double wm = 0.0, ws = 0.0;
    for (int i = 0; i < n; i++) { wm += p->mc[i] * p_f[i]; ws += p->mc[i]; }
    for (int i = 0; i < n; i++) p_f[i] -= wm / ws;
  }
  int s5 = orc_correct(p, g_next, ut, p_f, u, tol_mass, maxit, st);
  if (status == ORC_OK) status = s3;
  if (status == ORC_OK) status = s5;
  free(ut); free(b); free(K);
  return status;
}
