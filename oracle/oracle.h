/*
 * Plain FP64 CPU oracle for the finite-element coarse-grid projection (IFE-CGP)
 * time step of Kashefi & Staples, "A Finite-Element Coarse-Grid Projection
 * Method" (Sections 2.1-2.2, Eqs. 16-23; Remark 2.2, Eqs. 29-30).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the reference the GPU path is checked against: only
 * the test suite, the package smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header or table with the GPU library, and
 * is written to be read against the paper, not to be fast: element loops in
 * natural order, textbook Krylov iterations, binary searches for CSR slots.
 *
 * Conventions (all arrays row-major, 0-based, caller-owned unless stated):
 *   xy[n][2] double, tri[t][3] int (counter-clockwise), bedge[nb][2] int,
 *   bkind[nb] int (1 = velocity Dirichlet edge, 2 = zero-traction outflow).
 *   Velocity vectors are interleaved [n][2].
 * Status codes: 0 ok, 1 bad argument, 2 invalid mesh, 3 no convergence,
 *   4 non-finite value.
 */
#ifndef CGP_ORACLE_H
#define CGP_ORACLE_H

#include <stdint.h>

#define ORC_MAXLEV 6
#define ORC_OK 0
#define ORC_E_ARG 1
#define ORC_E_MESH 2
#define ORC_E_NOCONV 3
#define ORC_E_NONFINITE 4

#define ORC_EDGE_VEL 1
#define ORC_EDGE_OUT 2

typedef struct {
  int n, t, nb;      /* nodes, triangles, boundary edges */
  double *xy;        /* [n][2] */
  int *tri;          /* [t][3] */
  int *bedge;        /* [nb][2] */
  int *bkind;        /* [nb] */
  int ne;            /* unique edges of this level */
  int *edge;         /* [ne][2], (min,max), lexicographically sorted */
  int *parent;       /* [n - n_prev][2] endpoints of each midpoint (NULL on level 0) */
} orc_level;

typedef struct {       /* compressed sparse row pattern + values */
  int n, nnz;
  int *rp, *col;
} orc_csr;

typedef struct {
  int levels;                  /* number of 1:4 subdivisions l */
  orc_level lev[ORC_MAXLEV + 1];
  orc_csr pf, pc;              /* fine (level l) and coarse (level 0) patterns */
  int *colour_f, ncol_f;       /* element colours (S4) of the fine and coarse meshes */
  int *colour_c, ncol_c;
  unsigned char *vdir;         /* [n_f] velocity-Dirichlet node mask */
  unsigned char *pdir;         /* [n_c] pressure-Dirichlet node mask (coarse) */
  int n_pdir;
  /* physical parameters and modes */
  double rho, mu, dt;
  int restrict_mode;           /* 0 inject (Eq. 20/30), 1 transpose of prolongation */
  int mass_mode;               /* 0 consistent mass in Eq. 23, 1 lumped */
  int pressure_mode;           /* 0 non-incremental (Eqs. 9-15), 1 standard incremental, 2 rotational */
  int assembled;
  /* fine operators, values on pf */
  double *Mf, *Kf, *Dxf, *Dyf, *mlf;
  /* coarse operators, values on pc */
  double *Kc, *Kc_bc, *Dxc, *Dyc, *mc;
} orc_problem;

typedef struct {
  int mom_iters[2], p_iters, mass_iters[2];
  double mom_relres[2], p_relres, mass_relres[2];
} orc_stats;

/* ---- mesh (S1-S5) */
int orc_check_mesh(int n, const double *xy, int t, const int *tri, int nb, const int *bedge, const int *bkind);
orc_problem *orc_create(int n, const double *xy, int t, const int *tri, int nb, const int *bedge,
                        const int *bkind, int levels, int *status);
void orc_free(orc_problem *p);
void orc_info(const orc_problem *p, int64_t *out); /* 12 entries, see oracle/mesh.c */
int orc_export(const orc_problem *p, int what, int level, void *dst);
uint64_t orc_priority(uint64_t t);

/* ---- element operators and assembly (S6) */
void orc_element(const double *xy3, const double *u3, double rho, double *M, double *K, double *Dx,
                 double *Dy, double *N);
int orc_assemble(orc_problem *p, double rho, double mu, double dt, int restrict_mode, int mass_mode);
int orc_export_values(const orc_problem *p, int what, double *dst);

/* ---- Krylov and direct solvers */
int orc_pcg(const orc_csr *A, const double *val, const double *b, double *x, double tol, int maxit,
            int *iters, double *relres);
int orc_bicgstab(const orc_csr *A, const double *val, const double *b, double *x, double tol, int maxit,
                 int *iters, double *relres);
int orc_dense_solve(int n, double *A, double *b, double *x);
void orc_spmv(const orc_csr *A, const double *val, const double *x, double *y);

/* ---- the CGP step (S7) and its pieces */
int orc_restrict(const orc_problem *p, int mode, const double *ut_f, double *b_c);
void orc_prolong(const orc_problem *p, const double *pc, double *pf);
int orc_poisson_solve(const orc_problem *p, const double *b, double *x, double tol, int maxit,
                      int *iters, double *relres);
int orc_step(orc_problem *p, const double *g_next, const double *f_next, double *u, double *p_f,
             double *p_c, double tol_mom, double tol_p, double tol_mass, int maxit, int x0_prev,
             orc_stats *st);
int orc_projection_step(orc_problem *p, const double *g_next, const double *f_next, double *u,
                        double *p_f, double tol_mom, double tol_p, double tol_mass, int maxit,
                        orc_stats *st);
int orc_momentum(orc_problem *p, const double *g_next, const double *f_next, const double *u, double *ut,
                 double tol, int maxit, orc_stats *st);
int orc_set_pressure_mode(orc_problem *p, int mode);
int orc_pressure_update(const orc_problem *p, const double *bc, const double *phi, double *p_c);
int orc_correct(orc_problem *p, const double *g_next, const double *ut, const double *pf, double *u, double tol,
                int maxit, orc_stats *st);
/* values of the convection matrix N(u) of Eq. (16) (rho included) on the fine CSR pattern */
void orc_convection(const orc_problem *p, const double *u, double *Nval);

/* ---- learned guess network (oracle/learn.c) */
double orc_bf16(double x);
double orc_gelu(double z);
double orc_gelu_grad(double z);
void orc_mlp_forward_backward(int m, int h, int B, const float *params, const float *X, const float *T, int emulate,
                              double *loss, double *Y, double *grad);
void orc_adam(int n, double *w, const double *g, double *m1, double *m2, int t, double lr, double b1, double b2,
              double eps);

/* ---- POD of snapshots (oracle/pod.c) */
void orc_jacobi_eigen(int q, double *A, double *V);
int orc_pod(int S, int n, const double *snaps, const double *w, int m, double *phi, double *energy);

/* ---- the paper's error norms, Eqs. (31)-(33) (oracle/norms.c) */
int orc_quad_npts(void);
int orc_quad_points(const orc_problem *p, int level, double *xyq);
int orc_error_norms(const orc_problem *p, int level, int nc, const double *A, const double *aq, const double *an,
                    double *l2, double *linf);

/* ---- the paper's solver: ILU(0)-preconditioned GMRES(m) (oracle/gmres.c) */
int orc_ilu0(const orc_csr *A, const double *val, double *lu);
void orc_ilu0_apply(const orc_csr *A, const double *lu, const double *r, double *z);
int orc_gmres(const orc_csr *A, const double *val, const double *lu, const double *b, double *x, int m, double tol,
              int maxit, int orth, int *iters, double *relres);

/* ---- forces on a marked boundary (oracle/forces.c) */
int orc_surface_traction(const orc_problem *p, const int *mark, const double *u, const double *pf, double *out,
                         int cap);
int orc_surface_force(const orc_problem *p, const int *mark, const double *u, const double *pf, double *out);

#endif
