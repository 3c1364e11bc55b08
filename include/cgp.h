/*
 * cgp.h - C ABI of libcgp, an MI355X (gfx950) implementation of the
 * finite-element coarse-grid projection (IFE-CGP) time step of Kashefi &
 * Staples, "A Finite-Element Coarse-Grid Projection Method" (Section 2).
 *
 * The problem statement the arguments follow (Section 2.1): density rho,
 * viscosity mu, time step dt, body force f, velocity data u_GammaD on the
 * Dirichlet boundary Gamma_D, zero traction on Gamma_N (Eqs. 1-4, 9-15); P1
 * elements for velocity and pressure (Eqs. 16-18); pressure solved on a mesh
 * coarsened l times by inverting the 1:4 subdivision (Section 2.2), resolution
 * M:N with N = 4^-l M (Section 3).
 *
 * Conventions
 *  - Every function returns cgp_status (0 = CGP_OK).  On failure a message
 *    is available from cgp_last_error() (thread-local, valid until the next
 *    call on the same thread).
 *  - Host arrays passed in are copied; the caller keeps ownership.
 *  - Device arrays are raw HIP device pointers (e.g. torch tensor
 *    data_ptr()); the caller owns them and keeps them alive until the call
 *    returns.  Velocity-like vectors are interleaved [n][2] doubles.
 *  - All device work is enqueued on the stream given to cgp_mesh_create.
 *    Calls that run Krylov iterations synchronise that stream to test
 *    convergence, so they return with their results complete.
 *  - The library owns every internal device buffer and frees it in
 *    cgp_mesh_destroy.  One mesh handle must be used by one host thread at a
 *    time; calls on different handles are independent.
 *  - Node numbering (Section 2.2, Remark 2.2): the nodes of level k keep their
 *    numbers on level k+1 and the midpoint of the r-th edge of level k, edges
 *    taken as sorted (min,max) pairs, is node N_k + r.  Coarse nodes are
 *    therefore the first N_c fine nodes, which makes the injection of Eq. (30)
 *    the identity on that prefix, and the two endpoints of an edge are the
 *    parents of its midpoint in the linear interpolation of Eq. (29).
 */
#ifndef CGP_H
#define CGP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGP_ABI_VERSION 3

typedef enum {
  CGP_OK = 0,
  CGP_E_ARG = 1,       /* null pointer, bad size, bad enum, unsupported option */
  CGP_E_MESH = 2,      /* clockwise/degenerate triangle, non-manifold edge, untagged boundary edge */
  CGP_E_NOCONV = 3,    /* Krylov solve hit max_iter; last iterate kept, stats filled */
  CGP_E_NONFINITE = 4, /* NaN/Inf in an input or a residual */
  CGP_E_DEVICE = 5,    /* HIP runtime error */
  CGP_E_OOM = 6,       /* device allocation failed */
  CGP_E_STATE = 7      /* call out of order (e.g. step before assemble, device call on a host-only mesh) */
} cgp_status;

/* boundary edge kinds (Eqs. 3-4) */
enum { CGP_EDGE_VEL_DIRICHLET = 1, /* Gamma_D: velocity given; pressure Neumann (Eq. 13) */
       CGP_EDGE_OUTFLOW = 2 };     /* Gamma_N: zero traction; pressure p = 0 (Eq. 14)   */

enum { CGP_MESH_HOST_ONLY = 1 };   /* cgp_mesh_desc.flags: build topology only, no device memory */

enum { CGP_RESTRICT_INJECT = 0,    /* Eqs. (20), (30): values at shared nodes (the paper's choice) */
       CGP_RESTRICT_GALERKIN = 1 };/* transpose of prolongation applied to the fine divergence (Section 2.2) */

enum { CGP_MASS_CONSISTENT = 0,    /* Eq. (23) solved with the consistent mass matrix */
       CGP_MASS_LUMPED = 1 };      /* Eq. (23) with the row-sum lumped mass matrix */

enum { CGP_PRESSURE_NONINCREMENTAL = 0, /* Eqs. (9)-(15), (19)-(23): the paper's scheme; p^n is not used */
       CGP_PRESSURE_INCREMENTAL = 1,    /* standard incremental correction (the extension of Remark 3.1 and the
                                           conclusions): momentum right-hand side -dt G P_f^n, Eq. (21) solved for
                                           the increment, Eq. (23) corrected with the prolonged increment,
                                           P^{n+1} = P^n + increment */
       CGP_PRESSURE_ROTATIONAL = 2 };   /* as INCREMENTAL, and P^{n+1} also gets -mu times the restricted
                                           divergence of U~ divided by the coarse lumped mass (zero on
                                           pressure-Dirichlet nodes; zero lumped-mass mean without them) */

enum { CGP_PREC_FP64 = 0,          /* all Krylov arithmetic in FP64 */
       CGP_PREC_FP32_IR = 1 };     /* Poisson: FP32 Jacobi-PCG inside FP64 iterative refinement */

enum { CGP_X0_ZERO = 0,            /* Krylov initial guess zero */
       CGP_X0_PREV = 1,            /* initial guess = the output array's current contents */
       CGP_X0_LEARNED = 2,         /* Poisson only: x0 = Phi c, c from the attached POD/MLP model */
       CGP_X0_LEARNED_CORR = 3,    /* Poisson only: x0 = x + Phi dc, dc from the incremental model and b - K x */
       CGP_X0_POD_GALERKIN = 4,    /* Poisson only: previous pressure plus the Galerkin correction in span(Phi) */
       CGP_X0_EXTRAP = 5,          /* cgp_step momentum (and mass, see cgp_step_opts) only: x0 = 3 U~^n - 3 U~^(n-1) + U~^(n-2), the quadratic
                                      extrapolation of this mesh's three previous intermediate velocities
                                      (U^n after no such step, linear 2 U~^n - U~^(n-1) after one); the solve
                                      still meets its tolerance */
       CGP_X0_PROJECT = 6 };       /* cgp_step momentum only: per velocity component, x0 = the combination of
                                      this mesh's last (up to 8) intermediate velocities from consecutive
                                      cgp_step calls in this mode that minimises ||b - A x0||_2 over the
                                      non-Dirichlet rows of the current system (normal equations, scaled to a
                                      unit diagonal, ridge 1e-13, solved on the device); U^n before the first
                                      such step.  The span holds the quadratic extrapolation, so the starting
                                      residual is never larger than that of CGP_X0_EXTRAP beyond rounding.
                                      The first use allocates 128 bytes per fine node for the history. */

enum { CGP_METHOD_DEFAULT = 0,     /* Jacobi-PCG (Poisson, mass), Jacobi-BiCGStab (momentum) */
       CGP_METHOD_ILU_GMRES = 1,    /* Poisson only: GMRES(restart) preconditioned by ILU(0) of Kbar, the paper's solver
                                       (Section 2.3); FP64; factorised on the device at the first such solve
                                       after cgp_assemble */
       CGP_METHOD_CHEBYSHEV = 2 };  /* mass solve only (step 5, consistent mass): Jacobi-preconditioned Chebyshev
                                       iteration on the bounds [1/2, 2] that hold for the P1 mass matrix on any
                                       triangulation (Wathen 1987): no inner products, one kernel per step; runs
                                       as many steps as the last solve needed, then checks the true residual
                                       against tol and continues if it must; FP64.  Refused for the momentum
                                       and Poisson solves (CGP_E_ARG) */

enum { CGP_LAUNCH_AUTO = 0,        /* library choice (FUSED for the Poisson solve) */
       CGP_LAUNCH_LOOP = 1,        /* two kernels per PCG iteration (textbook recurrences), host polls every chunk */
       CGP_LAUNCH_PERSISTENT = 2,  /* Poisson: one cooperative kernel for the whole Krylov loop */
       CGP_LAUNCH_FUSED = 3 };     /* Poisson: one kernel per PCG iteration (Chronopoulos-Gear recurrences) */

typedef struct cgp_mesh cgp_mesh;

typedef struct {
  int32_t n_nodes;            /* coarse nodes */
  const double *xy;           /* host [n_nodes][2] */
  int32_t n_tris;
  const int32_t *tri;         /* host [n_tris][3], counter-clockwise, 0-based */
  int32_t n_bedges;
  const int32_t *bedge;       /* host [n_bedges][2]: every edge used by exactly one triangle, once */
  const int32_t *bedge_kind;  /* host [n_bedges]: CGP_EDGE_* */
  int32_t levels;             /* l >= 0 subdivisions; l = 0 is the standard projection method */
  int32_t flags;              /* CGP_MESH_* */
} cgp_mesh_desc;

typedef struct {
  double rho, mu, dt;         /* density, dynamic viscosity, time step (Eqs. 5-15) */
  int32_t restrict_mode;      /* CGP_RESTRICT_* */
  int32_t mass_mode;          /* CGP_MASS_* */
  int32_t pressure_mode;      /* CGP_PRESSURE_*; the incremental modes are cgp_step-only (not cgp_batch_step) */
} cgp_params;

typedef struct {
  int32_t precision;          /* CGP_PREC_*; FP32_IR: the Poisson solve (FP32 Jacobi-PCG) and the momentum
                                 solve (FP32 Jacobi-BiCGStab on both components, inner_tol 0 = 1e-5)
                                 inside FP64 iterative refinement; the mass solve is FP64 only */
  double tol;                 /* stop when ||b - A x||_2 <= tol ||b||_2 (unpreconditioned) */
  int32_t max_iter;           /* Krylov iterations (inner iterations summed for FP32_IR) */
  double inner_tol;           /* FP32_IR: relative reduction asked of each inner FP32 solve; an inner
                                 solve asks for less (half the reduction the outer tolerance still needs)
                                 when that is enough, except under CGP_LAUNCH_PERSISTENT */
  int32_t x0_mode;            /* CGP_X0_* */
  int32_t launch;             /* CGP_LAUNCH_* (the default method only) */
  int32_t method;             /* CGP_METHOD_* */
  int32_t restart;            /* CGP_METHOD_ILU_GMRES: Krylov vectors per cycle, 1..200 (0 = 30) */
} cgp_solver_opts;

typedef struct {
  cgp_solver_opts momentum;   /* step 1, Eq. (19): Jacobi-BiCGStab, both components together */
  cgp_solver_opts poisson;    /* step 3, Eq. (21): Jacobi-PCG on the coarse mesh */
  cgp_solver_opts mass;       /* step 5, Eq. (23): Jacobi-PCG with the consistent mass matrix, started
                                 from the lumped-mass correction (from 0 when x0_mode = CGP_X0_ZERO; with
                                 CGP_X0_EXTRAP, from the lumped correction plus the previous cgp_step's
                                 consistent-minus-lumped difference, kept per mesh, 16 bytes a fine node
                                 allocated at first use) */
  int32_t timing;             /* 1: per-phase HIP-event times in cgp_stats; 2: also bracket every launch of
                                 the Poisson Krylov kernel with HIP events (slows the step; for measurement) */
} cgp_step_opts;

typedef struct {
  int32_t mom_iters, p_iters, p_outer, mass_iters;
  double mom_relres, p_relres, mass_relres;   /* max over components */
  float ms_assemble, ms_momentum, ms_restrict, ms_poisson, ms_prolong, ms_correct;
  double ms_dominant;         /* timing == 2: summed duration of the Poisson Krylov kernel launches (the SpMV
                                 kernel of the launch-per-phase loop, or the persistent kernel) */
  int32_t n_dominant;         /* timing == 2: number of those launches */
  int32_t dominant_iters;     /* timing == 2: Krylov iterations those launches performed */
} cgp_stats;

typedef struct {
  int64_t n_f, t_f, n_c, t_c, nnz_f, nnz_c, ncol_f, ncol_c, nb_f, nb_c, levels, n_pdir;
} cgp_mesh_info;

/* cgp_mesh_export selectors.  Topology (int32 unless noted, host copies): */
enum {
  CGP_X_XY = 0,          /* double [n][2] of the given level */
  CGP_X_TRI = 1,         /* [t][3] of the given level, subdivision order (children of t are 4t..4t+3) */
  CGP_X_BEDGE = 2,       /* [nb][2]; a tagged edge (a,b) becomes (a,m),(m,b) */
  CGP_X_BKIND = 3,       /* [nb] */
  CGP_X_PARENT = 4,      /* [n_k - n_{k-1}][2] interpolation parents of level k >= 1 (Eq. 29) */
  CGP_X_EDGES = 5,       /* [ne][2] sorted unique edges of the level */
  CGP_X_ROWPTR_F = 6, CGP_X_COL_F = 7, CGP_X_SLOT_F = 8, CGP_X_COLOUR_F = 9,
  CGP_X_ROWPTR_C = 10, CGP_X_COL_C = 11, CGP_X_SLOT_C = 12, CGP_X_COLOUR_C = 13,
  CGP_X_VDIR = 14,       /* [n_f] velocity-Dirichlet node mask (0/1) */
  CGP_X_PDIR = 15,       /* [n_c] pressure-Dirichlet node mask (0/1) */
  CGP_X_SIZES = 16,      /* int32[4]: n, t, nb, ne of the level */
  /* assembled values, copied from the device after cgp_assemble (double): */
  CGP_X_S_F = 20,        /* rho M + dt mu K on the fine pattern */
  CGP_X_M_F = 21, CGP_X_DX_F = 22, CGP_X_DY_F = 23,
  CGP_X_K_C = 24,        /* coarse stiffness, no boundary conditions */
  CGP_X_KBC_C = 25,      /* coarse stiffness with p = 0 rows/columns eliminated */
  CGP_X_DX_C = 26, CGP_X_DY_C = 27,
  CGP_X_MC = 28,         /* coarse lumped mass [n_c] */
  CGP_X_A_F = 29,        /* momentum matrix of the last step, after Dirichlet elimination */
  CGP_X_ML_F = 30,       /* fine lumped mass [n_f] */
  CGP_X_ILU_C = 31       /* ILU(0) factors of the coarse Poisson matrix on its pattern [nnz_c] (unit L below the
                            diagonal, U on and above), after the first CGP_METHOD_ILU_GMRES solve */
};

/* operators for cgp_spmv */
enum { CGP_OP_KBC_C = 0,   /* y[n_c]   = Kbar_bc x           (FP64) */
       CGP_OP_M_F = 1,     /* y[n_f][2] = M_f x, both columns  (FP64) */
       CGP_OP_A_F = 2,     /* y[n_f][2] = A x, momentum matrix of the last step */
       CGP_OP_KBC_C32 = 3  /* float y[n_c] = Kbar_bc x in FP32 (after cgp_assemble) */ };

/* Launch shape of the Krylov kernels on one mesh level (set by hand or by the autotuner). */
typedef struct {
  int32_t lanes;   /* threads per CSR row in SpMV-type kernels: 2, 4, 8 or 16 */
  int32_t block;   /* threads per block of the Krylov kernels: 64, 128, 256, 512 or 1024 */
  int32_t passes;  /* rows (SpMV-type kernels) or entries (vector kernels) per lane group: 1..64 */
} cgp_tuning_knobs;

typedef struct {
  cgp_tuning_knobs fine;    /* momentum and mass solves */
  cgp_tuning_knobs coarse;  /* pressure Poisson solve */
  int32_t pcg_barrier;      /* persistent Poisson kernel: 0 = library grid barrier, 1 = HIP cooperative-groups sync */
  int32_t pcg_grid;         /* persistent Poisson kernel: blocks of 1024 threads, 0 = one per compute unit (the
                               default); at most one per compute unit (256 on a host-only mesh), since a grid of
                               two blocks per CU was not all resident and never passed its first barrier */
  int32_t pcg_spin_log2;    /* persistent Poisson kernel: a grid-barrier wait gives up after 2^pcg_spin_log2 polls
                               and the solve returns CGP_E_DEVICE (0 = 2^24; 1..30) */
  int32_t pcg_graph;        /* fused Poisson PCG: 1 = runs of 8 iterations go out as one launch of a captured HIP
                               graph (kept per buffer set, at most 8 sets per mesh); 0 (the default) = every
                               iteration its own launch, which measured faster on gfx950 (10.4 against 10.9 us
                               per FP64 iteration at 125k rows).  Ignored while kernel events are timed. */
} cgp_tuning;

int32_t cgp_abi_version(void);
const char *cgp_last_error(void);

/* Validate the coarse mesh (CCW, manifold, every boundary edge tagged),
 * subdivide it `levels` times, build numbering, parents, CSR patterns (sorted
 * columns, diagonal included), slot maps, element colourings and boundary
 * masks, and upload them.  hip_stream: hipStream_t (NULL = default stream). */
cgp_status cgp_mesh_create(const cgp_mesh_desc *desc, void *hip_stream, cgp_mesh **out);
cgp_status cgp_mesh_query(const cgp_mesh *mesh, cgp_mesh_info *out);
/* Copy a topology array or an assembled operator into host memory; bytes must equal its size. */
cgp_status cgp_mesh_export(const cgp_mesh *mesh, int32_t what, int32_t level, void *host_dst, size_t bytes);
void cgp_mesh_destroy(cgp_mesh *mesh);

/* Assemble the step-independent operators (Eqs. 16-18, Section 2.2):
 * fine rho M + dt mu K, M, (Dx, Dy); coarse Kbar and (Dbar_x, Dbar_y) from
 * coarse shape functions, coarse lumped mass, pressure-Dirichlet elimination,
 * Jacobi diagonals.  Element contributions are added colour by colour. */
cgp_status cgp_assemble(cgp_mesh *mesh, const cgp_params *params);

/* One IFE-CGP step n -> n+1 (Eqs. 19-23):
 *   g_next   dev [n_f][2]  velocity data at t^{n+1}; read at velocity-Dirichlet nodes only
 *   f_next   dev [n_f][2]  body force F^{n+1}, or NULL for F = 0
 *   u        dev [n_f][2]  in: U^n, out: U^{n+1}
 *   p_fine   dev [n_f]     out: P_f^{n+1} (prolonged pressure)
 *   p_coarse dev [n_c]     in: initial guess when poisson.x0_mode = CGP_X0_PREV (incremental pressure
 *                          modes: P_c^n, required; the increment's solve then starts from the previous
 *                          increment, kept by the library, under CGP_X0_PREV), out: P_c^{n+1}
 *   stats    host or NULL
 * Returns CGP_E_NOCONV if a solve hits its iteration limit (the step is still
 * completed with the last iterates), CGP_E_NONFINITE on NaN/Inf residuals. */
cgp_status cgp_step(cgp_mesh *mesh, const cgp_step_opts *opts, const double *g_next, const double *f_next,
                    double *u, double *p_fine, double *p_coarse, cgp_stats *stats);

/* The five steps one at a time (same arguments and layouts as cgp_step). */
cgp_status cgp_momentum(cgp_mesh *mesh, const cgp_solver_opts *opts, const double *g_next, const double *f_next,
                        const double *u, double *u_tilde, cgp_stats *stats);                 /* Eq. (19) */
cgp_status cgp_restrict(cgp_mesh *mesh, const double *u_tilde, double *b_coarse);            /* Eqs. (20)-(21) rhs, no BCs */
cgp_status cgp_poisson_solve(cgp_mesh *mesh, const double *b_coarse, double *x, const cgp_solver_opts *opts,
                             cgp_stats *stats);                                             /* Eq. (21), BCs applied */
cgp_status cgp_prolong(cgp_mesh *mesh, const double *p_coarse, double *p_fine);              /* Eq. (22) */
cgp_status cgp_correct(cgp_mesh *mesh, const cgp_solver_opts *opts, const double *g_next, const double *u_tilde,
                       const double *p_fine, double *u, cgp_stats *stats);                  /* Eq. (23) */

/* ---- learned initial guess (Poisson x0): a POD basis of pressure snapshots, M_c-orthonormal, and
 * an MLP n_modes -> hidden -> hidden -> n_modes (GELU) from the normalised modal projection of the
 * Poisson right-hand side to the normalised modal coefficients of the pressure.  GEMMs run in BF16
 * with FP32 accumulation on the matrix cores; basis projections are FP64.  PCG still converges to
 * the requested tolerance whatever the guess. */
typedef struct cgp_guess cgp_guess;
typedef struct { int32_t n_modes; int32_t hidden; uint64_t seed; } cgp_guess_desc;   /* n_modes <= 64 */
/* p_prev = NULL: the network maps Phi^T b to the modal coefficients Phi^T M p of the pressure (serves
 * CGP_X0_LEARNED).  p_prev = device [S][n_c], the previous-step pressure of each sample: the network maps
 * Phi^T (b - K p_prev) to Phi^T M (p - p_prev) (an incremental model, serves CGP_X0_LEARNED_CORR). */
typedef struct { int32_t epochs; int32_t batch; double lr, beta1, beta2, eps; uint64_t seed; const double *p_prev; }
    cgp_train_opts;
typedef struct { double loss_first, loss_last; int32_t steps; float ms; } cgp_train_stats;

cgp_status cgp_guess_create(cgp_mesh *mesh, const cgp_guess_desc *desc, cgp_guess **out);
void cgp_guess_destroy(cgp_guess *g);
/* Basis from snapshots (device [S][n_c], rows = snapshots): eigenvectors of S M_c S^T for the n_modes
 * eigenvalues largest in magnitude (randomised subspace iteration on the host when S > n_modes + 16,
 * else the whole S x S Gram matrix; Householder tridiagonalisation and shifted QR),
 * Phi = S^T V |Lambda|^-1/2.  Modes below 1e-20 of the largest magnitude are left out (zero columns,
 * energy 0); a rounding-level eigenvalue that comes out negative keeps its mode.
 * energy: host [n_modes] |eigenvalues| or NULL.  CGP_E_NOCONV if the QR iteration does not converge. */
cgp_status cgp_guess_build_pod(cgp_guess *g, const double *snaps, int32_t S, double *energy);
/* Train on S (2..65536) samples: device [S][n_c] right-hand sides after boundary conditions and the
 * [S][n_c] pressures solving them.  Mini-batch Adam on FP32 master weights; the basis must be built
 * first. */
cgp_status cgp_guess_train(cgp_guess *g, const double *rhs, const double *p, int32_t S, const cgp_train_opts *opts,
                           cgp_train_stats *stats);
/* Online basis: while the guess is attached, every converged Poisson solve of the mesh keeps its solution
 * in a window of the last `window` solutions (device memory owned by the guess), and every `refresh`
 * solves the basis is rebuilt from the window (as cgp_guess_build_pod).  The basis then spans recent
 * pressures, including the components the solver converges on slowest, so that CGP_X0_POD_GALERKIN acts
 * as a recycled Krylov subspace; until the window holds n_modes solutions that mode keeps the previous
 * pressure.  A rebuilt basis invalidates a trained network.  window = 0 turns it off; otherwise
 * n_modes <= window <= 1024 and refresh >= 1.  Synchronises the mesh stream at each rebuild. */
cgp_status cgp_guess_set_online(cgp_guess *g, int32_t window, int32_t refresh);
/* Enable CGP_X0_LEARNED / _CORR / POD_GALERKIN on the mesh's Poisson solve (NULL detaches). */
cgp_status cgp_guess_attach(cgp_mesh *mesh, cgp_guess *g);
/* x0 (device [n_c]) for right-hand side b (device [n_c]); x holds the previous pressure for _CORR/_GALERKIN. */
cgp_status cgp_guess_predict(cgp_guess *g, int32_t mode, const double *b, double *x);
/* Parameters (host FP32, layout [W1 h*m | b1 h | W2 h*h | b2 h | W3 m*h | b3 m], W row-major [out][in]). */
cgp_status cgp_guess_get_params(const cgp_guess *g, float *host, size_t count);
cgp_status cgp_guess_set_params(cgp_guess *g, const float *host, size_t count);
/* One forward/backward pass on a given batch (host, already normalised): x [B][m], t [B][m];
 * returns the MSE loss, outputs y [B][m] and parameter gradients (host, layout as above). */
cgp_status cgp_guess_mlp_grad(cgp_guess *g, const float *x, const float *t, int32_t B, double *loss, float *y,
                              float *grad);
/* Basis export (host [n_c][n_modes]) */
cgp_status cgp_guess_export_basis(const cgp_guess *g, double *host, size_t count);
/* Normalisation of the trained model (host [4][n_modes]): feature mean, feature scale, target mean,
 * target scale.  Features enter the network as bf16((a - mean) / scale); coefficients leave it as
 * y * scale + mean.  CGP_E_STATE before training. */
cgp_status cgp_guess_export_norm(const cgp_guess *g, double *host, size_t count);
/* Copy the right-hand side of the last Poisson solve, after boundary conditions (device [n_c]). */
cgp_status cgp_last_poisson_rhs(const cgp_mesh *mesh, double *dst);

/* ---- many independent simulations on one GPU.  A batch holds meshes that share one stream and have
 * been assembled (their coarse operators are copied at creation: re-assembling a mesh needs a new
 * batch).  The coarse Poisson solves (Eq. 21) of all instances run as one Jacobi-PCG over the
 * concatenated block-diagonal system, one kernel launch per iteration for all instances, each instance
 * with its own scalars and convergence test; chunks of `chunk` iterations are captured into HIP graphs
 * (use_graph = 1) and replayed, with one poll per chunk.  The other phases of cgp_batch_step run per
 * instance as in cgp_step, on up to 4 streams of the batch driven from as many host threads (each
 * mesh runs on one of them for the phase; the meshes' stream waits for all of them afterwards), so
 * the meshes must not be used elsewhere during the call.  Pointer arrays are host arrays of n
 * device pointers. */
typedef struct cgp_batch cgp_batch;
/* ahead = 1 or 2 selects the iteration kernel that issues a tile's loads before the instance's scalars
 * are formed (lanes 4 or 8, passes 1, 2 or 4, or 8 with 8 lanes; 2: the columns of all of a lane group's rows before its
 * first gather); ahead = 0 the row loop. */
typedef struct { int32_t lanes, block, passes, use_graph, chunk, ahead; } cgp_batch_tuning;
cgp_status cgp_batch_create(cgp_mesh *const *meshes, int32_t n, cgp_batch **out);
void cgp_batch_destroy(cgp_batch *batch);
/* rhs[i], x[i]: instance i's coarse right-hand side and solution (x: initial guess when x0_mode =
 * CGP_X0_PREV, base of the guess for the learned and POD-Galerkin modes).  precision CGP_PREC_FP64,
 * or CGP_PREC_FP32_IR: every instance's FP32 inner solves run batched inside its own FP64 iterative
 * refinement (p_iters = inner iterations, p_outer = residual checks; graphs are not used).  With
 * x0_mode >= CGP_X0_LEARNED every mesh forms its initial guess from its own attached model or online
 * basis (cgp_guess_attach; CGP_E_STATE as in cgp_poisson_solve when one is missing), and a mesh with
 * an online window records its converged solution.  stats: host [n] or NULL (p_iters, p_relres per
 * instance; n_dominant = iteration launches).  CGP_E_NOCONV when max_iter launches pass before every
 * instance converged. */
cgp_status cgp_batch_poisson_solve(cgp_batch *batch, const double *const *rhs, double *const *x,
                                   const cgp_solver_opts *opts, cgp_stats *stats);
/* One IFE-CGP step of every instance (arguments as cgp_step, one pointer per instance; f may be NULL).
 * With opts->timing >= 1 every instance's ms_momentum, ms_poisson and ms_correct hold the batch's host
 * wall time of that phase for all instances (momentum with restriction, the batched Poisson solve,
 * prolongation with correction). */
cgp_status cgp_batch_step(cgp_batch *batch, const cgp_step_opts *opts, const double *const *g,
                          const double *const *f, double *const *u, double *const *p_fine, double *const *p_coarse,
                          cgp_stats *stats);
cgp_status cgp_batch_get_tuning(const cgp_batch *batch, cgp_batch_tuning *out);
/* lanes 2/4/8/16 per row, block a power of two in 64..1024, passes 1..64, chunk even in 2..256, ahead 0/1/2. */
cgp_status cgp_batch_set_tuning(cgp_batch *batch, const cgp_batch_tuning *tuning);
/* Time 69 launch shapes on the batch's own system and keep the fastest; the choice is cached in the JSON
 * file cache_path (NULL: no cache) under the batch's size class and reused without timing. */
cgp_status cgp_batch_autotune(cgp_batch *batch, const char *cache_path, cgp_batch_tuning *chosen);

/* ---- flow functionals: the force of the fluid on a marked part of the boundary, for drag and lift on
 * the body (Section 3.3, Eq. 42 and Table 6; their pressure and viscous parts, Fig. 13) and for the
 * wall shear stress that locates the reattachment point behind the step (Section 3.2, Fig. 7).
 * Each fine boundary edge e = (a, b) of the surface, with n its unit normal pointing into the fluid
 * and the stress -p I + mu (grad u + grad u^T) of the P1 fields (pressure linear along e, velocity
 * gradient constant on e's triangle), contributes -|e| (p_a + p_b)/2 n (pressure part) and
 * |e| mu (grad u + grad u^T) n (viscous part). */
/* Mark the surface by coarse boundary-edge indices (into cgp_mesh_desc.bedge; their children on
 * every finer level inherit the mark).  count = 0 clears it.  Allocates on first use or growth. */
cgp_status cgp_surface_set(cgp_mesh *mesh, int32_t count, const int32_t *coarse_bedge_ids);
/* Per fine edge of the surface, rows of 8 doubles (dev [n_rows][8]): midpoint x, y, length, pressure
 * force x, y, viscous force x, y, 0.  u dev [n_f][2], p_fine dev [n_f]; rows NULL only returns n_rows. */
cgp_status cgp_surface_traction(cgp_mesh *mesh, const double *u, const double *p_fine, double *rows,
                                int32_t *n_rows);
/* Totals over the surface, host out[4]: pressure force x, y, viscous force x, y (zeros if none is
 * marked).  Synchronises the mesh stream. */
cgp_status cgp_surface_force(cgp_mesh *mesh, const double *u, const double *p_fine, double *out);

/* Read or replace the Krylov launch shapes of a mesh (results do not depend on them beyond
 * rounding order).  Invalid knobs return CGP_E_ARG and leave the mesh unchanged. */
cgp_status cgp_mesh_get_tuning(const cgp_mesh *mesh, cgp_tuning *out);
cgp_status cgp_mesh_set_tuning(cgp_mesh *mesh, const cgp_tuning *tuning);

/* y = op x on device vectors (layouts listed with CGP_OP_*). */
cgp_status cgp_spmv(cgp_mesh *mesh, int32_t op, const void *x, void *y);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): cgp_poisson_solve without any allocation.  Same arguments and
 * results as cgp_poisson_solve (FP64 fused PCG; x0_mode CGP_X0_ZERO or CGP_X0_PREV; launch AUTO or
 * FUSED; anything else is CGP_E_ARG).  The solve's working memory (right-hand side with boundary
 * conditions, search direction, node records, partial sums, solver state) is one fixed device array of
 * about 21 MB per GPU, held from the first cgp_mesh_create on that GPU until the process ends, instead
 * of the mesh's buffers; coarse systems above 262144 rows are CGP_E_ARG.  Every call on one GPU uses
 * the same array: calls that overlap on one GPU (other threads, other streams) race and must not be
 * issued.  The mesh's attached learned guess is not used or updated.  Synchronises the mesh stream. */
cgp_status cgp_poisson_solve_noalloc(cgp_mesh *mesh, const double *b, double *x, const cgp_solver_opts *opts,
                                     cgp_stats *stats);

#ifdef __cplusplus
}
#endif
#endif
