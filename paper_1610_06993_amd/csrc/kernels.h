// Device-side reduction scratch and the host drivers that enqueue libcgp's kernels.
#pragma once

#include <type_traits>

#include "internal.h"

namespace cgp {

constexpr int kMaxGrid = 2048;        // cap on blocks of non-reducing row kernels (grid-stride loops)
constexpr int kMaxRedGrid = 8192;     // cap on blocks of reducing kernels (one partial each)

// projected momentum guess (CGP_X0_PROJECT): ring of the last kProj momentum solutions; per
// component the Gram matrix's upper triangle (kProjTri entries) and kProj right-hand-side entries;
// ridge added to the unit-diagonal scaled Gram matrix; blocks of the Gram kernel
constexpr int kProj = 8;
constexpr int kProjTri = kProj * (kProj + 1) / 2;
constexpr int kProjPer = kProjTri + kProj;
constexpr double kProjRidge = 1e-13;
constexpr int kProjGrid = 1024;

// Launch shape of a reducing kernel: `lanes` threads per CSR row (row kernels),
// `block` threads per block, each lane group covering `passes` rows.
struct Shape {
  int grid, block;
};
inline Shape shape_rows(const cgp_tuning_knobs &t, long long n, int lanes) {
  long long per_block = (long long)t.block * t.passes / lanes;
  long long g = (n + per_block - 1) / per_block;
  g = g < 8 ? 8 : (g + 7) / 8 * 8;
  return Shape{int(g < kMaxRedGrid ? g : kMaxRedGrid), t.block};
}

inline int grid_for(long long threads) {
  long long b = (threads + 255) / 256;
  b = b < 8 ? 8 : (b + 7) / 8 * 8;
  return int(b < kMaxGrid ? b : kMaxGrid);
}
inline int blocks_1d(long long n) { return int(n < 1 ? 1 : (n + 255) / 256); }

// run f with std::integral_constant<int, L> for the supported lanes-per-row values
template <typename F>
void dispatch_L(int L, F &&f) {
  switch (L) {
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
  }
}

// with `device` current: the device address of the allocation-free solve's array (once per device)
cgp_status noalloc_setup(int device);

// ILU(0)-GMRES(m) of the coarse Poisson equation (gmres.hip): b with boundary conditions, x the guess
cgp_status gmres_solve(cgp_mesh *m, const double *b, double *x, const cgp_solver_opts *o, KrylovState *fin);

// drivers (implemented in kernels.hip); all enqueue on mesh->stream
cgp_status drv_assemble(cgp_mesh *m);
// pn: prolonged previous pressure P_f^n (incremental pressure modes: the right-hand side gets -dt G P_f^n) or NULL
cgp_status drv_momentum(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *f, const double *u,
                        double *ut, cgp_stats *st, const double *pn = nullptr);
cgp_status drv_restrict(cgp_mesh *m, const double *ut, double *bc);
cgp_status drv_poisson(cgp_mesh *m, const double *b, double *x, const cgp_solver_opts *o, cgp_stats *st);
cgp_status drv_prolong(cgp_mesh *m, const double *pc, double *pf);
cgp_status drv_correct(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *ut, const double *pf,
                       double *u, cgp_stats *st);
cgp_status drv_spmv(cgp_mesh *m, int op, const void *x, void *y);

// launchers of kernels.hip used by the Krylov drivers (enqueue only)
void launch_conv_assembly(cgp_mesh *m, const double *u);  // d_A = S + dt N(u), every entry
void launch_mom_rhs(cgp_mesh *m, const double *g, const double *u, const double *f, const double *pn, double *rhs);
// forces on the marked surface: per-edge rows (or NULL) and the four totals into d_scalar[0..3]
void launch_surface(cgp_mesh *m, const double *u, const double *p, double *rows);
// incremental pressure modes: pc <- pc + phi (- mu dt/rho ... rotational term), pressure-Dirichlet nodes 0
void launch_pressure_update(cgp_mesh *m, double *pc, const double *phi, const double *bc);
void launch_correct_rhs(cgp_mesh *m, const double *g, const double *ut, const double *pf, double *rhs);
void launch_correct_lumped(cgp_mesh *m, const double *g, const double *ut, const double *pf, double *u);
void launch_set_dirichlet(cgp_mesh *m, const double *g, double *u);
void launch_pdir_zero(cgp_mesh *m, double *b, double *x);
// a <- 2 a - b and b <- a (old), element-wise
void launch_extrapolate(cgp_mesh *m, long count, double *a, double *b);
void launch_extrapolate3(cgp_mesh *m, long count, double *a, double *b, double *c);
// x -= (sum_i w_i x_i) / den over the coarse vector (w = NULL: plain sum); P: partial scratch
void launch_mean_shift(cgp_mesh *m, double *x, const double *w, double den, double *P);

}  // namespace cgp
