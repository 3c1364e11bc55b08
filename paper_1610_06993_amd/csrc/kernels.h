// Device-side reduction scratch and the host drivers that enqueue libcgp's kernels.
#pragma once

#include "internal.h"

namespace cgp {

struct Reduce {
  double *partials;   // [K][gridDim.x] block partials
  unsigned *counter;  // blocks finished; reset to 0 by the last block
};

constexpr int kMaxGrid = 2048;        // cap on blocks of reducing kernels (grid-stride loops)
constexpr int kPartials = 8 * 4096;   // doubles in the partials buffer

// drivers (implemented in kernels.hip); all enqueue on mesh->stream
cgp_status drv_assemble(cgp_mesh *m);
cgp_status drv_momentum(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *f, const double *u,
                        double *ut, cgp_stats *st);
cgp_status drv_restrict(cgp_mesh *m, const double *ut, double *bc);
cgp_status drv_poisson(cgp_mesh *m, const double *b, double *x, const cgp_solver_opts *o, cgp_stats *st);
cgp_status drv_prolong(cgp_mesh *m, const double *pc, double *pf);
cgp_status drv_correct(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *ut, const double *pf,
                       double *u, cgp_stats *st);
cgp_status drv_spmv(cgp_mesh *m, int op, const void *x, void *y);
cgp_status drv_check_finite(cgp_mesh *m, const double *x, size_t n, bool *finite);

}  // namespace cgp
