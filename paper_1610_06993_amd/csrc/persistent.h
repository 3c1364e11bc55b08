// Persistent (cooperative) Jacobi-PCG for the coarse Poisson solve.
#pragma once

#include "internal.h"

namespace cgp {

struct PersistArgs {
  const int *rp, *col;
  const void *val, *dinv;     // T (double or float)
  const void *b;              // T right-hand side (FP64 solve)
  const double *b64;          // FP64 residual whose normalised copy is the inner right-hand side (FP32 solve)
  void *x, *r, *z, *p0, *p1, *q;
  const int *row_begin;       // [grid + 1] row range owned by each block
  double *partials;           // [2][4][grid]
  void *bar;                  // grid barrier state
  KrylovState *state;         // result: iterations, norms, status
  const KrylovState *outer;   // FP32 solve: the refinement state holding ||r64||
  double tol;
  int maxit;
  long long spin_limit;       // bounded wait of each grid barrier (polls before giving up)
};

int persistent_block();
cgp_status persistent_setup(cgp_mesh *m);
cgp_status persistent_pcg(cgp_mesh *m, bool fp32_inner, const double *b, void *x, void *const *w, double tol,
                          int maxit, KrylovState *state, const KrylovState *outer, const double *b64);

}  // namespace cgp
