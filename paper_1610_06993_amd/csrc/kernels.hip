// Device kernels of libcgp for gfx950 (CDNA4, wave64).
//
// Memory-bound work throughout: element assembly scatters into CSR values
// colour by colour (no atomics: elements of one colour share no node), CSR
// SpMV gives each row a group of L lanes so that one wavefront streams 64/L
// consecutive rows with coalesced value/column loads, and every Krylov vector
// update is fused with the dot products that follow it.  Dot products are
// reduced deterministically: wave64 butterfly, LDS across the waves of a
// block, one partial per block, and the last block to finish sums the
// partials in a fixed order and derives the solver scalars in device memory,
// so a Krylov loop needs no host round trip until its convergence check.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace cgp {
namespace dev {

// ------------------------------------------------------------------ helpers

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of the logical block index so that the rows a block
// touches, and their neighbours, stay in one XCD's L2.
__device__ __forceinline__ int xcd_block() {
  const int g = gridDim.x;
  if (g % 8 != 0) return blockIdx.x;
  return (blockIdx.x % 8) * (g / 8) + blockIdx.x / 8;
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

template <int L>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, L);
  return x;
}

__device__ __forceinline__ double ld_acq(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reduce K per-thread values over the grid.  Returns true in the last block
// to finish, where tot[] holds the grid totals in every thread.
template <int K>
__device__ __forceinline__ bool grid_reduce(double (&v)[K], const Reduce &R, double (&tot)[K]) {
  __shared__ double sh[K][16];
  __shared__ int s_last;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; k++) {
    double x = wave_sum(v[k]);
    if (lane == 0) sh[k][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < nw; w++) s += sh[threadIdx.x][w];
    R.partials[threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = (atomicAdd(R.counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!s_last) return false;
  __threadfence();
#pragma unroll
  for (int k = 0; k < K; k++) {
    double x = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x) x += ld_acq(&R.partials[k * gridDim.x + b]);
    x = wave_sum(x);
    __syncthreads();
    if (lane == 0) sh[k][wid] = x;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) {
    double s = 0.0;
    for (int w = 0; w < nw; w++) s += sh[k][w];
    tot[k] = s;
  }
  if (threadIdx.x == 0) *R.counter = 0u;
  return true;
}

__device__ __forceinline__ bool is_finite(double x) { return x == x && x - x == 0.0; }

// ------------------------------------------------------------------ assembly
// P1 element geometry: b = (y2-y3, y3-y1, y1-y2), c = (x3-x2, x1-x3, x2-x1), area.
struct Geo {
  double b[3], c[3], area;
};

__device__ __forceinline__ Geo geometry(const double2 *__restrict__ xy, int v0, int v1, int v2) {
  double2 p1 = xy[v0], p2 = xy[v1], p3 = xy[v2];
  Geo g;
  g.b[0] = p2.y - p3.y; g.b[1] = p3.y - p1.y; g.b[2] = p1.y - p2.y;
  g.c[0] = p3.x - p2.x; g.c[1] = p1.x - p3.x; g.c[2] = p2.x - p1.x;
  g.area = 0.5 * ((p2.x - p1.x) * (p3.y - p1.y) - (p3.x - p1.x) * (p2.y - p1.y));
  return g;
}

// Fine static operators: S = rho M + dt mu K, M, and the (Dx, Dy) pair
// (mass A/12(1+d_ij), stiffness (b_i b_j + c_i c_j)/4A, Dx b_j/6, Dy c_j/6).
__global__ void k_asm_fine_static(int begin, int count, const int *__restrict__ tri, const int *__restrict__ slot,
                                  const double2 *__restrict__ xy, double rho, double dtmu, double *__restrict__ S,
                                  double *__restrict__ M, double2 *__restrict__ D) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int e = begin + i;
  Geo g = geometry(xy, tri[3 * e], tri[3 * e + 1], tri[3 * e + 2]);
  const double inv4a = 1.0 / (4.0 * g.area), m1 = g.area / 12.0;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      const int s = slot[9 * e + 3 * a + b];
      const double m = (a == b) ? 2.0 * m1 : m1;
      const double k = (g.b[a] * g.b[b] + g.c[a] * g.c[b]) * inv4a;
      M[s] += m;
      S[s] += rho * m + dtmu * k;
      double2 d = D[s];
      d.x += g.b[b] / 6.0;
      d.y += g.c[b] / 6.0;
      D[s] = d;
    }
}

// Coarse static operators: Kbar, (Dbar_x, Dbar_y), lumped mass m_i += A/3.
__global__ void k_asm_coarse_static(int begin, int count, const int *__restrict__ tri, const int *__restrict__ slot,
                                    const double2 *__restrict__ xy, double *__restrict__ K,
                                    double2 *__restrict__ D, double *__restrict__ mc) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int e = begin + i;
  const int v[3] = {tri[3 * e], tri[3 * e + 1], tri[3 * e + 2]};
  Geo g = geometry(xy, v[0], v[1], v[2]);
  const double inv4a = 1.0 / (4.0 * g.area);
#pragma unroll
  for (int a = 0; a < 3; a++) {
#pragma unroll
    for (int b = 0; b < 3; b++) {
      const int s = slot[9 * e + 3 * a + b];
      K[s] += (g.b[a] * g.b[b] + g.c[a] * g.c[b]) * inv4a;
      double2 d = D[s];
      d.x += g.b[b] / 6.0;
      d.y += g.c[b] / 6.0;
      D[s] = d;
    }
    mc[v[a]] += g.area / 3.0;
  }
}

// Convection: A += dt * N(U^n), N_ab = rho/24 [(u_a + sum u) b_b + (v_a + sum v) c_b].
__global__ void k_asm_conv(int begin, int count, const int *__restrict__ tri, const int *__restrict__ slot,
                           const double2 *__restrict__ xy, const double2 *__restrict__ u, double dtrho24,
                           double *__restrict__ A) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int e = begin + i;
  const int v[3] = {tri[3 * e], tri[3 * e + 1], tri[3 * e + 2]};
  Geo g = geometry(xy, v[0], v[1], v[2]);
  const double2 u0 = u[v[0]], u1 = u[v[1]], u2 = u[v[2]];
  const double su = u0.x + u1.x + u2.x, sv = u0.y + u1.y + u2.y;
  const double ua[3] = {u0.x + su, u1.x + su, u2.x + su};
  const double va[3] = {u0.y + sv, u1.y + sv, u2.y + sv};
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) A[slot[9 * e + 3 * a + b]] += dtrho24 * (ua[a] * g.b[b] + va[a] * g.c[b]);
}

// Coarse p = 0 elimination (Eq. 14): rows/columns of pressure-Dirichlet nodes
// become identity; Jacobi inverse diagonal; FP32 copies for iterative refinement.
__global__ void k_coarse_bc(int n, const int *__restrict__ rp, const int *__restrict__ col,
                            const unsigned char *__restrict__ pdir, const double *__restrict__ K,
                            double *__restrict__ Kbc, double *__restrict__ dinv, float *__restrict__ K32,
                            float *__restrict__ dinv32) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 1.0;
  const bool di = pdir[i];
  for (int k = rp[i]; k < rp[i + 1]; k++) {
    const int j = col[k];
    double v = (di || pdir[j]) ? (i == j ? 1.0 : 0.0) : K[k];
    Kbc[k] = v;
    K32[k] = (float)v;
    if (j == i) d = v;
  }
  dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
  dinv32[i] = (float)dinv[i];
}

// Fine mass with velocity-Dirichlet identity rows/columns, its Jacobi inverse, lumped mass.
__global__ void k_mass_bc(int n, const int *__restrict__ rp, const int *__restrict__ col,
                          const unsigned char *__restrict__ vdir, const double *__restrict__ M,
                          double *__restrict__ Mbc, double *__restrict__ dinv, double *__restrict__ ml) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 1.0, s = 0.0;
  const bool di = vdir[i];
  for (int k = rp[i]; k < rp[i + 1]; k++) {
    const int j = col[k];
    s += M[k];
    double v = (di || vdir[j]) ? (i == j ? 1.0 : 0.0) : M[k];
    Mbc[k] = v;
    if (j == i) d = v;
  }
  dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
  ml[i] = s;
}

// Momentum right-hand side rho M U^n + dt M F with symmetric Dirichlet
// elimination of g on the fixed pattern, and the Jacobi inverse of A.
__global__ void k_mom_rhs_bc(int n, const int *__restrict__ rp, const int *__restrict__ col,
                             const unsigned char *__restrict__ vdir, const double *__restrict__ M,
                             double *__restrict__ A, const double2 *__restrict__ g, const double2 *__restrict__ u,
                             const double2 *__restrict__ f, double rho, double dt, double2 *__restrict__ rhs,
                             double *__restrict__ dinv) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int k0 = rp[j], k1 = rp[j + 1];
  if (vdir[j]) {
    for (int k = k0; k < k1; k++) A[k] = (col[k] == j) ? 1.0 : 0.0;
    rhs[j] = g[j];
    dinv[j] = 1.0;
    return;
  }
  double ax = 0.0, ay = 0.0, fx = 0.0, fy = 0.0, d = 1.0;
  for (int k = k0; k < k1; k++) {
    const double m = M[k];
    const double2 uc = u[col[k]];
    ax += m * uc.x;
    ay += m * uc.y;
    if (f) {
      const double2 fc = f[col[k]];
      fx += m * fc.x;
      fy += m * fc.y;
    }
  }
  double rx = rho * ax, ry = rho * ay;
  if (f) { rx += dt * fx; ry += dt * fy; }
  for (int k = k0; k < k1; k++) {
    const int c = col[k];
    if (vdir[c]) {
      const double a = A[k];
      const double2 gc = g[c];
      rx -= a * gc.x;
      ry -= a * gc.y;
      A[k] = 0.0;
    } else if (c == j) {
      d = A[k];
    }
  }
  rhs[j] = make_double2(rx, ry);
  dinv[j] = d != 0.0 ? 1.0 / d : 1.0;
}

// ------------------------------------------------------------------ SpMV
template <int L>
__global__ void k_spmv1(int n, const int *__restrict__ rp, const int *__restrict__ col,
                        const double *__restrict__ val, const double *__restrict__ x, double *__restrict__ y) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double s = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) s += val[k] * x[col[k]];
    s = group_sum<L>(s);
    if (lane == 0) y[row] = s;
  }
}

template <int L>
__global__ void k_spmv1_f32(int n, const int *__restrict__ rp, const int *__restrict__ col,
                            const float *__restrict__ val, const float *__restrict__ x, float *__restrict__ y) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    float s = 0.0f;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) s += val[k] * x[col[k]];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
    if (lane == 0) y[row] = s;
  }
}

template <int L>
__global__ void k_spmv2(int n, const int *__restrict__ rp, const int *__restrict__ col,
                        const double *__restrict__ val, const double2 *__restrict__ x, double2 *__restrict__ y) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sx = 0.0, sy = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const double a = val[k];
      const double2 xc = x[col[k]];
      sx += a * xc.x;
      sy += a * xc.y;
    }
    sx = group_sum<L>(sx);
    sy = group_sum<L>(sy);
    if (lane == 0) y[row] = make_double2(sx, sy);
  }
}

// ------------------------------------------------------------------ PCG (NC = 1 or 2 components)
// Vectors of NC components are stored interleaved [n][NC].
template <int NC>
struct V;
template <>
struct V<1> {
  using T = double;
  static __device__ __forceinline__ void get(const double *p, int i, double (&o)[1]) { o[0] = p[i]; }
  static __device__ __forceinline__ void put(double *p, int i, const double (&o)[1]) { p[i] = o[0]; }
};
template <>
struct V<2> {
  static __device__ __forceinline__ void get(const double *p, int i, double (&o)[2]) {
    double2 t = reinterpret_cast<const double2 *>(p)[i];
    o[0] = t.x;
    o[1] = t.y;
  }
  static __device__ __forceinline__ void put(double *p, int i, const double (&o)[2]) {
    reinterpret_cast<double2 *>(p)[i] = make_double2(o[0], o[1]);
  }
};

// r = b - A x, z = D^-1 r, p_old = 0; totals (r.z, r.r, b.b) per component.
template <int NC, int L>
__global__ void k_cg_init(int n, const int *__restrict__ rp, const int *__restrict__ col,
                          const double *__restrict__ A, const double *__restrict__ b, const double *__restrict__ x,
                          const double *__restrict__ dinv, double *__restrict__ r, double *__restrict__ z,
                          double *__restrict__ p0, double *__restrict__ p1, KrylovState *__restrict__ st, Reduce R) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[3 * NC];
#pragma unroll
  for (int c = 0; c < 3 * NC; c++) acc[c] = 0.0;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) s[c] = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      double xc[NC];
      V<NC>::get(x, col[k], xc);
      const double a = A[k];
#pragma unroll
      for (int c = 0; c < NC; c++) s[c] += a * xc[c];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) s[c] = group_sum<L>(s[c]);
    if (lane == 0) {
      double bb[NC], rr[NC], zz[NC], zero[NC];
      V<NC>::get(b, row, bb);
      const double d = dinv[row];
#pragma unroll
      for (int c = 0; c < NC; c++) {
        rr[c] = bb[c] - s[c];
        zz[c] = d * rr[c];
        zero[c] = 0.0;
        acc[c] += rr[c] * zz[c];
        acc[NC + c] += rr[c] * rr[c];
        acc[2 * NC + c] += bb[c] * bb[c];
      }
      V<NC>::put(r, row, rr);
      V<NC>::put(z, row, zz);
      V<NC>::put(p0, row, zero);
      V<NC>::put(p1, row, zero);
    }
  }
  double tot[3 * NC];
  if (grid_reduce<3 * NC>(acc, R, tot) && threadIdx.x == 0) {
    for (int c = 0; c < NC; c++) {
      const double bn = sqrt(tot[2 * NC + c]), rn = sqrt(tot[NC + c]);
      st->bnorm[c] = bn;
      st->rnorm[c] = rn;
      st->rz[c] = tot[c];
      st->beta[c] = 0.0;
      st->zero_b[c] = (bn == 0.0);
      st->done[c] = (bn == 0.0) || (rn <= st->tol * bn);
      if (!is_finite(bn) || !is_finite(rn)) st->status = CGP_E_NONFINITE;
    }
    st->iters = 0;
  }
}

// p_new = z + beta p_old (own rows), q = A p_new with p_new gathered on the fly,
// total p_new.q -> alpha = rz / (p.q).
template <int NC, int L>
__global__ void k_cg_spmv(int n, const int *__restrict__ rp, const int *__restrict__ col,
                          const double *__restrict__ A, const double *__restrict__ z,
                          const double *__restrict__ p_old, double *__restrict__ p_new, double *__restrict__ q,
                          KrylovState *__restrict__ st, Reduce R) {
  if (st->status) return;
  bool all_done = true;
  double beta[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) {
    all_done = all_done && st->done[c];
    beta[c] = st->beta[c];
  }
  if (all_done) return;
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) acc[c] = 0.0;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) s[c] = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const int j = col[k];
      double zc[NC], pc[NC];
      V<NC>::get(z, j, zc);
      V<NC>::get(p_old, j, pc);
      const double a = A[k];
#pragma unroll
      for (int c = 0; c < NC; c++) s[c] += a * (zc[c] + beta[c] * pc[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; c++) s[c] = group_sum<L>(s[c]);
    if (lane == 0) {
      double zc[NC], pc[NC];
      V<NC>::get(z, row, zc);
      V<NC>::get(p_old, row, pc);
#pragma unroll
      for (int c = 0; c < NC; c++) {
        pc[c] = zc[c] + beta[c] * pc[c];
        acc[c] += pc[c] * s[c];
      }
      V<NC>::put(p_new, row, pc);
      V<NC>::put(q, row, s);
    }
  }
  double tot[NC];
  if (grid_reduce<NC>(acc, R, tot) && threadIdx.x == 0) {
    for (int c = 0; c < NC; c++) {
      st->alpha[c] = st->rz[c] / tot[c];
      if (!is_finite(st->alpha[c]) && !st->done[c]) st->status = CGP_E_NONFINITE;
    }
  }
}

// x += alpha p, r -= alpha q, z = D^-1 r (components not yet converged);
// totals r.z, r.r -> beta, residual norm, convergence.
template <int NC>
__global__ void k_cg_update(int n, double *__restrict__ x, double *__restrict__ r, double *__restrict__ z,
                            const double *__restrict__ dinv, const double *__restrict__ p,
                            const double *__restrict__ q, KrylovState *__restrict__ st, Reduce R) {
  if (st->status) return;
  bool all_done = true, act[NC];
  double alpha[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) {
    act[c] = !st->done[c];
    all_done = all_done && !act[c];
    alpha[c] = st->alpha[c];
  }
  if (all_done) return;
  double acc[2 * NC];
#pragma unroll
  for (int c = 0; c < 2 * NC; c++) acc[c] = 0.0;
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    double xx[NC], rr[NC], zz[NC], pp[NC], qq[NC];
    V<NC>::get(x, i, xx);
    V<NC>::get(r, i, rr);
    V<NC>::get(p, i, pp);
    V<NC>::get(q, i, qq);
    V<NC>::get(z, i, zz);
    const double d = dinv[i];
#pragma unroll
    for (int c = 0; c < NC; c++) {
      if (act[c]) {
        xx[c] += alpha[c] * pp[c];
        rr[c] -= alpha[c] * qq[c];
        zz[c] = d * rr[c];
      }
      acc[c] += rr[c] * zz[c];
      acc[NC + c] += rr[c] * rr[c];
    }
    V<NC>::put(x, i, xx);
    V<NC>::put(r, i, rr);
    V<NC>::put(z, i, zz);
  }
  double tot[2 * NC];
  if (grid_reduce<2 * NC>(acc, R, tot) && threadIdx.x == 0) {
    for (int c = 0; c < NC; c++) {
      if (!act[c]) continue;
      const double rn = sqrt(tot[NC + c]);
      st->beta[c] = tot[c] / st->rz[c];
      st->rz[c] = tot[c];
      st->rnorm[c] = rn;
      if (!is_finite(rn)) st->status = CGP_E_NONFINITE;
      if (rn <= st->tol * st->bnorm[c]) st->done[c] = 1;
    }
    st->iters += 1;
    bool all = true;
    for (int c = 0; c < NC; c++) all = all && st->done[c];
    if (!all && st->iters >= st->maxit) st->status = CGP_E_NOCONV;
  }
}

// components whose right-hand side is zero get x = 0
template <int NC>
__global__ void k_zero_b_fix(int n, double *__restrict__ x, const KrylovState *__restrict__ st) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < NC; c++)
    if (st->zero_b[c]) x[NC * i + c] = 0.0;
}

// ------------------------------------------------------------------ BiCGStab, 2 components
// r = b - A x, r^ = r, p = v = 0; totals r.r and b.b; rho = r^.r = r.r.
template <int L>
__global__ void k_bi_init(int n, const int *__restrict__ rp, const int *__restrict__ col,
                          const double *__restrict__ A, const double2 *__restrict__ b, const double2 *__restrict__ x,
                          double2 *__restrict__ r, double2 *__restrict__ rh, double2 *__restrict__ p,
                          double2 *__restrict__ v, KrylovState *__restrict__ st, Reduce R) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sx = 0.0, sy = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const double a = A[k];
      const double2 xc = x[col[k]];
      sx += a * xc.x;
      sy += a * xc.y;
    }
    sx = group_sum<L>(sx);
    sy = group_sum<L>(sy);
    if (lane == 0) {
      const double2 bb = b[row];
      const double2 rr = make_double2(bb.x - sx, bb.y - sy);
      r[row] = rr;
      rh[row] = rr;
      p[row] = make_double2(0.0, 0.0);
      v[row] = make_double2(0.0, 0.0);
      acc[0] += rr.x * rr.x;
      acc[1] += rr.y * rr.y;
      acc[2] += bb.x * bb.x;
      acc[3] += bb.y * bb.y;
    }
  }
  double tot[4];
  if (grid_reduce<4>(acc, R, tot) && threadIdx.x == 0) {
    for (int c = 0; c < 2; c++) {
      const double bn = sqrt(tot[2 + c]), rn = sqrt(tot[c]);
      st->bnorm[c] = bn;
      st->rnorm[c] = rn;
      st->zero_b[c] = (bn == 0.0);
      st->done[c] = (bn == 0.0) || (rn <= st->tol * bn);
      // first iteration: rho_old = alpha = omega = 1, rho_new = r^.r
      st->beta[c] = tot[c];       // (rho_new / 1) * (1 / 1)
      st->rho[c] = tot[c];
      st->omega[c] = 1.0;
      st->alpha[c] = 1.0;
      if (!is_finite(bn) || !is_finite(rn)) st->status = CGP_E_NONFINITE;
    }
    st->iters = 0;
  }
}

// p = r + beta (p - omega v), p^ = D^-1 p
__global__ void k_bi_p(int n, const double2 *__restrict__ r, double2 *__restrict__ p, const double2 *__restrict__ v,
                       const double *__restrict__ dinv, double2 *__restrict__ ph, const KrylovState *__restrict__ st) {
  if (st->status || (st->done[0] && st->done[1])) return;
  // beta holds rho_new/rho_old * alpha/omega for the iteration about to run
  const double b0 = st->beta[0], b1 = st->beta[1], w0 = st->omega[0], w1 = st->omega[1];
  const bool a0 = !st->done[0], a1 = !st->done[1];
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double2 rr = r[i], vv = v[i];
    double2 pp = p[i];
    if (a0) pp.x = rr.x + b0 * (pp.x - w0 * vv.x);
    if (a1) pp.y = rr.y + b1 * (pp.y - w1 * vv.y);
    p[i] = pp;
    const double d = dinv[i];
    ph[i] = make_double2(d * pp.x, d * pp.y);
  }
}

// v = A p^; total r^.v -> alpha = rho / (r^.v)
template <int L>
__global__ void k_bi_v(int n, const int *__restrict__ rp, const int *__restrict__ col, const double *__restrict__ A,
                       const double2 *__restrict__ ph, double2 *__restrict__ v, const double2 *__restrict__ rh,
                       KrylovState *__restrict__ st, Reduce R) {
  if (st->status || (st->done[0] && st->done[1])) return;
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[2] = {0.0, 0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sx = 0.0, sy = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const double a = A[k];
      const double2 xc = ph[col[k]];
      sx += a * xc.x;
      sy += a * xc.y;
    }
    sx = group_sum<L>(sx);
    sy = group_sum<L>(sy);
    if (lane == 0) {
      v[row] = make_double2(sx, sy);
      const double2 h = rh[row];
      acc[0] += h.x * sx;
      acc[1] += h.y * sy;
    }
  }
  double tot[2];
  if (grid_reduce<2>(acc, R, tot) && threadIdx.x == 0) {
    for (int c = 0; c < 2; c++) {
      if (st->done[c]) continue;
      st->alpha[c] = st->rho[c] / tot[c];
      if (!is_finite(st->alpha[c])) st->status = CGP_E_NONFINITE;
    }
  }
}

// s = r - alpha v formed on the fly, t = A (D^-1 s); totals t.s, t.t -> omega
template <int L>
__global__ void k_bi_t(int n, const int *__restrict__ rp, const int *__restrict__ col, const double *__restrict__ A,
                       const double2 *__restrict__ r, const double2 *__restrict__ v, const double *__restrict__ dinv,
                       double2 *__restrict__ t, KrylovState *__restrict__ st, Reduce R) {
  if (st->status || (st->done[0] && st->done[1])) return;
  const double al0 = st->alpha[0], al1 = st->alpha[1];
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sx = 0.0, sy = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const int j = col[k];
      const double a = A[k] * dinv[j];
      const double2 rr = r[j], vv = v[j];
      sx += a * (rr.x - al0 * vv.x);
      sy += a * (rr.y - al1 * vv.y);
    }
    sx = group_sum<L>(sx);
    sy = group_sum<L>(sy);
    if (lane == 0) {
      t[row] = make_double2(sx, sy);
      const double2 rr = r[row], vv = v[row];
      const double s0 = rr.x - al0 * vv.x, s1 = rr.y - al1 * vv.y;
      acc[0] += sx * s0;
      acc[1] += sy * s1;
      acc[2] += sx * sx;
      acc[3] += sy * sy;
    }
  }
  double tot[4];
  if (grid_reduce<4>(acc, R, tot) && threadIdx.x == 0) {
    for (int c = 0; c < 2; c++) {
      if (st->done[c]) continue;
      st->omega[c] = tot[2 + c] > 0.0 ? tot[c] / tot[2 + c] : 0.0;
    }
  }
}

// x += alpha p^ + omega D^-1 s, r = s - omega t; totals r.r, r^.r -> convergence, next beta
__global__ void k_bi_x(int n, double2 *__restrict__ x, double2 *__restrict__ r, const double2 *__restrict__ v,
                       const double2 *__restrict__ t, const double *__restrict__ dinv, const double2 *__restrict__ ph,
                       const double2 *__restrict__ rh, KrylovState *__restrict__ st, Reduce R) {
  if (st->status || (st->done[0] && st->done[1])) return;
  const bool a0 = !st->done[0], a1 = !st->done[1];
  const double al0 = st->alpha[0], al1 = st->alpha[1], w0 = st->omega[0], w1 = st->omega[1];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    double2 xx = x[i], rr = r[i];
    const double2 vv = v[i], tt = t[i], pp = ph[i], hh = rh[i];
    const double d = dinv[i];
    if (a0) {
      const double s = rr.x - al0 * vv.x;
      xx.x += al0 * pp.x + w0 * (d * s);
      rr.x = s - w0 * tt.x;
    }
    if (a1) {
      const double s = rr.y - al1 * vv.y;
      xx.y += al1 * pp.y + w1 * (d * s);
      rr.y = s - w1 * tt.y;
    }
    x[i] = xx;
    r[i] = rr;
    acc[0] += rr.x * rr.x;
    acc[1] += rr.y * rr.y;
    acc[2] += hh.x * rr.x;
    acc[3] += hh.y * rr.y;
  }
  double tot[4];
  if (grid_reduce<4>(acc, R, tot) && threadIdx.x == 0) {
    for (int c = 0; c < 2; c++) {
      if (st->done[c]) continue;
      const double rn = sqrt(tot[c]);
      st->rnorm[c] = rn;
      if (!is_finite(rn)) st->status = CGP_E_NONFINITE;
      if (rn <= st->tol * st->bnorm[c]) {
        st->done[c] = 1;
      } else if (st->omega[c] == 0.0) {
        st->status = CGP_E_NOCONV;  // breakdown
      }
      const double rho_new = tot[2 + c];
      st->beta[c] = (rho_new / st->rho[c]) * (st->alpha[c] / st->omega[c]);
      st->rho[c] = rho_new;
    }
    st->iters += 1;
    if (!(st->done[0] && st->done[1]) && st->iters >= st->maxit) st->status = CGP_E_NOCONV;
  }
}

// ------------------------------------------------------------------ pressure path
// INJECT (Eqs. 20-21, 30): b_c[i] = s * sum_k (Dbar_x u~_x + Dbar_y u~_y) at coarse
// column j, which is fine node j (coarse nodes are the prefix of the fine numbering).
template <int L>
__global__ void k_div(int n, const int *__restrict__ rp, const int *__restrict__ col, const double2 *__restrict__ D,
                      const double2 *__restrict__ ut, double s, double *__restrict__ b) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double acc = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const double2 d = D[k];
      const double2 u = ut[col[k]];
      acc += d.x * u.x + d.y * u.y;
    }
    acc = group_sum<L>(acc);
    if (lane == 0) b[row] = s * acc;
  }
}

// GALERKIN: b_{k-1}[i] = b_k[i] + 1/2 sum of b_k over the midpoints whose parent is i
__global__ void k_restrict_gather(int nprev, const int *__restrict__ ptr, const int *__restrict__ idx,
                                  const double *__restrict__ bk, double *__restrict__ bprev) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nprev) return;
  double acc = bk[i];
  for (int q = ptr[i]; q < ptr[i + 1]; q++) acc += 0.5 * bk[idx[q]];
  bprev[i] = acc;
}

// Prolongation (Eqs. 22, 29): copy the prefix, average the two parents of each midpoint.
__global__ void k_prolong(int nprev, int nk, const int2 *__restrict__ parent, const double *__restrict__ pc,
                          double *__restrict__ pf) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nk) return;
  if (i < nprev) {
    pf[i] = pc[i];
  } else {
    const int2 par = parent[i - nprev];
    pf[i] = 0.5 * (pc[par.x] + pc[par.y]);
  }
}

// p = 0 rows (Eq. 14): zero right-hand side and initial guess there
__global__ void k_pdir_zero(int n, const unsigned char *__restrict__ pdir, double *__restrict__ b,
                            double *__restrict__ x) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (pdir[i]) {
    b[i] = 0.0;
    x[i] = 0.0;
  }
}

// Sum of w[i] * x[i] (w = NULL: plain sum) over the grid into *out.
__global__ void k_wsum(int n, const double *__restrict__ w, const double *__restrict__ x, double *__restrict__ out,
                       Reduce R) {
  double acc[1] = {0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc[0] += (w ? w[i] : 1.0) * x[i];
  double tot[1];
  if (grid_reduce<1>(acc, R, tot) && threadIdx.x == 0) *out = tot[0];
}

// x -= (*num) / den
__global__ void k_shift(int n, double *__restrict__ x, const double *__restrict__ num, double den) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] -= *num / den;
}

// Correction right-hand side (Eq. 23): M u~ - (dt/rho)(Dx P, Dy P), lifted with g.
template <int L>
__global__ void k_correct_rhs(int n, const int *__restrict__ rp, const int *__restrict__ col,
                              const unsigned char *__restrict__ vdir, const double *__restrict__ M,
                              const double2 *__restrict__ D, const double2 *__restrict__ ut,
                              const double *__restrict__ pf, const double2 *__restrict__ g, double s,
                              double2 *__restrict__ rhs) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double mx = 0.0, my = 0.0, gx = 0.0, gy = 0.0, lx = 0.0, ly = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const int c = col[k];
      const double m = M[k];
      const double2 u = ut[c], d = D[k];
      const double p = pf[c];
      mx += m * u.x;
      my += m * u.y;
      gx += d.x * p;
      gy += d.y * p;
      if (vdir[c]) {
        const double2 gc = g[c];
        lx += m * gc.x;
        ly += m * gc.y;
      }
    }
    mx = group_sum<L>(mx); my = group_sum<L>(my);
    gx = group_sum<L>(gx); gy = group_sum<L>(gy);
    lx = group_sum<L>(lx); ly = group_sum<L>(ly);
    if (lane == 0) rhs[row] = vdir[row] ? g[row] : make_double2(mx - s * gx - lx, my - s * gy - ly);
  }
}

// LUMPED correction: u = u~ - s (G P) / m_L at free nodes, g at Dirichlet nodes.
template <int L>
__global__ void k_correct_lumped(int n, const int *__restrict__ rp, const int *__restrict__ col,
                                 const unsigned char *__restrict__ vdir, const double2 *__restrict__ D,
                                 const double2 *__restrict__ ut, const double *__restrict__ pf,
                                 const double *__restrict__ ml, const double2 *__restrict__ g, double s,
                                 double2 *__restrict__ u) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double gx = 0.0, gy = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const double2 d = D[k];
      const double p = pf[col[k]];
      gx += d.x * p;
      gy += d.y * p;
    }
    gx = group_sum<L>(gx);
    gy = group_sum<L>(gy);
    if (lane == 0) {
      const double2 t = ut[row];
      const double m = ml[row];
      u[row] = vdir[row] ? g[row] : make_double2(t.x - s * gx / m, t.y - s * gy / m);
    }
  }
}

__global__ void k_set_dirichlet(int n, const unsigned char *__restrict__ vdir, const double2 *__restrict__ g,
                                double2 *__restrict__ u) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (vdir[i]) u[i] = g[i];
}

// finiteness check of an input vector; sets *flag = 1 on NaN/Inf
__global__ void k_check_finite(size_t n, const double *__restrict__ x, int *__restrict__ flag) {
  size_t i = size_t(blockIdx.x) * blockDim.x + threadIdx.x;
  size_t stride = size_t(gridDim.x) * blockDim.x;
  bool bad = false;
  for (; i < n; i += stride) bad |= !is_finite(x[i]);
  if (bad) atomicOr(flag, 1);
}

// ------------------------------------------------------------------ FP32 iterative refinement pieces
// r64 = b - K x (FP64), totals r.r and b.b; writes r32 = r64 / ||r64|| is done by a second kernel
template <int L>
__global__ void k_ir_residual(int n, const int *__restrict__ rp, const int *__restrict__ col,
                              const double *__restrict__ A, const double *__restrict__ b, const double *__restrict__ x,
                              double *__restrict__ r, KrylovState *__restrict__ st, Reduce R) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[2] = {0.0, 0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double s = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) s += A[k] * x[col[k]];
    s = group_sum<L>(s);
    if (lane == 0) {
      const double bb = b[row], rr = bb - s;
      r[row] = rr;
      acc[0] += rr * rr;
      acc[1] += bb * bb;
    }
  }
  double tot[2];
  if (grid_reduce<2>(acc, R, tot) && threadIdx.x == 0) {
    const double rn = sqrt(tot[0]), bn = sqrt(tot[1]);
    st->rnorm[0] = rn;
    st->bnorm[0] = bn;
    st->zero_b[0] = (bn == 0.0);
    st->done[0] = (bn == 0.0) || (rn <= st->tol * bn);
    if (!is_finite(rn) || !is_finite(bn)) st->status = CGP_E_NONFINITE;
  }
}

// Inner FP32 Jacobi-PCG on d with K32 d = r / ||r||; vectors in FP32, dots in FP64.
// init: r32 = r64 / ||r64||, z = D^-1 r32, d = 0, p = 0
__global__ void k_ir_inner_init(int n, const double *__restrict__ r64, const float *__restrict__ dinv,
                                float *__restrict__ r, float *__restrict__ z, float *__restrict__ d,
                                float *__restrict__ p0, float *__restrict__ p1, const KrylovState *__restrict__ outer,
                                KrylovState *__restrict__ st, Reduce R) {
  const double inv = outer->rnorm[0] > 0.0 ? 1.0 / outer->rnorm[0] : 0.0;
  double acc[2] = {0.0, 0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float rr = (float)(r64[i] * inv);
    const float zz = dinv[i] * rr;
    r[i] = rr;
    z[i] = zz;
    d[i] = 0.0f;
    p0[i] = 0.0f;
    p1[i] = 0.0f;
    acc[0] += (double)rr * (double)zz;
    acc[1] += (double)rr * (double)rr;
  }
  double tot[2];
  if (grid_reduce<2>(acc, R, tot) && threadIdx.x == 0) {
    st->rz[0] = tot[0];
    st->rnorm[0] = sqrt(tot[1]);
    st->bnorm[0] = sqrt(tot[1]);
    st->beta[0] = 0.0;
    st->iters = 0;
    st->done[0] = outer->done[0] || outer->status != 0;
    st->status = 0;
  }
}

template <int L>
__global__ void k_cg32_spmv(int n, const int *__restrict__ rp, const int *__restrict__ col,
                            const float *__restrict__ A, const float *__restrict__ z, const float *__restrict__ p_old,
                            float *__restrict__ p_new, float *__restrict__ q, KrylovState *__restrict__ st, Reduce R) {
  if (st->status || st->done[0]) return;
  const float beta = (float)st->beta[0];
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[1] = {0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    float s = 0.0f;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const int j = col[k];
      s += A[k] * (z[j] + beta * p_old[j]);
    }
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
    if (lane == 0) {
      const float pn = z[row] + beta * p_old[row];
      p_new[row] = pn;
      q[row] = s;
      acc[0] += (double)pn * (double)s;
    }
  }
  double tot[1];
  if (grid_reduce<1>(acc, R, tot) && threadIdx.x == 0) {
    st->alpha[0] = st->rz[0] / tot[0];
    if (!is_finite(st->alpha[0])) st->status = CGP_E_NONFINITE;
  }
}

__global__ void k_cg32_update(int n, float *__restrict__ x, float *__restrict__ r, float *__restrict__ z,
                              const float *__restrict__ dinv, const float *__restrict__ p,
                              const float *__restrict__ q, KrylovState *__restrict__ st, Reduce R) {
  if (st->status || st->done[0]) return;
  const float alpha = (float)st->alpha[0];
  double acc[2] = {0.0, 0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float xx = x[i] + alpha * p[i];
    const float rr = r[i] - alpha * q[i];
    const float zz = dinv[i] * rr;
    x[i] = xx;
    r[i] = rr;
    z[i] = zz;
    acc[0] += (double)rr * (double)zz;
    acc[1] += (double)rr * (double)rr;
  }
  double tot[2];
  if (grid_reduce<2>(acc, R, tot) && threadIdx.x == 0) {
    const double rn = sqrt(tot[1]);
    st->beta[0] = tot[0] / st->rz[0];
    st->rz[0] = tot[0];
    st->rnorm[0] = rn;
    st->iters += 1;
    if (!is_finite(rn)) st->status = CGP_E_NONFINITE;
    if (rn <= st->tol * st->bnorm[0] || st->iters >= st->maxit) st->done[0] = 1;
  }
}

// x += ||r64|| * d (FP64 update of the outer iterate)
__global__ void k_ir_update(int n, double *__restrict__ x, const float *__restrict__ d,
                            const KrylovState *__restrict__ outer) {
  if (outer->done[0] || outer->status) return;
  const double s = outer->rnorm[0];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] += s * (double)d[i];
}

}  // namespace dev
}  // namespace cgp

// ====================================================================== host drivers
#include <algorithm>
#include <type_traits>

namespace cgp {
using namespace dev;

namespace {

inline int grid_for(long long threads) {
  long long b = (threads + 255) / 256;
  b = std::max<long long>(8, (b + 7) / 8 * 8);
  return int(std::min<long long>(b, kMaxGrid));
}
inline int blocks_1d(long long n) { return int(std::max<long long>(1, (n + 255) / 256)); }

template <typename F>
void dispatch_L(int L, F &&f) {
  switch (L) {
    case 4: f(std::integral_constant<int, 4>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 8>{}); break;
  }
}

inline Reduce red(cgp_mesh *m) { return Reduce{m->red.partials, m->red.counter}; }

__global__ void k_state_init(KrylovState *st, double tol, int maxit, int ncomp) {
  KrylovState s{};
  s.tol = tol;
  s.maxit = maxit;
  s.ncomp = ncomp;
  *st = s;
}

enum { SLOT_MOM = 0, SLOT_P = 1, SLOT_PIN = 2, SLOT_MASS = 3 };

cgp_status poll(cgp_mesh *m, int slot, int count = 1) {
  CGP_HIP(hipMemcpyAsync(&m->h_state[slot], m->d_state + slot, sizeof(KrylovState) * count, hipMemcpyDeviceToHost,
                         m->stream));
  CGP_HIP(hipStreamSynchronize(m->stream));
  return CGP_OK;
}

bool all_done(const KrylovState &s) {
  for (int c = 0; c < s.ncomp; c++)
    if (!s.done[c]) return false;
  return true;
}

cgp_status status_of(const KrylovState &s) {
  if (s.status == CGP_E_NONFINITE) {
    set_error("Krylov solve produced a non-finite residual");
    return CGP_E_NONFINITE;
  }
  if (s.status == CGP_E_NOCONV || !all_done(s)) {
    set_error("Krylov solve reached its iteration limit");
    return CGP_E_NOCONV;
  }
  return CGP_OK;
}

// Jacobi-PCG on NC interleaved components; x holds the initial guess.
template <int NC>
cgp_status run_pcg(cgp_mesh *m, int slot, int n, const int *rp, const int *col, const double *A, const double *dinv,
                   const double *b, double *x, double **w, int L, double tol, int maxit, int *first_chunk,
                   KrylovState *out) {
  double *r = w[0], *z = w[1], *p0 = w[2], *p1 = w[3], *q = w[4];
  KrylovState *st = m->d_state + slot;
  Reduce R = red(m);
  hipStream_t s = m->stream;
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, tol, maxit, NC);
  const int gL = grid_for((long long)n * L), g1 = grid_for(n);
  dispatch_L(L, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    hipLaunchKernelGGL((k_cg_init<NC, LL>), dim3(gL), dim3(256), 0, s, n, rp, col, A, b, x, dinv, r, z, p0, p1, st, R);
  });
  int it = 0, chunk = std::max(1, *first_chunk);
  for (;;) {
    dispatch_L(L, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      for (int c = 0; c < chunk; c++, it++) {
        double *po = (it & 1) ? p1 : p0, *pn = (it & 1) ? p0 : p1;
        hipLaunchKernelGGL((k_cg_spmv<NC, LL>), dim3(gL), dim3(256), 0, s, n, rp, col, A, z, po, pn, q, st, R);
        hipLaunchKernelGGL((k_cg_update<NC>), dim3(g1), dim3(256), 0, s, n, x, r, z, dinv, pn, q, st, R);
      }
    });
    CGP_HIP(hipGetLastError());
    cgp_status ps = poll(m, slot);
    if (ps) return ps;
    const KrylovState &h = m->h_state[slot];
    if (h.status || all_done(h) || it >= maxit + 1) break;
    chunk = 8;
  }
  hipLaunchKernelGGL((k_zero_b_fix<NC>), dim3(blocks_1d(n)), dim3(256), 0, s, n, x, st);
  *out = m->h_state[slot];
  *first_chunk = std::max(1, out->iters - 4);
  return status_of(*out);
}

}  // namespace

// ------------------------------------------------------------------ assembly
cgp_status drv_assemble(cgp_mesh *m) {
  hipStream_t s = m->stream;
  const size_t nf = m->pf.nnz, nc = m->pc.nnz;
  const int Nf = m->pf.n, Nc = m->pc.n;
  CGP_HIP(hipMemsetAsync(m->d_S, 0, nf * sizeof(double), s));
  CGP_HIP(hipMemsetAsync(m->d_M, 0, nf * sizeof(double), s));
  CGP_HIP(hipMemsetAsync(m->d_D, 0, 2 * nf * sizeof(double), s));
  CGP_HIP(hipMemsetAsync(m->d_K, 0, nc * sizeof(double), s));
  CGP_HIP(hipMemsetAsync(m->d_Dc, 0, 2 * nc * sizeof(double), s));
  CGP_HIP(hipMemsetAsync(m->d_mc, 0, Nc * sizeof(double), s));
  const double rho = m->params.rho, dtmu = m->params.dt * m->params.mu;
  for (int c = 0; c < m->col_f.ncol; c++) {
    const int b0 = m->col_f.cptr[c], cnt = m->col_f.cptr[c + 1] - b0;
    hipLaunchKernelGGL(k_asm_fine_static, dim3(blocks_1d(cnt)), dim3(256), 0, s, b0, cnt, m->d_tri_f, m->d_slot_f,
                       (const double2 *)m->d_xy_f, rho, dtmu, m->d_S, m->d_M, (double2 *)m->d_D);
  }
  for (int c = 0; c < m->col_c.ncol; c++) {
    const int b0 = m->col_c.cptr[c], cnt = m->col_c.cptr[c + 1] - b0;
    hipLaunchKernelGGL(k_asm_coarse_static, dim3(blocks_1d(cnt)), dim3(256), 0, s, b0, cnt, m->d_tri_c, m->d_slot_c,
                       (const double2 *)m->d_xy_c, m->d_K, (double2 *)m->d_Dc, m->d_mc);
  }
  hipLaunchKernelGGL(k_coarse_bc, dim3(blocks_1d(Nc)), dim3(256), 0, s, Nc, m->d_rp_c, m->d_col_c, m->d_pdir, m->d_K,
                     m->d_Kbc, m->d_dinvK, m->d_Kbc32, m->d_dinvK32);
  hipLaunchKernelGGL(k_mass_bc, dim3(blocks_1d(Nf)), dim3(256), 0, s, Nf, m->d_rp_f, m->d_col_f, m->d_vdir, m->d_M,
                     m->d_Mbc, m->d_dinvM, m->d_ml);
  hipLaunchKernelGGL(k_wsum, dim3(grid_for(Nc)), dim3(256), 0, s, Nc, (const double *)nullptr, m->d_mc,
                     m->d_scalar, red(m));
  CGP_HIP(hipGetLastError());
  CGP_HIP(hipMemcpyAsync(&m->h_scalar[0], m->d_scalar, sizeof(double), hipMemcpyDeviceToHost, s));
  CGP_HIP(hipStreamSynchronize(s));
  m->mc_sum = m->h_scalar[0];
  return CGP_OK;
}

// ------------------------------------------------------------------ step 1
cgp_status drv_momentum(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *f, const double *u,
                        double *ut, cgp_stats *stats) {
  hipStream_t s = m->stream;
  const int n = m->pf.n;
  const size_t nnz = m->pf.nnz;
  CGP_HIP(hipMemcpyAsync(m->d_A, m->d_S, nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
  const double dtrho24 = m->params.dt * m->params.rho / 24.0;
  for (int c = 0; c < m->col_f.ncol; c++) {
    const int b0 = m->col_f.cptr[c], cnt = m->col_f.cptr[c + 1] - b0;
    hipLaunchKernelGGL(k_asm_conv, dim3(blocks_1d(cnt)), dim3(256), 0, s, b0, cnt, m->d_tri_f, m->d_slot_f,
                       (const double2 *)m->d_xy_f, (const double2 *)u, dtrho24, m->d_A);
  }
  double2 *rhs = (double2 *)m->d_wf[0];
  hipLaunchKernelGGL(k_mom_rhs_bc, dim3(blocks_1d(n)), dim3(256), 0, s, n, m->d_rp_f, m->d_col_f, m->d_vdir, m->d_M,
                     m->d_A, (const double2 *)g, (const double2 *)u, (const double2 *)f, m->params.rho,
                     m->params.dt, rhs, m->d_dinvA);
  if (o->x0_mode == CGP_X0_ZERO)
    CGP_HIP(hipMemsetAsync(ut, 0, 2 * n * sizeof(double), s));
  else
    CGP_HIP(hipMemcpyAsync(ut, u, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  double2 *r = (double2 *)m->d_wf[1], *rh = (double2 *)m->d_wf[2], *p = (double2 *)m->d_wf[3];
  double2 *v = (double2 *)m->d_wf[4], *t = (double2 *)m->d_wf[5], *ph = (double2 *)m->d_wf[6];
  KrylovState *st = m->d_state + SLOT_MOM;
  Reduce R = red(m);
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, o->tol, o->max_iter, 2);
  const int L = m->lanes_f, gL = grid_for((long long)n * L), g1 = grid_for(n);
  const int *rp = m->d_rp_f, *col = m->d_col_f;
  const double *A = m->d_A, *dinv = m->d_dinvA;
  double2 *x = (double2 *)ut;
  dispatch_L(L, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    hipLaunchKernelGGL((k_bi_init<LL>), dim3(gL), dim3(256), 0, s, n, rp, col, A, (const double2 *)rhs,
                       (const double2 *)x, r, rh, p, v, st, R);
  });
  int it = 0, chunk = std::max(1, m->mom_chunk);
  for (;;) {
    dispatch_L(L, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      for (int c = 0; c < chunk; c++, it++) {
        hipLaunchKernelGGL(k_bi_p, dim3(g1), dim3(256), 0, s, n, (const double2 *)r, p, (const double2 *)v, dinv, ph,
                           (const KrylovState *)st);
        hipLaunchKernelGGL((k_bi_v<LL>), dim3(gL), dim3(256), 0, s, n, rp, col, A, (const double2 *)ph, v,
                           (const double2 *)rh, st, R);
        hipLaunchKernelGGL((k_bi_t<LL>), dim3(gL), dim3(256), 0, s, n, rp, col, A, (const double2 *)r,
                           (const double2 *)v, dinv, t, st, R);
        hipLaunchKernelGGL(k_bi_x, dim3(g1), dim3(256), 0, s, n, x, r, (const double2 *)v, (const double2 *)t, dinv,
                           (const double2 *)ph, (const double2 *)rh, st, R);
      }
    });
    CGP_HIP(hipGetLastError());
    cgp_status ps = poll(m, SLOT_MOM);
    if (ps) return ps;
    const KrylovState &h = m->h_state[SLOT_MOM];
    if (h.status || all_done(h) || it >= o->max_iter + 1) break;
    chunk = 2;
  }
  hipLaunchKernelGGL((k_zero_b_fix<2>), dim3(blocks_1d(n)), dim3(256), 0, s, n, ut, (const KrylovState *)st);
  const KrylovState h = m->h_state[SLOT_MOM];
  m->mom_chunk = std::max(1, h.iters - 1);
  if (stats) {
    stats->mom_iters = h.iters;
    stats->mom_relres = 0.0;
    for (int c = 0; c < 2; c++)
      stats->mom_relres = std::max(stats->mom_relres, h.bnorm[c] > 0 ? h.rnorm[c] / h.bnorm[c] : 0.0);
  }
  return status_of(h);
}

// ------------------------------------------------------------------ step 2
cgp_status drv_restrict(cgp_mesh *m, const double *ut, double *bc) {
  hipStream_t s = m->stream;
  const double sc = -m->params.rho / m->params.dt;
  if (m->params.restrict_mode == CGP_RESTRICT_INJECT || m->levels == 0) {
    const int n = m->pc.n, L = m->lanes_c;
    dispatch_L(L, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_div<LL>), dim3(grid_for((long long)n * LL)), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c,
                         (const double2 *)m->d_Dc, (const double2 *)ut, sc, bc);
    });
  } else {
    const int n = m->pf.n, L = m->lanes_f;
    double *bf = m->d_wlev[m->levels];
    dispatch_L(L, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_div<LL>), dim3(grid_for((long long)n * LL)), dim3(256), 0, s, n, m->d_rp_f, m->d_col_f,
                         (const double2 *)m->d_D, (const double2 *)ut, sc, bf);
    });
    for (int lv = m->levels; lv >= 1; lv--) {
      const int nprev = m->lev[lv - 1].n;
      double *dst = (lv == 1) ? bc : m->d_wlev[lv - 1];
      hipLaunchKernelGGL(k_restrict_gather, dim3(blocks_1d(nprev)), dim3(256), 0, s, nprev, m->d_rt_ptr[lv],
                         m->d_rt_idx[lv], (const double *)m->d_wlev[lv], dst);
    }
  }
  CGP_HIP(hipGetLastError());
  return CGP_OK;
}

// ------------------------------------------------------------------ step 3
cgp_status drv_poisson(cgp_mesh *m, const double *b_in, double *x, const cgp_solver_opts *o, cgp_stats *stats) {
  hipStream_t s = m->stream;
  const int n = m->pc.n;
  double *b = m->d_wc[0];
  CGP_HIP(hipMemcpyAsync(b, b_in, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (o->x0_mode == CGP_X0_ZERO) CGP_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
  if (m->n_pdir > 0) {
    hipLaunchKernelGGL(k_pdir_zero, dim3(blocks_1d(n)), dim3(256), 0, s, n, m->d_pdir, b, x);
  } else {
    // pure Neumann (Eq. 13 on all of the boundary): project b onto the range of Kbar
    hipLaunchKernelGGL(k_wsum, dim3(grid_for(n)), dim3(256), 0, s, n, (const double *)nullptr, (const double *)b,
                       m->d_scalar, red(m));
    hipLaunchKernelGGL(k_shift, dim3(blocks_1d(n)), dim3(256), 0, s, n, b, (const double *)m->d_scalar, double(n));
  }
  KrylovState fin{};
  cgp_status rs = CGP_OK;
  int total_iters = 0, outer = 0;
  if (o->precision == CGP_PREC_FP64) {
    double *w[5] = {m->d_wc[1], m->d_wc[2], m->d_wc[3], m->d_wc[4], m->d_wc[5]};
    rs = run_pcg<1>(m, SLOT_P, n, m->d_rp_c, m->d_col_c, m->d_Kbc, m->d_dinvK, b, x, w, m->lanes_c, o->tol,
                    o->max_iter, &m->p_chunk, &fin);
    total_iters = fin.iters;
    outer = 1;
  } else {
    // FP32 Jacobi-PCG inside FP64 iterative refinement
    KrylovState *so = m->d_state + SLOT_P, *si = m->d_state + SLOT_PIN;
    Reduce R = red(m);
    double *r64 = m->d_wc[1];
    float *r = m->d_wc32[0], *z = m->d_wc32[1], *d = m->d_wc32[2], *p0 = m->d_wc32[3], *p1 = m->d_wc32[4],
          *q = m->d_wc32[5];
    const double inner_tol = o->inner_tol > 0 ? o->inner_tol : 1e-4;
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, so, o->tol, o->max_iter, 1);
    hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, si, inner_tol, o->max_iter, 1);
    const int L = m->lanes_c, gL = grid_for((long long)n * L), g1 = grid_for(n);
    for (outer = 0; outer < 200; outer++) {
      int it = 0, chunk = std::max(1, m->p32_chunk);
      dispatch_L(L, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_ir_residual<LL>), dim3(gL), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c,
                           (const double *)m->d_Kbc, (const double *)b, (const double *)x, r64, so, R);
      });
      hipLaunchKernelGGL(k_ir_inner_init, dim3(g1), dim3(256), 0, s, n, (const double *)r64,
                         (const float *)m->d_dinvK32, r, z, d, p0, p1, (const KrylovState *)so, si, R);
      for (;;) {
        dispatch_L(L, [&](auto LC) {
          constexpr int LL = decltype(LC)::value;
          for (int c = 0; c < chunk; c++, it++) {
            float *po = (it & 1) ? p1 : p0, *pn = (it & 1) ? p0 : p1;
            hipLaunchKernelGGL((k_cg32_spmv<LL>), dim3(gL), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c,
                               (const float *)m->d_Kbc32, (const float *)z, (const float *)po, pn, q, si, R);
            hipLaunchKernelGGL(k_cg32_update, dim3(g1), dim3(256), 0, s, n, d, r, z, (const float *)m->d_dinvK32,
                               (const float *)pn, (const float *)q, si, R);
          }
        });
        CGP_HIP(hipGetLastError());
        cgp_status ps = poll(m, SLOT_P, 2);
        if (ps) return ps;
        const KrylovState &hi = m->h_state[SLOT_PIN];
        if (hi.done[0] || hi.status) break;
        chunk = 8;
      }
      const KrylovState ho = m->h_state[SLOT_P], hi = m->h_state[SLOT_PIN];
      if (ho.done[0] || ho.status) { fin = ho; break; }
      m->p32_chunk = std::max(1, hi.iters - 2);
      total_iters += hi.iters;
      if (hi.status) { fin = hi; break; }
      hipLaunchKernelGGL(k_ir_update, dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const float *)d,
                         (const KrylovState *)so);
      if (total_iters >= o->max_iter) {
        // final residual to report
        dispatch_L(L, [&](auto LC) {
          constexpr int LL = decltype(LC)::value;
          hipLaunchKernelGGL((k_ir_residual<LL>), dim3(gL), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c,
                             (const double *)m->d_Kbc, (const double *)b, (const double *)x, r64, so, R);
        });
        cgp_status ps = poll(m, SLOT_P);
        if (ps) return ps;
        fin = m->h_state[SLOT_P];
        outer++;
        break;
      }
    }
    hipLaunchKernelGGL((k_zero_b_fix<1>), dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const KrylovState *)so);
    rs = status_of(fin);
  }
  if (m->n_pdir == 0) {
    // zero lumped-mass-weighted mean
    hipLaunchKernelGGL(k_wsum, dim3(grid_for(n)), dim3(256), 0, s, n, (const double *)m->d_mc, (const double *)x,
                       m->d_scalar, red(m));
    hipLaunchKernelGGL(k_shift, dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const double *)m->d_scalar, m->mc_sum);
  }
  CGP_HIP(hipGetLastError());
  if (stats) {
    stats->p_iters = total_iters;
    stats->p_outer = outer;
    stats->p_relres = fin.bnorm[0] > 0 ? fin.rnorm[0] / fin.bnorm[0] : 0.0;
  }
  return rs;
}

// ------------------------------------------------------------------ step 4
cgp_status drv_prolong(cgp_mesh *m, const double *pc, double *pf) {
  hipStream_t s = m->stream;
  if (m->levels == 0) {
    CGP_HIP(hipMemcpyAsync(pf, pc, m->pc.n * sizeof(double), hipMemcpyDeviceToDevice, s));
    return CGP_OK;
  }
  const double *src = pc;
  for (int lv = 1; lv <= m->levels; lv++) {
    const int nprev = m->lev[lv - 1].n, nk = m->lev[lv].n;
    double *dst = (lv == m->levels) ? pf : m->d_wlev[lv];
    hipLaunchKernelGGL(k_prolong, dim3(blocks_1d(nk)), dim3(256), 0, s, nprev, nk, (const int2 *)m->d_parent[lv], src,
                       dst);
    src = dst;
  }
  CGP_HIP(hipGetLastError());
  return CGP_OK;
}

// ------------------------------------------------------------------ step 5
cgp_status drv_correct(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *ut, const double *pf,
                       double *u, cgp_stats *stats) {
  hipStream_t s = m->stream;
  const int n = m->pf.n, L = m->lanes_f;
  const double sc = m->params.dt / m->params.rho;
  if (m->params.mass_mode == CGP_MASS_LUMPED) {
    dispatch_L(L, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_correct_lumped<LL>), dim3(grid_for((long long)n * LL)), dim3(256), 0, s, n, m->d_rp_f,
                         m->d_col_f, m->d_vdir, (const double2 *)m->d_D, (const double2 *)ut, pf, m->d_ml,
                         (const double2 *)g, sc, (double2 *)u);
    });
    CGP_HIP(hipGetLastError());
    if (stats) { stats->mass_iters = 0; stats->mass_relres = 0.0; }
    return CGP_OK;
  }
  double *rhs = m->d_wf[0];
  dispatch_L(L, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    hipLaunchKernelGGL((k_correct_rhs<LL>), dim3(grid_for((long long)n * LL)), dim3(256), 0, s, n, m->d_rp_f,
                       m->d_col_f, m->d_vdir, m->d_M, (const double2 *)m->d_D, (const double2 *)ut, pf,
                       (const double2 *)g, sc, (double2 *)rhs);
  });
  if (o->x0_mode == CGP_X0_ZERO)
    CGP_HIP(hipMemsetAsync(u, 0, 2 * n * sizeof(double), s));
  else
    CGP_HIP(hipMemcpyAsync(u, ut, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  double *w[5] = {m->d_wf[1], m->d_wf[2], m->d_wf[3], m->d_wf[4], m->d_wf[5]};
  KrylovState fin{};
  cgp_status rs = run_pcg<2>(m, SLOT_MASS, n, m->d_rp_f, m->d_col_f, m->d_Mbc, m->d_dinvM, rhs, u, w, L, o->tol,
                             o->max_iter, &m->mass_chunk, &fin);
  hipLaunchKernelGGL(k_set_dirichlet, dim3(blocks_1d(n)), dim3(256), 0, s, n, m->d_vdir, (const double2 *)g,
                     (double2 *)u);
  CGP_HIP(hipGetLastError());
  if (stats) {
    stats->mass_iters = fin.iters;
    stats->mass_relres = 0.0;
    for (int c = 0; c < 2; c++)
      stats->mass_relres = std::max(stats->mass_relres, fin.bnorm[c] > 0 ? fin.rnorm[c] / fin.bnorm[c] : 0.0);
  }
  return rs;
}

// ------------------------------------------------------------------ operators
cgp_status drv_spmv(cgp_mesh *m, int op, const void *x, void *y) {
  hipStream_t s = m->stream;
  switch (op) {
    case CGP_OP_KBC_C:
      dispatch_L(m->lanes_c, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_spmv1<LL>), dim3(grid_for((long long)m->pc.n * LL)), dim3(256), 0, s, m->pc.n,
                           m->d_rp_c, m->d_col_c, (const double *)m->d_Kbc, (const double *)x, (double *)y);
      });
      break;
    case CGP_OP_KBC_C32:
      dispatch_L(m->lanes_c, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_spmv1_f32<LL>), dim3(grid_for((long long)m->pc.n * LL)), dim3(256), 0, s, m->pc.n,
                           m->d_rp_c, m->d_col_c, (const float *)m->d_Kbc32, (const float *)x, (float *)y);
      });
      break;
    case CGP_OP_M_F:
    case CGP_OP_A_F:
      dispatch_L(m->lanes_f, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_spmv2<LL>), dim3(grid_for((long long)m->pf.n * LL)), dim3(256), 0, s, m->pf.n,
                           m->d_rp_f, m->d_col_f, (const double *)(op == CGP_OP_M_F ? m->d_M : m->d_A),
                           (const double2 *)x, (double2 *)y);
      });
      break;
    default:
      set_error("cgp_spmv: unknown operator");
      return CGP_E_ARG;
  }
  CGP_HIP(hipGetLastError());
  return CGP_OK;
}

}  // namespace cgp
