// Device kernels of libcgp for gfx950 (CDNA4, wave64): element assembly,
// CSR SpMV and the grid-transfer / pressure-path kernels, with their host
// launchers.  The Krylov solvers live in krylov.hip.
//
// Everything here is memory-bound.  The static element assembly scatters into
// CSR values colour by colour (elements of one colour share no node, so no
// atomics and a fixed summation order); the per-step momentum matrix is formed
// entry by entry from a node-to-element list instead (one launch, no scatter);
// CSR kernels give each row a group of L lanes so that
// one wavefront streams 64/L consecutive rows with coalesced value and column
// loads; grid-transfer kernels are gathers over index tables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "devutil.h"
#include "kernels.h"

namespace cgp {
namespace dev {

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

// Momentum matrix A = S + dt N(U^n), N_ab = rho/24 [(u_a + sum u) b_b + (v_a + sum v) c_b], formed
// per row: a group of L lanes takes row i, each lane one element around i (vertex triples,
// contiguous per row in element order; more than L elements are taken L at a time) and forms
// that element's row (u_i + sum u) b + (v_i + sum v) c.  For each entry (i, j) of the row the
// group sums, in a fixed butterfly order, what the elements containing j contribute, and lane
// (s mod L) keeps the total of the row's s-th entry; every entry is written once, from S.
template <int L>
__global__ void k_asm_conv_rows(int n, const int *__restrict__ rp, const int *__restrict__ col,
                                const double *__restrict__ S, const int *__restrict__ inc_ptr,
                                const int4 *__restrict__ incv, const double2 *__restrict__ xy,
                                const double2 *__restrict__ u, double dtrho24, double *__restrict__ A) {
  const int lane = threadIdx.x & (L - 1);
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) / L;
  if (row >= n) return;  // the whole group
  const int k0 = rp[row], deg = rp[row + 1] - k0, p0 = inc_ptr[row], p1 = inc_ptr[row + 1];
  const double2 ui = u[row];
  for (int s0 = 0; s0 < deg; s0 += 2 * L) {  // entries s0 .. s0 + 2L - 1 of the row
    double acc0 = 0.0, acc1 = 0.0;          // totals of entries s0 + lane and s0 + L + lane
    for (int q0 = p0; q0 < p1; q0 += L) {
      const int q = q0 + lane;
      int4 v = make_int4(-1, -1, -1, 0);
      double cb[3] = {0.0, 0.0, 0.0};
      if (q < p1) {
        v = incv[q];
        const Geo g = geometry(xy, v.x, v.y, v.z);
        const double2 u0 = u[v.x], u1 = u[v.y], u2 = u[v.z];
        const double ua = ui.x + (u0.x + u1.x + u2.x), va = ui.y + (u0.y + u1.y + u2.y);
#pragma unroll
        for (int b = 0; b < 3; b++) cb[b] = ua * g.b[b] + va * g.c[b];
      }
      const int s1 = min(deg, s0 + 2 * L);
      for (int s = s0; s < s1; s++) {
        const int j = col[k0 + s];
        double c = (v.x == j) ? cb[0] : (v.y == j) ? cb[1] : (v.z == j) ? cb[2] : 0.0;
        c = group_sum<L>(c);
        if (s - s0 == lane) acc0 += c;
        if (s - s0 == L + lane) acc1 += c;
      }
    }
    if (s0 + lane < deg) A[k0 + s0 + lane] = S[k0 + s0 + lane] + dtrho24 * acc0;
    if (s0 + L + lane < deg) A[k0 + s0 + L + lane] = S[k0 + s0 + L + lane] + dtrho24 * acc1;
  }
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

// Fine mass with velocity-Dirichlet rows/columns cleared except for the diagonal, which keeps
// its value; its Jacobi inverse; lumped mass.
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
    double v = (di || vdir[j]) ? (i == j ? (M[k] > 0.0 ? M[k] : 1.0) : 0.0) : M[k];
    Mbc[k] = v;
    if (j == i) d = v;
  }
  dinv[i] = d != 0.0 ? 1.0 / d : 1.0;
  ml[i] = s;
}

// Momentum right-hand side rho M U^n + dt M F (- dt G P_f^n with GRAD, the incremental pressure
// modes) with symmetric Dirichlet elimination of g on the fixed pattern, and the Jacobi inverse of A;
// a group of L lanes per row, group sums in a fixed order.
template <int L, bool GRAD>
__global__ void k_mom_rhs_bc(int n, const int *__restrict__ rp, const int *__restrict__ col,
                             const unsigned char *__restrict__ vdir, const double *__restrict__ M,
                             double *__restrict__ A, const double2 *__restrict__ g, const double2 *__restrict__ u,
                             const double2 *__restrict__ f, const double2 *__restrict__ D,
                             const double *__restrict__ pn, double rho, double dt, double2 *__restrict__ rhs,
                             double *__restrict__ dinv) {
  const int lane = threadIdx.x & (L - 1);
  const int j = (blockIdx.x * blockDim.x + threadIdx.x) / L;
  if (j >= n) return;  // the whole group
  const int k0 = rp[j], k1 = rp[j + 1];
  if (vdir[j]) {  // the row keeps its diagonal a_jj (1 if not positive): a_jj u_j = a_jj g_j
    double a = 0.0;
    for (int k = k0 + lane; k < k1; k += L)
      if (col[k] == j) a = A[k];
    a = group_sum<L>(a);
    const double d = a > 0.0 ? a : 1.0;
    for (int k = k0 + lane; k < k1; k += L) A[k] = (col[k] == j) ? d : 0.0;
    if (lane == 0) {
      const double2 gj = g[j];
      rhs[j] = make_double2(d * gj.x, d * gj.y);
      dinv[j] = 1.0 / d;
    }
    return;
  }
  double ax = 0.0, ay = 0.0, fx = 0.0, fy = 0.0, gx = 0.0, gy = 0.0, d = 0.0, px = 0.0, py = 0.0;
  for (int k = k0 + lane; k < k1; k += L) {
    const int c = col[k];
    const double m = M[k];
    const double2 uc = u[c];
    ax += m * uc.x;
    ay += m * uc.y;
    if (GRAD) {
      const double2 dk = D[k];
      const double pc = pn[c];
      px += dk.x * pc;
      py += dk.y * pc;
    }
    if (f) {
      const double2 fc = f[c];
      fx += m * fc.x;
      fy += m * fc.y;
    }
    if (vdir[c]) {
      const double a = A[k];
      const double2 gc = g[c];
      gx += a * gc.x;
      gy += a * gc.y;
      A[k] = 0.0;
    } else if (c == j) {
      d = A[k];
    }
  }
  ax = group_sum<L>(ax);
  ay = group_sum<L>(ay);
  gx = group_sum<L>(gx);
  gy = group_sum<L>(gy);
  d = group_sum<L>(d);  // one lane holds the diagonal
  if (f) {
    fx = group_sum<L>(fx);
    fy = group_sum<L>(fy);
  }
  if (GRAD) {
    px = group_sum<L>(px);
    py = group_sum<L>(py);
  }
  if (lane == 0) {
    double rx = rho * ax, ry = rho * ay;
    if (f) {
      rx += dt * fx;
      ry += dt * fy;
    }
    if (GRAD) {
      rx -= dt * px;
      ry -= dt * py;
    }
    rhs[j] = make_double2(rx - gx, ry - gy);
    dinv[j] = d != 0.0 ? 1.0 / d : 1.0;
  }
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

// x0 = 2 a - b, b = a (element-wise over `count` values)
__global__ void k_extrapolate(long count, double *__restrict__ a, double *__restrict__ b) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double ai = a[i];
  a[i] = 2.0 * ai - b[i];
  b[i] = ai;
}

// x0 = 3 a - 3 b + c, then c = b, b = a (element-wise over `count` values)
__global__ void k_extrapolate3(long count, double *__restrict__ a, double *__restrict__ b, double *__restrict__ c) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double ai = a[i], bi = b[i];
  a[i] = 3.0 * (ai - bi) + c[i];
  c[i] = bi;
  b[i] = ai;
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

// Partials of sum_i w[i] x[i] (w = NULL: plain sum), one per block.
__global__ void __launch_bounds__(kMaxBlock) k_wsum(int n, const double *__restrict__ w, const double *__restrict__ x,
                                                    double *__restrict__ P) {
  double acc[1] = {0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) acc[0] += (w ? w[i] : 1.0) * x[i];
  put_partials<1>(acc, P);
}

// x -= (sum of the G partials) / den
__global__ void __launch_bounds__(kMaxBlock) k_shift(int n, double *__restrict__ x, const double *__restrict__ P,
                                                     int G, double den) {
  double tot[1];
  sum_partials<1>(P, G, tot);
  const double s = tot[0] / den;
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] -= s;
}

// *out = sum of the G partials (one block)
__global__ void __launch_bounds__(kMaxBlock) k_reduce_scalar(const double *__restrict__ P, int G,
                                                             double *__restrict__ out) {
  double tot[1];
  sum_partials<1>(P, G, tot);
  if (threadIdx.x == 0) *out = tot[0];
}

// Correction right-hand side (Eq. 23): M u~ - (dt/rho)(Dx P, Dy P), lifted with g; m_ii g_i on
// velocity-Dirichlet rows.
template <int L>
__global__ void k_correct_rhs(int n, const int *__restrict__ rp, const int *__restrict__ col,
                              const unsigned char *__restrict__ vdir, const double *__restrict__ M,
                              const double2 *__restrict__ D, const double2 *__restrict__ ut,
                              const double *__restrict__ pf, const double2 *__restrict__ g, double s,
                              double2 *__restrict__ rhs) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double mx = 0.0, my = 0.0, gx = 0.0, gy = 0.0, lx = 0.0, ly = 0.0, md = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const int c = col[k];
      const double m = M[k];
      const double2 u = ut[c], d = D[k];
      const double p = pf[c];
      mx += m * u.x;
      my += m * u.y;
      gx += d.x * p;
      gy += d.y * p;
      if (c == row) md = m;
      if (vdir[c]) {
        const double2 gc = g[c];
        lx += m * gc.x;
        ly += m * gc.y;
      }
    }
    mx = group_sum<L>(mx); my = group_sum<L>(my);
    gx = group_sum<L>(gx); gy = group_sum<L>(gy);
    lx = group_sum<L>(lx); ly = group_sum<L>(ly);
    md = group_sum<L>(md);
    if (lane == 0) {
      if (vdir[row]) {  // m_ii u_i = m_ii g_i, as the eliminated mass matrix keeps m_ii
        const double d = md > 0.0 ? md : 1.0;
        const double2 gr = g[row];
        rhs[row] = make_double2(d * gr.x, d * gr.y);
      } else {
        rhs[row] = make_double2(mx - s * gx - lx, my - s * gy - ly);
      }
    }
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

// New coarse pressure of the incremental modes: pc + phi, minus (rotational) mu times the restricted
// divergence of U~ over the lumped mass; bc = -(rho/dt) (restricted divergence), so the rotational
// term is + (mu dt / rho) bc / m_c.  Pressure-Dirichlet nodes stay 0.
__global__ void k_pressure_update(int n, const unsigned char *__restrict__ pdir, const double *__restrict__ phi,
                                  const double *__restrict__ bc, const double *__restrict__ mc, double rot,
                                  double *__restrict__ pc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pc[i] = pdir[i] ? 0.0 : pc[i] + phi[i] + rot * bc[i] / mc[i];
}

// Force of the fluid on a marked boundary surface, one fine boundary edge e = (a, b) per thread, with
// c the third vertex of its triangle: n the unit normal of e towards c (into the fluid), the stress
// -p I + mu (grad u + grad u^T) of the P1 fields; the edge carries -|e| (p_a + p_b)/2 n (pressure) and
// |e| mu (grad u + grad u^T) n (viscous).  One block: per-edge rows (x, y, |e|, pressure x, y,
// viscous x, y, 0) when `rows` is set, and the four totals summed in a fixed order into `tot`.
__global__ void __launch_bounds__(1024) k_surface(int ne, const int4 *__restrict__ e, const double2 *__restrict__ xy,
                                                  const double2 *__restrict__ u, const double *__restrict__ p,
                                                  double mu, double *__restrict__ rows, double *__restrict__ tot) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < ne; i += blockDim.x) {
    const int4 v = e[i];
    const double2 xa = xy[v.x], xb = xy[v.y], xc = xy[v.z];
    const double ex = xb.x - xa.x, ey = xb.y - xa.y;
    const double len = sqrt(ex * ex + ey * ey);
    double nx = -ey / len, ny = ex / len;
    if (nx * (xc.x - xa.x) + ny * (xc.y - xa.y) < 0.0) {
      nx = -nx;
      ny = -ny;
    }
    // P1 gradient on (a, b, c): grad phi_k = (y_j - y_l, x_l - x_j) / (2A) with (k, j, l) cyclic
    const double a2 = (xb.x - xa.x) * (xc.y - xa.y) - (xc.x - xa.x) * (xb.y - xa.y);
    const double2 ua = u[v.x], ub = u[v.y], uc = u[v.z];
    const double ga_x = (xb.y - xc.y) / a2, ga_y = (xc.x - xb.x) / a2;
    const double gb_x = (xc.y - xa.y) / a2, gb_y = (xa.x - xc.x) / a2;
    const double gc_x = (xa.y - xb.y) / a2, gc_y = (xb.x - xa.x) / a2;
    const double uxx = ua.x * ga_x + ub.x * gb_x + uc.x * gc_x, uxy = ua.x * ga_y + ub.x * gb_y + uc.x * gc_y;
    const double uyx = ua.y * ga_x + ub.y * gb_x + uc.y * gc_x, uyy = ua.y * ga_y + ub.y * gb_y + uc.y * gc_y;
    const double pm = 0.5 * (p[v.x] + p[v.y]);
    const double sxx = 2.0 * uxx, syy = 2.0 * uyy, sxy = uxy + uyx;
    const double fpx = -len * pm * nx, fpy = -len * pm * ny;
    const double fvx = len * mu * (sxx * nx + sxy * ny), fvy = len * mu * (sxy * nx + syy * ny);
    acc[0] += fpx;
    acc[1] += fpy;
    acc[2] += fvx;
    acc[3] += fvy;
    if (rows) {
      double *o = rows + 8 * (size_t)i;
      o[0] = 0.5 * (xa.x + xb.x);
      o[1] = 0.5 * (xa.y + xb.y);
      o[2] = len;
      o[3] = fpx;
      o[4] = fpy;
      o[5] = fvx;
      o[6] = fvy;
      o[7] = 0.0;
    }
  }
  double t[4];
  block_sum<4>(acc, t);
  if (threadIdx.x < 4) tot[threadIdx.x] = t[threadIdx.x];
}

__global__ void k_set_dirichlet(int n, const unsigned char *__restrict__ vdir, const double2 *__restrict__ g,
                                double2 *__restrict__ u) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (vdir[i]) u[i] = g[i];
}


}  // namespace dev

// ====================================================================== host launchers
using namespace dev;

void launch_conv_assembly(cgp_mesh *m, const double *u) {
  constexpr int L = 8;  // lanes per row: P1 rows hold about seven entries
  const double dtrho24 = m->params.dt * m->params.rho / 24.0;
  const int n = m->pf.n;
  hipLaunchKernelGGL((k_asm_conv_rows<L>), dim3(blocks_1d((long long)n * L)), dim3(256), 0, m->stream, n, m->d_rp_f,
                     m->d_col_f, (const double *)m->d_S, m->d_inc_ptr_f, (const int4 *)m->d_incv_f,
                     (const double2 *)m->d_xy_f, (const double2 *)u, dtrho24, m->d_A);
}

void launch_mom_rhs(cgp_mesh *m, const double *g, const double *u, const double *f, const double *pn, double *rhs) {
  const int n = m->pf.n;
  constexpr int L = 8;
  auto kern = pn ? k_mom_rhs_bc<L, true> : k_mom_rhs_bc<L, false>;
  hipLaunchKernelGGL(kern, dim3(blocks_1d((long long)n * L)), dim3(256), 0, m->stream, n, m->d_rp_f,
                     m->d_col_f, m->d_vdir,
                     m->d_M, m->d_A, (const double2 *)g, (const double2 *)u, (const double2 *)f,
                     (const double2 *)m->d_D, pn, m->params.rho, m->params.dt, (double2 *)rhs, m->d_dinvA);
}

void launch_surface(cgp_mesh *m, const double *u, const double *p, double *rows) {
  hipLaunchKernelGGL(k_surface, dim3(1), dim3(1024), 0, m->stream, m->n_surf, (const int4 *)m->d_surf,
                     (const double2 *)m->d_xy_f, (const double2 *)u, p, m->params.mu, rows, m->d_scalar);
}

void launch_pressure_update(cgp_mesh *m, double *pc, const double *phi, const double *bc) {
  const int n = m->pc.n;
  const double rot = m->params.pressure_mode == CGP_PRESSURE_ROTATIONAL
                         ? m->params.mu * m->params.dt / m->params.rho : 0.0;
  hipLaunchKernelGGL(k_pressure_update, dim3(blocks_1d(n)), dim3(256), 0, m->stream, n, m->d_pdir, phi, bc,
                     (const double *)m->d_mc, rot, pc);
  if (rot != 0.0 && m->n_pdir == 0) launch_mean_shift(m, pc, m->d_mc, m->mc_sum, m->red.partials);
}

void launch_correct_rhs(cgp_mesh *m, const double *g, const double *ut, const double *pf, double *rhs) {
  const int n = m->pf.n;
  const double sc = m->params.dt / m->params.rho;
  dispatch_L(m->tune.fine.lanes, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    hipLaunchKernelGGL((k_correct_rhs<LL>), dim3(grid_for((long long)n * LL)), dim3(256), 0, m->stream, n, m->d_rp_f,
                       m->d_col_f, m->d_vdir, m->d_M, (const double2 *)m->d_D, (const double2 *)ut, pf,
                       (const double2 *)g, sc, (double2 *)rhs);
  });
}

void launch_correct_lumped(cgp_mesh *m, const double *g, const double *ut, const double *pf, double *u) {
  const int n = m->pf.n;
  const double sc = m->params.dt / m->params.rho;
  dispatch_L(m->tune.fine.lanes, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    hipLaunchKernelGGL((k_correct_lumped<LL>), dim3(grid_for((long long)n * LL)), dim3(256), 0, m->stream, n,
                       m->d_rp_f, m->d_col_f, m->d_vdir, (const double2 *)m->d_D, (const double2 *)ut, pf, m->d_ml,
                       (const double2 *)g, sc, (double2 *)u);
  });
}

void launch_set_dirichlet(cgp_mesh *m, const double *g, double *u) {
  const int n = m->pf.n;
  hipLaunchKernelGGL(k_set_dirichlet, dim3(blocks_1d(n)), dim3(256), 0, m->stream, n, m->d_vdir,
                     (const double2 *)g, (double2 *)u);
}

void launch_extrapolate(cgp_mesh *m, long count, double *a, double *b) {
  hipLaunchKernelGGL(dev::k_extrapolate, dim3((count + 255) / 256), dim3(256), 0, m->stream, count, a, b);
}

void launch_extrapolate3(cgp_mesh *m, long count, double *a, double *b, double *c) {
  hipLaunchKernelGGL(dev::k_extrapolate3, dim3((count + 255) / 256), dim3(256), 0, m->stream, count, a, b, c);
}

void launch_pdir_zero(cgp_mesh *m, double *b, double *x) {
  const int n = m->pc.n;
  hipLaunchKernelGGL(k_pdir_zero, dim3(blocks_1d(n)), dim3(256), 0, m->stream, n, m->d_pdir, b, x);
}

void launch_mean_shift(cgp_mesh *m, double *x, const double *w, double den, double *P) {
  const int n = m->pc.n, G = 256;
  hipLaunchKernelGGL(k_wsum, dim3(G), dim3(256), 0, m->stream, n, w, (const double *)x, P);
  hipLaunchKernelGGL(k_shift, dim3(G), dim3(256), 0, m->stream, n, x, (const double *)P, G, den);
}


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
  hipLaunchKernelGGL(k_wsum, dim3(256), dim3(256), 0, s, Nc, (const double *)nullptr, (const double *)m->d_mc,
                     m->red.partials);
  hipLaunchKernelGGL(k_reduce_scalar, dim3(1), dim3(256), 0, s, (const double *)m->red.partials, 256, m->d_scalar);
  CGP_HIP(hipGetLastError());
  CGP_HIP(hipMemcpyAsync(&m->h_scalar[0], m->d_scalar, sizeof(double), hipMemcpyDeviceToHost, s));
  CGP_HIP(hipStreamSynchronize(s));
  m->mc_sum = m->h_scalar[0];
  return CGP_OK;
}

// ------------------------------------------------------------------ step 2
cgp_status drv_restrict(cgp_mesh *m, const double *ut, double *bc) {
  hipStream_t s = m->stream;
  const double sc = -m->params.rho / m->params.dt;
  if (m->params.restrict_mode == CGP_RESTRICT_INJECT || m->levels == 0) {
    const int n = m->pc.n, L = m->tune.coarse.lanes;
    dispatch_L(L, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_div<LL>), dim3(grid_for((long long)n * LL)), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c,
                         (const double2 *)m->d_Dc, (const double2 *)ut, sc, bc);
    });
  } else {
    const int n = m->pf.n, L = m->tune.fine.lanes;
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

// ------------------------------------------------------------------ operators
cgp_status drv_spmv(cgp_mesh *m, int op, const void *x, void *y) {
  hipStream_t s = m->stream;
  switch (op) {
    case CGP_OP_KBC_C:
      dispatch_L(m->tune.coarse.lanes, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_spmv1<LL>), dim3(grid_for((long long)m->pc.n * LL)), dim3(256), 0, s, m->pc.n,
                           m->d_rp_c, m->d_col_c, (const double *)m->d_Kbc, (const double *)x, (double *)y);
      });
      break;
    case CGP_OP_KBC_C32:
      dispatch_L(m->tune.coarse.lanes, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_spmv1_f32<LL>), dim3(grid_for((long long)m->pc.n * LL)), dim3(256), 0, s, m->pc.n,
                           m->d_rp_c, m->d_col_c, (const float *)m->d_Kbc32, (const float *)x, (float *)y);
      });
      break;
    case CGP_OP_M_F:
    case CGP_OP_A_F:
      dispatch_L(m->tune.fine.lanes, [&](auto LC) {
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
