// The paper's linear solver for the coarse pressure Poisson equation (Eq. 21; Section 2.3,
// "Computational implementation"): GMRES(m) with an ILU(0) preconditioner on the CSR matrix.
//
// ILU(0) keeps the pattern of Kbar: for every row i in order and every column k < i of row i in
// increasing order, l_ik = a_ik / u_kk and each later entry (i, j) that also exists in row k loses
// l_ik u_kj.  Row i needs only rows k < i that it touches, so the rows fall into levels (level(i) =
// 1 + the largest level of those rows): all rows of a level are factored, and solved in the forward
// substitution, at once, one launch per level; the backward substitution uses the mirrored levels.
// The levels come from the pattern alone (host, once per mesh); the factorisation runs on the device
// after each cgp_assemble, at the first GMRES solve.
//
// GMRES(m) with right preconditioning: x = x0 + M^-1 V y.  Each Arnoldi step applies M^-1 and Kbar,
// orthogonalises against the basis by classical Gram-Schmidt done twice (two fused multi-dot passes
// in place of j sequential dots), and rotates the Hessenberg column on the host (Givens).  The
// rotated right-hand side estimates ||b - Kbar x|| inside a cycle; the true residual is formed at
// every restart and decides convergence.  Slower than the fused Jacobi-PCG on this hardware (the
// triangular solves are chains of dependent levels); it serves the paper's iteration counts.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "devutil.h"
#include "internal.h"
#include "kernels.h"

#define TRYS(x)                   \
  do {                            \
    const cgp_status s_ = (x);    \
    if (s_ != CGP_OK) return s_;  \
  } while (0)

namespace cgp {
namespace gdev {

constexpr int kMultiBlocks = 256;

// factor the rows of one level (one thread per row); diag[i] = index of (i, i) in the pattern
__global__ void k_ilu_factor(int count, const int *__restrict__ rows, const int *__restrict__ rp,
                             const int *__restrict__ col, const int *__restrict__ diag, double *__restrict__ lu) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int i = rows[t];
  const int e = rp[i + 1];
  for (int kk = rp[i]; kk < e; kk++) {
    const int k = col[kk];
    if (k >= i) break;
    const double lik = lu[kk] / lu[diag[k]];
    lu[kk] = lik;
    // entries j > k of row i against the upper part of row k (both sorted): a merge
    int kj = diag[k] + 1;
    const int ke = rp[k + 1];
    for (int jj = kk + 1; jj < e && kj < ke; jj++) {
      const int j = col[jj];
      while (kj < ke && col[kj] < j) kj++;
      if (kj < ke && col[kj] == j) lu[jj] -= lik * lu[kj];
    }
  }
}

// forward substitution with the unit lower factor over the rows of one level: z_i = r_i - sum l_ik z_k
__global__ void k_ilu_lower(int count, const int *__restrict__ rows, const int *__restrict__ rp,
                            const int *__restrict__ col, const int *__restrict__ diag, const double *__restrict__ lu,
                            const double *__restrict__ r, double *__restrict__ z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int i = rows[t];
  double s = r[i];
  for (int k = rp[i]; k < diag[i]; k++) s -= lu[k] * z[col[k]];
  z[i] = s;
}

// backward substitution with the upper factor over the rows of one level: z_i = (z_i - sum u_ij z_j) / u_ii
__global__ void k_ilu_upper(int count, const int *__restrict__ rows, const int *__restrict__ rp,
                            const int *__restrict__ col, const int *__restrict__ diag, const double *__restrict__ lu,
                            double *__restrict__ z) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const int i = rows[t];
  const int d = diag[i];
  double s = z[i];
  for (int k = d + 1; k < rp[i + 1]; k++) s -= lu[k] * z[col[k]];
  z[i] = s / lu[d];
}

// block partials of V[c] . w for c < J (V row-major [J][n]): P[c][blockIdx]
__global__ void __launch_bounds__(256) k_multidot(int n, int J, const double *__restrict__ V,
                                                  const double *__restrict__ w, double *__restrict__ P) {
  __shared__ double sh[4];
  for (int c = 0; c < J; c++) {
    const double *v = V + (size_t)c * n;
    double s = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) s += v[i] * w[i];
    s = dev::wave_sum(s);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) P[(size_t)c * gridDim.x + blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
  }
}

// w -= sum_c h[c] V[c]
__global__ void k_sub_combination(int n, int J, const double *__restrict__ V, const double *__restrict__ h,
                                  double *__restrict__ w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = w[i];
  for (int c = 0; c < J; c++) s -= h[c] * V[(size_t)c * n + i];
  w[i] = s;
}

// out = sum_c y[c] V[c]
__global__ void k_combination(int n, int J, const double *__restrict__ V, const double *__restrict__ y,
                              double *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < J; c++) s += y[c] * V[(size_t)c * n + i];
  out[i] = s;
}

// r = b - K x
__global__ void k_residual(int n, const int *__restrict__ rp, const int *__restrict__ col,
                           const double *__restrict__ K, const double *__restrict__ b, const double *__restrict__ x,
                           double *__restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; k++) s += K[k] * x[col[k]];
  r[i] = b[i] - s;
}

__global__ void k_matvec(int n, const int *__restrict__ rp, const int *__restrict__ col, const double *__restrict__ K,
                         const double *__restrict__ x, double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; k++) s += K[k] * x[col[k]];
  y[i] = s;
}

__global__ void k_scale_into(int n, double a, const double *__restrict__ x, double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

__global__ void k_add(int n, const double *__restrict__ x, double *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += x[i];
}

}  // namespace gdev

namespace {

using namespace gdev;

// Levels of the lower (ascending) and upper (descending) dependence of the coarse pattern, and the
// diagonal positions; device copies.  Pattern-only: once per mesh.
cgp_status gmres_setup(cgp_mesh *m, int restart) {
  const int n = m->pc.n;
  auto alloc = [&](void **p, size_t bytes) -> cgp_status {
    if (hipMalloc(p, bytes) != hipSuccess) {
      set_error("GMRES: out of device memory");
      return CGP_E_OOM;
    }
    m->allocations.push_back(*p);
    return CGP_OK;
  };
  if (!m->gm.ready) {
    const std::vector<int> &rp = m->pc.rp, &col = m->pc.col;
    std::vector<int> diag(n, -1), lev(n, 0);
    for (int i = 0; i < n; i++)
      for (int k = rp[i]; k < rp[i + 1]; k++)
        if (col[k] == i) diag[i] = k;
    for (int i = 0; i < n; i++)
      if (diag[i] < 0) {
        set_error("GMRES: the coarse pattern lacks a diagonal entry");
        return CGP_E_STATE;
      }
    int nl = 0;
    for (int i = 0; i < n; i++) {
      int l = 0;
      for (int k = rp[i]; k < diag[i]; k++) l = std::max(l, lev[col[k]] + 1);
      lev[i] = l;
      nl = std::max(nl, l + 1);
    }
    auto bucket = [&](const std::vector<int> &lv, int nlev, std::vector<int> &rows, std::vector<int> &ptr) {
      ptr.assign(nlev + 1, 0);
      for (int i = 0; i < n; i++) ptr[lv[i] + 1]++;
      for (int l = 0; l < nlev; l++) ptr[l + 1] += ptr[l];
      rows.assign(n, 0);
      std::vector<int> fill(ptr.begin(), ptr.end() - 1);
      for (int i = 0; i < n; i++) rows[fill[lv[i]]++] = i;
    };
    std::vector<int> lrows, urows;
    bucket(lev, nl, lrows, m->gm.lptr);
    std::vector<int> ulev(n, 0);
    int nu = 0;
    for (int i = n - 1; i >= 0; i--) {
      int l = 0;
      for (int k = diag[i] + 1; k < rp[i + 1]; k++) l = std::max(l, ulev[col[k]] + 1);
      ulev[i] = l;
      nu = std::max(nu, l + 1);
    }
    bucket(ulev, nu, urows, m->gm.uptr);
    void *p = nullptr;
    TRYS(alloc(&p, sizeof(int) * n));
    m->gm.d_diag = static_cast<int *>(p);
    TRYS(alloc(&p, sizeof(int) * n));
    m->gm.d_lrows = static_cast<int *>(p);
    TRYS(alloc(&p, sizeof(int) * n));
    m->gm.d_urows = static_cast<int *>(p);
    TRYS(alloc(&p, sizeof(double) * m->pc.nnz));
    m->gm.d_lu = static_cast<double *>(p);
    TRYS(alloc(&p, sizeof(double) * 3 * n));
    m->gm.d_work = static_cast<double *>(p);
    TRYS(alloc(&p, sizeof(double) * kMultiBlocks * 2 * 256));
    m->gm.d_part = static_cast<double *>(p);
    TRYS(alloc(&p, sizeof(double) * 2 * 256));
    m->gm.d_h = static_cast<double *>(p);
    CGP_HIP(hipMemcpy(m->gm.d_diag, diag.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    CGP_HIP(hipMemcpy(m->gm.d_lrows, lrows.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    CGP_HIP(hipMemcpy(m->gm.d_urows, urows.data(), sizeof(int) * n, hipMemcpyHostToDevice));
    m->gm.ready = true;
  }
  if (restart > m->gm.cap) {
    void *p = nullptr;
    TRYS(alloc(&p, sizeof(double) * (size_t)(restart + 1) * n));
    m->gm.d_V = static_cast<double *>(p);
    m->gm.cap = restart;
  }
  return CGP_OK;
}

void ilu_apply(cgp_mesh *m, const double *r, double *z) {
  hipStream_t s = m->stream;
  const std::vector<int> &lp = m->gm.lptr, &up = m->gm.uptr;
  for (size_t l = 0; l + 1 < lp.size(); l++) {
    const int cnt = lp[l + 1] - lp[l];
    hipLaunchKernelGGL(k_ilu_lower, dim3(blocks_1d(cnt)), dim3(256), 0, s, cnt, m->gm.d_lrows + lp[l], m->d_rp_c,
                       m->d_col_c, (const int *)m->gm.d_diag, (const double *)m->gm.d_lu, r, z);
  }
  for (size_t l = 0; l + 1 < up.size(); l++) {
    const int cnt = up[l + 1] - up[l];
    hipLaunchKernelGGL(k_ilu_upper, dim3(blocks_1d(cnt)), dim3(256), 0, s, cnt, m->gm.d_urows + up[l], m->d_rp_c,
                       m->d_col_c, (const int *)m->gm.d_diag, (const double *)m->gm.d_lu, z);
  }
}

// host dot products of w with the first J basis vectors (fixed-order sums of the block partials)
cgp_status multidot(cgp_mesh *m, int J, const double *V, const double *w, std::vector<double> &out) {
  const int n = m->pc.n;
  hipLaunchKernelGGL(k_multidot, dim3(kMultiBlocks), dim3(256), 0, m->stream, n, J, V, w, m->gm.d_part);
  std::vector<double> part((size_t)J * kMultiBlocks);
  CGP_HIP(hipMemcpyAsync(part.data(), m->gm.d_part, sizeof(double) * part.size(), hipMemcpyDeviceToHost, m->stream));
  CGP_HIP(hipStreamSynchronize(m->stream));
  out.assign(J, 0.0);
  for (int c = 0; c < J; c++)
    for (int b = 0; b < kMultiBlocks; b++) out[c] += part[(size_t)c * kMultiBlocks + b];
  return CGP_OK;
}

}  // namespace

// ILU(0) of the eliminated coarse Poisson matrix, on the device, level by level
cgp_status gmres_factor(cgp_mesh *m) {
  const int n = m->pc.n;
  CGP_HIP(hipMemcpyAsync(m->gm.d_lu, m->d_Kbc, sizeof(double) * m->pc.nnz, hipMemcpyDeviceToDevice, m->stream));
  const std::vector<int> &lp = m->gm.lptr;
  for (size_t l = 0; l + 1 < lp.size(); l++) {
    const int cnt = lp[l + 1] - lp[l];
    hipLaunchKernelGGL(k_ilu_factor, dim3(blocks_1d(cnt)), dim3(256), 0, m->stream, cnt, m->gm.d_lrows + lp[l],
                       m->d_rp_c, m->d_col_c, (const int *)m->gm.d_diag, m->gm.d_lu);
  }
  CGP_HIP(hipGetLastError());
  (void)n;
  m->gm.factored = true;
  return CGP_OK;
}

// Solve Kbar x = b (b already carries the boundary conditions; x holds the initial guess).
cgp_status gmres_solve(cgp_mesh *m, const double *b, double *x, const cgp_solver_opts *o, KrylovState *fin) {
  const int n = m->pc.n;
  const int M = o->restart > 0 ? o->restart : 30;
  TRYS(gmres_setup(m, M));
  if (!m->gm.factored) TRYS(gmres_factor(m));
  hipStream_t s = m->stream;
  double *V = m->gm.d_V, *w = m->gm.d_work, *z = w + n, *t = w + 2 * n;
  const int nb = blocks_1d(n);
  std::vector<double> h, h2, H((size_t)(M + 1) * M), cs(M), sn(M), g(M + 1), y(M);
  std::vector<double> dots;
  *fin = KrylovState{};
  fin->ncomp = 1;
  // ||b||
  TRYS(multidot(m, 1, b, b, dots));
  const double bn = std::sqrt(dots[0]);
  fin->bnorm[0] = bn;
  if (!std::isfinite(bn)) {
    fin->status = CGP_E_NONFINITE;
    return CGP_OK;
  }
  if (bn == 0.0) {
    CGP_HIP(hipMemsetAsync(x, 0, sizeof(double) * n, s));
    fin->done[0] = 1;
    fin->zero_b[0] = 1;
    return CGP_OK;
  }
  int k = 0;
  for (;;) {
    hipLaunchKernelGGL(k_residual, dim3(nb), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c, (const double *)m->d_Kbc, b,
                       (const double *)x, V);
    TRYS(multidot(m, 1, V, V, dots));
    const double rn = std::sqrt(dots[0]);
    fin->rnorm[0] = rn;
    fin->iters = k;
    if (!std::isfinite(rn)) {
      fin->status = CGP_E_NONFINITE;
      return CGP_OK;
    }
    if (rn <= o->tol * bn) {
      fin->done[0] = 1;
      return CGP_OK;
    }
    if (k >= o->max_iter) {
      fin->status = CGP_E_NOCONV;
      return CGP_OK;
    }
    hipLaunchKernelGGL(k_scale_into, dim3(nb), dim3(256), 0, s, n, 1.0 / rn, (const double *)V, V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = rn;
    int j = 0;
    bool stop = false;
    for (; j < M && k < o->max_iter && !stop; j++, k++) {
      double *vj = V + (size_t)j * n, *vn = V + (size_t)(j + 1) * n;
      ilu_apply(m, vj, z);
      hipLaunchKernelGGL(k_matvec, dim3(nb), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c, (const double *)m->d_Kbc,
                         (const double *)z, w);
      // classical Gram-Schmidt, twice
      std::vector<double> hc(j + 1, 0.0);
      for (int pass = 0; pass < 2; pass++) {
        TRYS(multidot(m, j + 1, V, w, h));
        CGP_HIP(hipMemcpyAsync(m->gm.d_h, h.data(), sizeof(double) * (j + 1), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_sub_combination, dim3(nb), dim3(256), 0, s, n, j + 1, (const double *)V,
                           (const double *)m->gm.d_h, w);
        for (int i = 0; i <= j; i++) hc[i] += h[i];
      }
      TRYS(multidot(m, 1, w, w, dots));
      const double hn = std::sqrt(dots[0]);
      if (hn > 0.0) hipLaunchKernelGGL(k_scale_into, dim3(nb), dim3(256), 0, s, n, 1.0 / hn, (const double *)w, vn);
      for (int i = 0; i <= j; i++) H[(size_t)i * M + j] = hc[i];
      H[(size_t)(j + 1) * M + j] = hn;
      for (int i = 0; i < j; i++) {
        const double a = H[(size_t)i * M + j], c = H[(size_t)(i + 1) * M + j];
        H[(size_t)i * M + j] = cs[i] * a + sn[i] * c;
        H[(size_t)(i + 1) * M + j] = -sn[i] * a + cs[i] * c;
      }
      const double a = H[(size_t)j * M + j], c = H[(size_t)(j + 1) * M + j];
      const double r = std::hypot(a, c);
      cs[j] = r > 0.0 ? a / r : 1.0;
      sn[j] = r > 0.0 ? c / r : 0.0;
      H[(size_t)j * M + j] = r;
      H[(size_t)(j + 1) * M + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      if (!std::isfinite(g[j + 1])) {
        fin->status = CGP_E_NONFINITE;
        return CGP_OK;
      }
      stop = std::fabs(g[j + 1]) <= o->tol * bn || hn == 0.0;
    }
    // y = H^-1 g, x += M^-1 (V y)
    for (int i = j - 1; i >= 0; i--) {
      double sum = g[i];
      for (int q = i + 1; q < j; q++) sum -= H[(size_t)i * M + q] * y[q];
      y[i] = sum / H[(size_t)i * M + i];
    }
    CGP_HIP(hipMemcpyAsync(m->gm.d_h, y.data(), sizeof(double) * j, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_combination, dim3(nb), dim3(256), 0, s, n, j, (const double *)V, (const double *)m->gm.d_h,
                       t);
    ilu_apply(m, t, z);
    hipLaunchKernelGGL(k_add, dim3(nb), dim3(256), 0, s, n, (const double *)z, x);
    CGP_HIP(hipGetLastError());
  }
}

}  // namespace cgp
