// Persistent Jacobi-PCG for the coarse pressure Poisson solve (Eq. 21).
//
// One cooperative launch runs the whole Krylov loop.  Each block owns a fixed
// contiguous range of rows (balanced by nonzeros) for the life of the kernel,
// so a block's matrix rows and vector segments stay in the L2 of the XCD it
// runs on.  Per iteration there are two grid-wide synchronisations, each of
// which also completes a deterministic reduction: every block writes one
// partial, passes the barrier, and then sums all partials in the same fixed
// order, so every block derives bit-identical alpha, beta and convergence
// decisions and leaves the loop together.
//
//   phase A: p_new = z + beta p_old (own rows); q = K p_new, with p_new formed
//            on the fly for the gathered columns; partial p_new.q  -> sync
//   phase B: x += alpha p_new; r -= alpha q; z = D^-1 r; partials r.z, r.r -> sync
//
// The same kernel serves the FP64 solve (T = double) and the inner FP32 solve
// of iterative refinement (T = float, right-hand side r64/||r64||, zero guess);
// dot products are accumulated in FP64 in both.  Every barrier wait is bounded:
// a block that spins too long sets an abort flag; a block that finds the flag
// set after a barrier leaves before it uses the (possibly stale) reduction, and
// every block that left that way raises the solve's status to CGP_E_DEVICE
// (atomic maximum, so no later write can hide it).  The grid is at most one
// block per compute unit: a launch of two blocks per CU, which the occupancy
// query allowed, did not have every block resident and never passed the first
// barrier.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "persistent.h"

namespace cgp {
namespace pdev {

constexpr int kBlock = 1024;

struct GridBar {
  unsigned count;
  unsigned gen;
  int abort;
  int pad;
};

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  return x;
}

// Grid barrier.  BAR = 0: one arrival counter that only ever grows (zeroed
// before the launch); barrier number k of the kernel completes when it
// reaches gridDim.x * (k + 1), so there is no reset to race with.  Only
// thread 0 of a block orders memory (agent-scope release on arrival, acquire
// after the wait); the workgroup barriers around it cover the block's other
// waves, so a block pays one L2 writeback and one invalidate per barrier.
// BAR = 1: the HIP cooperative-groups grid barrier.
// Returns true in every thread of the block when the solve is being abandoned:
// this block gave up waiting, or another block did before this one passed.
template <int BAR>
__device__ __forceinline__ bool grid_sync(GridBar *bar, unsigned &epoch, long long spin_limit) {
  if (BAR == 1) {
    cooperative_groups::this_grid().sync();
    return false;
  }
  __shared__ int gave_up;
  epoch += 1;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned target = gridDim.x * epoch;
    __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    long long spins = 0;
    while (__hip_atomic_load(&bar->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > spin_limit) {
        __hip_atomic_store(&bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see every block's writes made before the barrier
    gave_up = __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  return gave_up != 0;
}

// Block-reduce K values, publish one partial per block in buf[k][grid], barrier,
// then sum all partials in a fixed order; tot[] is identical in every block.
// Returns true (tot[] not formed) when the solve is being abandoned.
template <int K, int BAR>
__device__ __forceinline__ bool grid_allreduce(double (&v)[K], double *buf, GridBar *bar, unsigned &epoch,
                                               long long spin_limit, double (&tot)[K]) {
  __shared__ double sh[K][kBlock / 64];
  __shared__ double res[K];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; k++) {
    const double x = wave_sum(v[k]);
    if (lane == 0) sh[k][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < nw; w++) s += sh[threadIdx.x][w];
    buf[threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
  if (grid_sync<BAR>(bar, epoch, spin_limit)) return true;
#pragma unroll
  for (int k = 0; k < K; k++) {
    double x = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
      x += buf[k * gridDim.x + b];
    x = wave_sum(x);
    if (lane == 0) sh[k][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int w = 0; w < nw; w++) s += sh[threadIdx.x][w];
    res[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) tot[k] = res[k];
  return false;
}

// a classification test: x - x == 0 can contract into an fma that rejects finite products
__device__ __forceinline__ bool finite(double x) { return __builtin_isfinite(x); }

template <typename T, int L, bool IR, int BAR>
__global__ void __launch_bounds__(kBlock) k_pcg_persistent(PersistArgs args) {
  const PersistArgs &a = args;
  const T *__restrict__ K = static_cast<const T *>(a.val);
  const T *__restrict__ dinv = static_cast<const T *>(a.dinv);
  T *__restrict__ x = static_cast<T *>(a.x);
  T *__restrict__ r = static_cast<T *>(a.r);
  T *__restrict__ z = static_cast<T *>(a.z);
  T *__restrict__ pv[2] = {static_cast<T *>(a.p0), static_cast<T *>(a.p1)};
  T *__restrict__ q = static_cast<T *>(a.q);
  const int *__restrict__ rp = a.rp;
  const int *__restrict__ col = a.col;
  GridBar *bar = reinterpret_cast<GridBar *>(a.bar);
  const int r0 = a.row_begin[blockIdx.x], r1 = a.row_begin[blockIdx.x + 1];
  const int lane = threadIdx.x & (L - 1), grp = threadIdx.x / L, ngrp = blockDim.x / L;
  int red = 0;          // alternates the two partial buffers
  unsigned epoch = 0;   // grid barriers passed
  auto buf = [&]() { double *b = a.partials + (red & 1) * 4 * gridDim.x; red++; return b; };

  // ---- init: r = b - K x, z = D^-1 r, p_old = 0
  double scale = 1.0;
  if (IR) {
    const double rn = a.outer->rnorm[0];
    scale = rn > 0.0 ? 1.0 / rn : 0.0;
  }
  for (int row = r0 + grp; row < r1; row += ngrp) {
    double s = 0.0;
    if (!IR)
      for (int k = rp[row] + lane; k < rp[row + 1]; k += L) s += (double)K[k] * (double)x[col[k]];
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
    if (lane == 0) {
      double bb = IR ? a.b64[row] * scale : (double)static_cast<const T *>(a.b)[row];
      const T rr = (T)(bb - s);
      r[row] = rr;
      z[row] = dinv[row] * rr;
      pv[0][row] = (T)0;
      if (IR) x[row] = (T)0;
    }
  }
  __syncthreads();
  double acc3[3] = {0.0, 0.0, 0.0};
  for (int row = r0 + threadIdx.x; row < r1; row += blockDim.x) {
    const double rr = r[row], zz = z[row];
    const double bb = IR ? a.b64[row] * scale : (double)static_cast<const T *>(a.b)[row];
    acc3[0] += rr * zz;
    acc3[1] += rr * rr;
    acc3[2] += bb * bb;
  }
  double tot3[3] = {0.0, 1.0, 1.0};
  const bool gave_up = grid_allreduce<3, BAR>(acc3, buf(), bar, epoch, a.spin_limit, tot3);
  double rz = tot3[0], rnorm = sqrt(tot3[1]);
  const double bnorm = sqrt(tot3[2]);
  const double tol = a.tol;
  int status = gave_up ? CGP_E_DEVICE : ((finite(rnorm) && finite(bnorm)) ? 0 : CGP_E_NONFINITE);
  bool done = !gave_up && ((bnorm == 0.0) || (rnorm <= tol * bnorm));
  if (IR && (a.outer->done[0] || a.outer->status)) done = true;  // refinement already converged
  double beta = 0.0;
  int it = 0;
  while (!done && status == 0 && it < a.maxit) {
    T *p_old = pv[it & 1], *p_new = pv[(it + 1) & 1];
    const T bt = (T)beta;
    // ---- phase A
    double acc1[1] = {0.0};
    for (int row = r0 + grp; row < r1; row += ngrp) {
      T s = (T)0;
      for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
        const int j = col[k];
        s += K[k] * (z[j] + bt * p_old[j]);
      }
#pragma unroll
      for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
      if (lane == 0) {
        const T pn = z[row] + bt * p_old[row];
        p_new[row] = pn;
        q[row] = s;
        acc1[0] += (double)pn * (double)s;
      }
    }
    double tot1[1];
    if (grid_allreduce<1, BAR>(acc1, buf(), bar, epoch, a.spin_limit, tot1)) {
      status = CGP_E_DEVICE;
      break;
    }
    const double alpha = rz / tot1[0];
    if (!finite(alpha)) {
      status = CGP_E_NONFINITE;
      break;
    }
    const T al = (T)alpha;
    // ---- phase B
    double acc2[2] = {0.0, 0.0};
    for (int row = r0 + threadIdx.x; row < r1; row += blockDim.x) {
      const T xx = x[row] + al * p_new[row];
      const T rr = r[row] - al * q[row];
      const T zz = dinv[row] * rr;
      x[row] = xx;
      r[row] = rr;
      z[row] = zz;
      acc2[0] += (double)rr * (double)zz;
      acc2[1] += (double)rr * (double)rr;
    }
    double tot2[2];
    if (grid_allreduce<2, BAR>(acc2, buf(), bar, epoch, a.spin_limit, tot2)) {
      status = CGP_E_DEVICE;
      break;
    }
    beta = tot2[0] / rz;
    rz = tot2[0];
    rnorm = sqrt(tot2[1]);
    it++;
    if (!finite(rnorm)) status = CGP_E_NONFINITE;
    done = rnorm <= tol * bnorm;
  }
  // status codes order by severity (NOCONV 3 < NONFINITE 4 < DEVICE 5); the state was set to 0
  // before the launch, so an abandoning block's CGP_E_DEVICE survives block 0's own report
  KrylovState *st = a.state;
  if (threadIdx.x == 0 && status == CGP_E_DEVICE)
    __hip_atomic_fetch_max(&st->status, (int)CGP_E_DEVICE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->iters = it;
    st->rnorm[0] = rnorm;
    st->bnorm[0] = bnorm;
    st->done[0] = done && status == 0;
    st->zero_b[0] = (bnorm == 0.0);
    const int mine = status ? status : ((!done && !IR) ? CGP_E_NOCONV : 0);
    __hip_atomic_fetch_max(&st->status, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace pdev

// ---------------------------------------------------------------- host side
namespace {
template <typename T, bool IR>
const void *kernel_ptr(int L, int bar) {
  const void *fn = nullptr;
  dispatch_L(L, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    fn = bar == 1 ? reinterpret_cast<const void *>(&pdev::k_pcg_persistent<T, LL, IR, 1>)
                  : reinterpret_cast<const void *>(&pdev::k_pcg_persistent<T, LL, IR, 0>);
  });
  return fn;
}
}  // namespace

int persistent_block() { return pdev::kBlock; }

cgp_status persistent_setup(cgp_mesh *m) {
  int dev = 0;
  CGP_HIP(hipGetDevice(&dev));
  if (m->coop_max == 0) {
    int coop = 0;
    CGP_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
    if (!coop) {
      set_error("device does not support cooperative launches");
      return CGP_E_DEVICE;
    }
    int per_cu = 0;
    for (int bar = 0; bar < 2; bar++)
      for (const void *fn : {kernel_ptr<double, false>(m->tune.coarse.lanes, bar),
                             kernel_ptr<float, true>(m->tune.coarse.lanes, bar)}) {
        int b = 0;
        CGP_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, fn, pdev::kBlock, 0));
        per_cu = per_cu == 0 ? b : std::min(per_cu, b);
      }
    if (per_cu < 1) {
      set_error("persistent PCG kernel cannot be resident");
      return CGP_E_DEVICE;
    }
    m->coop_max = per_cu * m->cu_count;
  }
  const int n = m->pc.n;
  int grid = m->tune.pcg_grid > 0 ? m->tune.pcg_grid : m->cu_count;
  grid = std::min(grid, std::min(m->coop_max, m->cu_count));  // at most one block per compute unit
  grid = std::max(1, std::min(grid, (n + 255) / 256));
  if (grid == m->coop_blocks) return CGP_OK;
  // rows split by nonzeros: block b owns rows [rb[b], rb[b+1])
  std::vector<int> rb(grid + 1, n);
  rb[0] = 0;
  const long long nnz = m->pc.nnz;
  int row = 0;
  for (int b = 1; b < grid; b++) {
    const long long target = nnz * b / grid;
    while (row < n && m->pc.rp[row] < target) row++;
    rb[b] = row;
  }
  void *p = nullptr;
  if (!m->d_bar) {
    CGP_HIP(hipMalloc(&p, sizeof(pdev::GridBar)));
    m->allocations.push_back(p);
    m->d_bar = p;
  }
  CGP_HIP(hipMalloc(&p, sizeof(int) * (grid + 1)));
  m->allocations.push_back(p);
  m->d_row_begin = static_cast<int *>(p);
  CGP_HIP(hipMemcpy(m->d_row_begin, rb.data(), sizeof(int) * (grid + 1), hipMemcpyHostToDevice));
  CGP_HIP(hipMalloc(&p, sizeof(double) * 8 * grid));
  m->allocations.push_back(p);
  m->d_ppartials = static_cast<double *>(p);
  m->coop_blocks = grid;
  return CGP_OK;
}

cgp_status persistent_pcg(cgp_mesh *m, bool fp32_inner, const double *b, void *x, void *const *w, double tol,
                          int maxit, KrylovState *state, const KrylovState *outer, const double *b64) {
  CGP_HIP(hipMemsetAsync(m->d_bar, 0, sizeof(pdev::GridBar), m->stream));
  PersistArgs a{};
  a.rp = m->d_rp_c;
  a.col = m->d_col_c;
  a.val = fp32_inner ? (const void *)m->d_Kbc32 : (const void *)m->d_Kbc;
  a.dinv = fp32_inner ? (const void *)m->d_dinvK32 : (const void *)m->d_dinvK;
  a.b = b;
  a.b64 = b64;
  a.x = x;
  a.r = w[0];
  a.z = w[1];
  a.p0 = w[2];
  a.p1 = w[3];
  a.q = w[4];
  a.row_begin = m->d_row_begin;
  a.partials = m->d_ppartials;
  a.bar = m->d_bar;
  a.state = state;
  a.outer = outer;
  a.tol = tol;
  a.maxit = maxit;
  a.spin_limit = 1ll << (m->tune.pcg_spin_log2 > 0 ? m->tune.pcg_spin_log2 : 24);
  void *args[] = {&a};
  const int bar = m->tune.pcg_barrier;
  const void *fn = fp32_inner ? kernel_ptr<float, true>(m->tune.coarse.lanes, bar)
                              : kernel_ptr<double, false>(m->tune.coarse.lanes, bar);
  CGP_HIP(hipLaunchCooperativeKernel(fn, dim3(m->coop_blocks), dim3(pdev::kBlock), args, 0, m->stream));
  return CGP_OK;
}

}  // namespace cgp
