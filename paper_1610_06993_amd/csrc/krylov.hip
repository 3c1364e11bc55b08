// Krylov solvers of libcgp: Jacobi-PCG (pressure Poisson, Eq. 21, and the
// consistent-mass correction, Eq. 23), Jacobi-BiCGStab for the two velocity
// components of the momentum system (Eq. 19), and FP32 Jacobi-PCG inside FP64
// iterative refinement for the pressure.
//
// Structure of every loop: the host enqueues a chunk of iterations, each a
// fixed sequence of kernels that all take the iteration index, then one
// single-block "finish" kernel, then reads the small solver state back.  Grid
// sums are fence-free (devutil.h): a kernel reduces the partials of the kernel
// before it, every block derives the same scalars, block 0 publishes them in
// the state (scalars read by a later kernel live in slots indexed by the
// iteration parity, so no kernel writes a slot that one of its own blocks
// reads).  Once a component converges it is frozen; once all have, every
// remaining kernel of the chunk returns at its first instruction.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <type_traits>

#include "devutil.h"
#include "kernels.h"
#include "learn.h"
#include "persistent.h"

namespace cgp {
namespace dev {

template <typename T, int NC>
struct Vec;
template <typename T>
struct Vec<T, 1> {
  static __device__ __forceinline__ void get(const T *p, int i, double (&o)[1]) { o[0] = (double)p[i]; }
  static __device__ __forceinline__ void put(T *p, int i, const double (&o)[1]) { p[i] = (T)o[0]; }
};
template <>
struct Vec<double, 2> {
  static __device__ __forceinline__ void get(const double *p, int i, double (&o)[2]) {
    const double2 t = reinterpret_cast<const double2 *>(p)[i];
    o[0] = t.x;
    o[1] = t.y;
  }
  static __device__ __forceinline__ void put(double *p, int i, const double (&o)[2]) {
    reinterpret_cast<double2 *>(p)[i] = make_double2(o[0], o[1]);
  }
};

template <int NC>
__device__ __forceinline__ bool all_done(const KrylovState *st) {
  bool a = true;
#pragma unroll
  for (int c = 0; c < NC; c++) a = a && st->done[c];
  return a;
}

// ------------------------------------------------------------------ PCG
// r = b - A x, z = D^-1 r, p0 = p1 = 0; partials (r.z, r.r, b.b) per component.
template <int NC, int L>
__global__ void __launch_bounds__(kMaxBlock) k_cg_init(int n, const int *__restrict__ rp, const int *__restrict__ col,
                                                      const double *__restrict__ A, const double *__restrict__ b,
                                                      const double *__restrict__ x, const double *__restrict__ dinv,
                                                      double *__restrict__ r, double *__restrict__ z,
                                                      double *__restrict__ p0, double *__restrict__ p1,
                                                      double *__restrict__ Pout) {
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
      Vec<double, NC>::get(x, col[k], xc);
      const double a = A[k];
#pragma unroll
      for (int c = 0; c < NC; c++) s[c] += a * xc[c];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) s[c] = group_sum<L>(s[c]);
    if (lane == 0) {
      double bb[NC], rr[NC], zz[NC], zero[NC];
      Vec<double, NC>::get(b, row, bb);
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
      Vec<double, NC>::put(r, row, rr);
      Vec<double, NC>::put(z, row, zz);
      Vec<double, NC>::put(p0, row, zero);
      Vec<double, NC>::put(p1, row, zero);
    }
  }
  put_partials<3 * NC>(acc, Pout);
}

// Iteration `it`, first half.  Reduces the partials of the kernel before it
// (the init partials for it = 0, else the update partials (r.z, r.r)), tests
// convergence, forms beta = (r.z)_it / (r.z)_{it-1}, then p_new = z + beta p_old
// on its own rows and q = A p_new with p_new formed on the fly for the
// gathered columns; partials p_new.q.  T is the vector/matrix type (double, or
// float for the inner solve of iterative refinement); sums are in double.
template <typename T, int NC, int L>
__global__ void __launch_bounds__(kMaxBlock) k_cg_spmv(int Gin, int it, int n, const int *__restrict__ rp,
                                                      const int *__restrict__ col, const T *__restrict__ A,
                                                      const T *__restrict__ z, const T *__restrict__ p_old,
                                                      T *__restrict__ p_new, T *__restrict__ q,
                                                      const double *__restrict__ Pin, double *__restrict__ Pout,
                                                      KrylovState *__restrict__ st) {
  if (st->status || all_done<NC>(st)) return;
  double rz[NC], rr[NC], bb[NC];
  if (it == 0) {
    double t3[3 * NC];
    sum_partials<3 * NC>(Pin, Gin, t3);
#pragma unroll
    for (int c = 0; c < NC; c++) {
      rz[c] = t3[c];
      rr[c] = t3[NC + c];
      bb[c] = t3[2 * NC + c];
    }
  } else {
    double t2[2 * NC];
    sum_partials<2 * NC>(Pin, Gin, t2);
#pragma unroll
    for (int c = 0; c < NC; c++) {
      rz[c] = t2[c];
      rr[c] = t2[NC + c];
      bb[c] = st->bnorm[c] * st->bnorm[c];
    }
  }
  const double tol = st->tol;
  bool done[NC], all = true, bad = false;
  double beta[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) {
    done[c] = st->done[c] || bb[c] == 0.0 || sqrt(rr[c]) <= tol * sqrt(bb[c]);
    all = all && done[c];
    bad = bad || !is_finite(rr[c]) || !is_finite(rz[c]);
    beta[c] = (it == 0 || done[c]) ? 0.0 : rz[c] / st->rz[(it - 1) & 1][c];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < NC; c++) {
      if (it == 0) {
        st->bnorm[c] = sqrt(bb[c]);
        st->zero_b[c] = (bb[c] == 0.0);
      }
      st->rz[it & 1][c] = rz[c];
      st->done[c] = done[c];
      st->rnorm[c] = sqrt(rr[c]);
    }
    st->iters = it;
    if (bad) st->status = CGP_E_NONFINITE;
  }
  if (all || bad) return;
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) acc[c] = 0.0;
  if (NC == 1) {
    const T bt = (T)beta[0];
    for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
      T s = (T)0;
      for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
        const int j = col[k];
        s += A[k] * (z[j] + bt * p_old[j]);
      }
      double sd;
      if constexpr (sizeof(T) == 4)
        sd = (double)group_sumf<L>(s);
      else
        sd = group_sum<L>(s);
      if (lane == 0) {
        const T pn = z[row] + bt * p_old[row];
        p_new[row] = pn;
        q[row] = (T)sd;
        acc[0] += (double)pn * (double)(T)sd;
      }
    }
  } else {
    for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
      double s[NC];
#pragma unroll
      for (int c = 0; c < NC; c++) s[c] = 0.0;
      for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
        const int j = col[k];
        double zc[NC], pc[NC];
        Vec<T, NC>::get(z, j, zc);
        Vec<T, NC>::get(p_old, j, pc);
        const double a = A[k];
#pragma unroll
        for (int c = 0; c < NC; c++) s[c] += a * (zc[c] + beta[c] * pc[c]);
      }
#pragma unroll
      for (int c = 0; c < NC; c++) s[c] = group_sum<L>(s[c]);
      if (lane == 0) {
        double zc[NC], pc[NC];
        Vec<T, NC>::get(z, row, zc);
        Vec<T, NC>::get(p_old, row, pc);
#pragma unroll
        for (int c = 0; c < NC; c++) {
          pc[c] = zc[c] + beta[c] * pc[c];
          acc[c] += pc[c] * s[c];
        }
        Vec<T, NC>::put(p_new, row, pc);
        Vec<T, NC>::put(q, row, s);
      }
    }
  }
  put_partials<NC>(acc, Pout);
}

// Iteration `it`, second half: alpha = (r.z)_it / (p.q); x += alpha p,
// r -= alpha q, z = D^-1 r on the components not yet converged; partials
// (r.z, r.r).
template <typename T, int NC>
__global__ void __launch_bounds__(kMaxBlock) k_cg_update(int Gin, int it, int n, T *__restrict__ x, T *__restrict__ r,
                                                        T *__restrict__ z, const T *__restrict__ dinv,
                                                        const T *__restrict__ p, const T *__restrict__ q,
                                                        const double *__restrict__ Pin, double *__restrict__ Pout,
                                                        KrylovState *__restrict__ st) {
  if (st->status || all_done<NC>(st)) return;
  double pq[NC];
  sum_partials<NC>(Pin, Gin, pq);
  bool act[NC], bad = false;
  double alpha[NC];
#pragma unroll
  for (int c = 0; c < NC; c++) {
    act[c] = !st->done[c];
    alpha[c] = act[c] ? st->rz[it & 1][c] / pq[c] : 0.0;
    bad = bad || !is_finite(alpha[c]);
  }
  if (bad) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->status = CGP_E_NONFINITE;
    return;
  }
  double acc[2 * NC];
#pragma unroll
  for (int c = 0; c < 2 * NC; c++) acc[c] = 0.0;
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    double xx[NC], rr[NC], zz[NC], pp[NC], qq[NC];
    Vec<T, NC>::get(x, i, xx);
    Vec<T, NC>::get(r, i, rr);
    Vec<T, NC>::get(p, i, pp);
    Vec<T, NC>::get(q, i, qq);
    Vec<T, NC>::get(z, i, zz);
    const T d = dinv[i];
#pragma unroll
    for (int c = 0; c < NC; c++) {
      if (act[c]) {
        const T xn = (T)xx[c] + (T)alpha[c] * (T)pp[c];
        const T rn = (T)rr[c] - (T)alpha[c] * (T)qq[c];
        xx[c] = (double)xn;
        rr[c] = (double)rn;
        zz[c] = (double)(d * rn);
      }
      acc[c] += rr[c] * zz[c];
      acc[NC + c] += rr[c] * rr[c];
    }
    Vec<T, NC>::put(x, i, xx);
    Vec<T, NC>::put(r, i, rr);
    Vec<T, NC>::put(z, i, zz);
  }
  put_partials<2 * NC>(acc, Pout);
}

// After a chunk: publish residual norms, convergence and the iteration count
// from the last update's partials (one block).
template <int NC>
__global__ void __launch_bounds__(kMaxBlock) k_cg_finish(int it_end, int G, const double *__restrict__ Pin,
                                                        KrylovState *__restrict__ st) {
  if (st->status || all_done<NC>(st)) return;
  double t2[2 * NC];
  sum_partials<2 * NC>(Pin, G, t2);
  if (threadIdx.x != 0) return;
  bool bad = false;
  for (int c = 0; c < NC; c++) {
    const double rn = sqrt(t2[NC + c]);
    st->rnorm[c] = rn;
    bad = bad || !is_finite(rn);
    if (!st->done[c] && rn <= st->tol * st->bnorm[c]) st->done[c] = 1;
  }
  st->iters = it_end;
  if (bad) st->status = CGP_E_NONFINITE;
}

// components with a zero right-hand side get x = 0
template <int NC>
__global__ void k_zero_b_fix(int n, double *__restrict__ x, const KrylovState *__restrict__ st) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < NC; c++)
    if (st->zero_b[c]) x[NC * i + c] = 0.0;
}

// ------------------------------------------------------------------ single-kernel PCG (Chronopoulos-Gear)
// The same Jacobi-PCG in the recurrences of Chronopoulos & Gear (1989), which
// need one global synchronisation per iteration instead of two:
//   p_i = u_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}   (s_i = K p_i)
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i,  u_{i+1} = D^-1 r_{i+1}
//   w_{i+1} = K u_{i+1},  gamma_{i+1} = r_{i+1}.u_{i+1},  delta_{i+1} = w_{i+1}.u_{i+1}
//   beta_{i+1} = gamma_{i+1}/gamma_i,  alpha_{i+1} = gamma_{i+1}/(delta_{i+1} - beta_{i+1} gamma_{i+1}/alpha_i)
// One kernel does a whole iteration: the SpMV forms u_{i+1} on the fly for its
// gathered columns from the previous iteration's r, w and s.  Those live in one
// record per node, {r, w, s, D^-1} (double4, or float4 for the FP32 inner solve),
// so a gathered column costs one 32- (16-) byte load; the records are
// double-buffered (slot it & 1 is read, the other written; D^-1 is filled into
// both at init and never rewritten).  p and x are only touched on their own rows
// and are updated in place.
//
// Latency, not bandwidth, bounds an iteration at the sizes the method is run at,
// so the kernel is laid out to overlap its dependent loads: every load that does
// not need this iteration's scalars (the row pointers, columns and values of the
// block's first chunk of rows, the gathered records, the own records, x and p) is
// issued before the scalars are formed; wave 0 reduces the previous iteration's
// block partials while those loads are in flight and hands the totals to the
// block through LDS, and the block's own partials leave after one more barrier.

template <typename T>
__device__ __forceinline__ T cg1_u_next(T dinv, T r, T w, T s, T alpha, T beta) {
  return dinv * (r - alpha * (w + beta * s));
}

// entries per lane loaded ahead of the scalars: ten per row (P1 rows on the meshes here have at
// most nine); longer rows finish in a loop
template <int L> constexpr int cg1_ahead() { return (10 + L - 1) / L; }

// init, second kernel: w0 = K u0 with u0 = D^-1 r0 gathered from the records (fields r and D^-1
// only: this kernel writes field w); partials (gamma0, delta0, r0.r0).  Reduces the first
// kernel's partials (b.b) and publishes ||b||.
template <typename T, int L>
__global__ void __launch_bounds__(kMaxBlock) k_cg1_init_w(int Gin, int n, const int *__restrict__ rp,
                                                         const int *__restrict__ col, const T *__restrict__ A,
                                                         rec_t<T> *__restrict__ R0, const double *__restrict__ Pin,
                                                         double *__restrict__ Pout, KrylovState *__restrict__ st) {
  if (st->status || st->done[0]) return;
  double tb[1];
  sum_partials<1>(Pin, Gin, tb);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->bnorm[0] = sqrt(tb[0]);
    st->zero_b[0] = (tb[0] == 0.0);
    if (!is_finite(tb[0])) st->status = CGP_E_NONFINITE;
  }
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sum = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const int j = col[k];
      sum += (double)(A[k] * (R0[j].w * R0[j].x));
    }
    sum = group_sum<L>(sum);
    if (lane == 0) {
      const T w = (T)sum, r0 = R0[row].x, d = R0[row].w;
      const double r = (double)r0, u = (double)(d * r0);
      R0[row].y = w;
      acc[0] += r * u;
      acc[1] += (double)w * u;
      acc[2] += r * r;
    }
  }
  put_partials<3>(acc, Pout);
}

template <typename T, int L, int P, int U, int E>
__global__ void __launch_bounds__(kMaxBlock) k_cg1_iter(int Gin, int it, int n, const int *__restrict__ rp,
                                                       const int *__restrict__ col, const T *__restrict__ A,
                                                       T *__restrict__ x, T *__restrict__ p,
                                                       const rec_t<T> *__restrict__ Rc, rec_t<T> *__restrict__ Rn,
                                                       const double *__restrict__ Pin, double *__restrict__ Pout,
                                                       KrylovState *__restrict__ st) {
  using R4 = rec_t<T>;
  constexpr int EA = E > 0 ? E : 1;  // E = 0: no entries ahead (bandwidth-bound sizes, fewer registers)
  // the previous iteration's state and partials, first in the load queue
  const int stopped = st->status | st->done[0];
  const double bnorm = st->bnorm[0], tol = st->tol;
  const double rz_prev = it ? st->rz[(it - 1) & 1][0] : 1.0;
  const double al_prev = it ? st->alpha[(it - 1) & 1][0] : 1.0;
  double t3[3];
  // Direct partials (E > 0): wave 0 alone loads them here and sums them once the row loads below are in
  // flight, and the block takes the totals from LDS; every wave summing them itself put its own partial
  // loads ahead of its row loads.  Summed partials (E = 0, 3 values): each wave reads them.
  __shared__ double tot_sh[3];
  double pa[3][U];
  const bool wave0 = (threadIdx.x >> 6) == 0;
  if constexpr (E > 0) {
    if (wave0) {
      const int l = threadIdx.x & 63;
#pragma unroll
      for (int u = 0; u < U; u++)
#pragma unroll
        for (int k = 0; k < 3; k++) pa[k][u] = l + 64 * u < Gin ? Pin[k * Gin + l + 64 * u] : 0.0;
    }
  } else {
    wave_partials<3, U>(Pin, Gin, t3);
  }

  const int lane = threadIdx.x & (L - 1);
  const int rpb = blockDim.x / L;  // rows per block and pass
  const long long rows_chunk = (long long)rpb * P;
  int k0[P], k1[P];
  T av[P][EA], xo[P], po[P];
  R4 qv[P][EA], own[P];
  auto load_chunk = [&](int c) {
#pragma unroll
    for (int q = 0; q < P; q++) {
      const long long row = c * rows_chunk + q * rpb + threadIdx.x / L;
      k0[q] = 0;
      k1[q] = 0;
      if (row < n) {
        k0[q] = rp[row];
        k1[q] = rp[row + 1];
      }
    }
#pragma unroll
    for (int q = 0; q < P; q++) {
      const long long row = c * rows_chunk + q * rpb + threadIdx.x / L;
#pragma unroll
      for (int e = 0; e < E; e++) {
        const int k = k0[q] + lane + e * L;
        if (k < k1[q]) {
          av[q][e] = A[k];
          qv[q][e] = Rc[col[k]];
        } else {
          av[q][e] = T(0);
          qv[q][e] = R4{};
        }
      }
      if (row < n && lane == 0) {
        own[q] = Rc[row];
        xo[q] = x[row];
        po[q] = p[row];
      } else {
        own[q] = R4{};
        xo[q] = T(0);
        po[q] = T(0);
      }
    }
  };
  int c = xcd_block();
  load_chunk(c);
  if constexpr (E > 0) {
    if (wave0) {
      const int l = threadIdx.x & 63;
#pragma unroll
      for (int k = 0; k < 3; k++) {
        double sum = 0.0;
#pragma unroll
        for (int u = 0; u < U; u++) sum += pa[k][u];
        for (int b = l + 64 * U; b < Gin; b += 64) sum += Pin[k * Gin + b];
        sum = wave_sum(sum);
        if (l == 0) tot_sh[k] = sum;
      }
    }
    __syncthreads();
    t3[0] = tot_sh[0];
    t3[1] = tot_sh[1];
    t3[2] = tot_sh[2];
  }
  if (stopped) return;

  const double gam = t3[0], del = t3[1], rr = t3[2];
  const double bb = bnorm * bnorm;
  const bool done = bb == 0.0 || sqrt(rr) <= tol * sqrt(bb);
  double beta = 0.0, alpha = 0.0;
  if (it == 0) {
    alpha = gam / del;
  } else {
    beta = gam / rz_prev;
    alpha = gam / (del - beta * gam / al_prev);
  }
  const bool bad = !is_finite(rr) || (!done && (!is_finite(alpha) || !is_finite(beta)));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rz[it & 1][0] = gam;
    st->alpha[it & 1][0] = alpha;
    st->rnorm[0] = sqrt(rr);
    // counted, not copied from `it`: a captured chunk replayed later carries its capture-time `it`
    // (same parity, so the slots above are right), and the count stays that of the launches that updated
    if (!done && !bad) st->iters += 1;
    if (done) st->done[0] = 1;
    if (bad) st->status = CGP_E_NONFINITE;
  }
  if (done || bad) return;
  const T al = (T)alpha, bt = (T)beta;
  double acc[3] = {0.0, 0.0, 0.0};
  for (;;) {
#pragma unroll
    for (int q = 0; q < P; q++) {
      const long long row = c * rows_chunk + q * rpb + threadIdx.x / L;
      double sum = 0.0;
#pragma unroll
      for (int e = 0; e < E; e++)
        if (k0[q] + lane + e * L < k1[q])
          sum += (double)(av[q][e] * cg1_u_next<T>(qv[q][e].w, qv[q][e].x, qv[q][e].y, qv[q][e].z, al, bt));
      for (int k = k0[q] + lane + E * L; k < k1[q]; k += L) {
        const R4 g = Rc[col[k]];
        sum += (double)(A[k] * cg1_u_next<T>(g.w, g.x, g.y, g.z, al, bt));
      }
      sum = group_sum<L>(sum);
      if (row < n && lane == 0) {
        const T d = own[q].w, rc = own[q].x, wc = own[q].y, sc = own[q].z;
        const T si = wc + bt * sc;
        const T pi = d * rc + bt * po[q];
        const T rn = rc - al * si;
        const T un = cg1_u_next<T>(d, rc, wc, sc, al, bt);
        const T wn = (T)sum;
        x[row] = xo[q] + al * pi;
        p[row] = pi;
        store_rws(&Rn[row], rn, wn, si);
        acc[0] += (double)rn * (double)un;
        acc[1] += (double)wn * (double)un;
        acc[2] += (double)rn * (double)rn;
      }
    }
    c += gridDim.x;
    if (c * rows_chunk >= n) break;
    load_chunk(c);
  }
  put_partials_last<3>(acc, Pout);
}

// Large grids: one block sums an iteration's G block partials into 3 totals in a fixed order, so that
// the next iteration's waves read 3 values instead of 3 G each (that read grows as G squared).
__global__ void __launch_bounds__(kMaxBlock) k_cg1_total(int G, const double *__restrict__ Pin,
                                                        double *__restrict__ Ptot,
                                                        const KrylovState *__restrict__ st) {
  if (st->status || st->done[0]) return;
  double t3[3];
  sum_partials<3>(Pin, G, t3);
  if (threadIdx.x < 3) Ptot[threadIdx.x] = t3[threadIdx.x];
}

// after a chunk: convergence from the last iteration's partials (the iterations count themselves)
__global__ void __launch_bounds__(kMaxBlock) k_cg1_finish(int G, const double *__restrict__ Pin,
                                                         KrylovState *__restrict__ st) {
  if (st->status || st->done[0]) return;
  double t3[3];
  sum_partials<3>(Pin, G, t3);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(t3[2]);
  st->rnorm[0] = rn;
  if (!is_finite(rn)) st->status = CGP_E_NONFINITE;
  else if (rn <= st->tol * st->bnorm[0]) st->done[0] = 1;
}

// FP64 init, first kernel: r0 = b - K x0, p = s_{-1} = 0, records {r0, -, 0, D^-1} in slot 0 and
// {-, -, -, D^-1} in slot 1; partials b.b
template <int L>
__global__ void __launch_bounds__(kMaxBlock) k_cg1_init_r(int n, const int *__restrict__ rp,
                                                         const int *__restrict__ col, const double *__restrict__ A,
                                                         const double *__restrict__ dinv, const double *__restrict__ b,
                                                         const double *__restrict__ x, double *__restrict__ p,
                                                         double4 *__restrict__ R0, double4 *__restrict__ R1,
                                                         double *__restrict__ Pout) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[1] = {0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sum = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) sum += A[k] * x[col[k]];
    sum = group_sum<L>(sum);
    if (lane == 0) {
      const double bb = b[row], d = dinv[row];
      R0[row] = make_double4(bb - sum, 0.0, 0.0, d);
      R1[row] = make_double4(0.0, 0.0, 0.0, d);
      p[row] = 0.0;
      acc[0] += bb * bb;
    }
  }
  put_partials<1>(acc, Pout);
}

// Reduction asked of an inner FP32 solve: `inner_tol`, or half of what the outer tolerance still
// needs when that is less (a warm start then ends in one refinement step instead of over-solving).
__device__ __forceinline__ double inner_tol_for(double inner_tol, double outer_tol, double rn, double bn) {
  const double need = 0.5 * outer_tol * bn / rn;
  return need > inner_tol ? need : inner_tol;
}

// FP32 inner solve of iterative refinement, first kernel: outer convergence test on
// the FP64 residual partials (r.r, b.b); r0 = r64/||r64|| in FP32, d = p = s_{-1} = 0,
// records as in k_cg1_init_r with the FP32 D^-1; partials r0.r0 (the inner right-hand side norm).
__global__ void __launch_bounds__(kMaxBlock) k_cg1_ir_init(int Gin, int n, double inner_tol,
                                                          const double *__restrict__ r64,
                                                          const float *__restrict__ dinv, float4 *__restrict__ R0,
                                                          float4 *__restrict__ R1, float *__restrict__ d,
                                                          float *__restrict__ p, const double *__restrict__ Pin,
                                                          double *__restrict__ Pout, KrylovState *__restrict__ so,
                                                          KrylovState *__restrict__ si) {
  double t2[2];
  sum_partials<2>(Pin, Gin, t2);
  const double rn = sqrt(t2[0]), bn = sqrt(t2[1]);
  const bool bad = !is_finite(rn) || !is_finite(bn);
  const bool done = bn == 0.0 || rn <= so->tol * bn;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    so->rnorm[0] = rn;
    so->bnorm[0] = bn;
    so->zero_b[0] = (bn == 0.0);
    so->done[0] = done;
    if (bad) so->status = CGP_E_NONFINITE;
    si->done[0] = done || bad;
    si->status = 0;
    si->iters = 0;
    si->tol = inner_tol_for(inner_tol, so->tol, rn, bn);
  }
  if (done || bad) return;
  const double inv = 1.0 / rn;
  double acc[1] = {0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    const float rr = (float)(r64[i] * inv), di = dinv[i];
    R0[i] = make_float4(rr, 0.0f, 0.0f, di);
    R1[i] = make_float4(0.0f, 0.0f, 0.0f, di);
    d[i] = 0.0f;
    p[i] = 0.0f;
    acc[0] += (double)rr * (double)rr;
  }
  put_partials<1>(acc, Pout);
}

// ------------------------------------------------------------------ BiCGStab, 2 components
// r = b - A x, r^ = r, p = v = 0; partials (r.r, b.b) per component.
template <int L>
__global__ void __launch_bounds__(kMaxBlock) k_bi_init(int n, const int *__restrict__ rp, const int *__restrict__ col,
                                                      const double *__restrict__ A, const double2 *__restrict__ b,
                                                      const double2 *__restrict__ x, double2 *__restrict__ r,
                                                      double2 *__restrict__ rh, double2 *__restrict__ p,
                                                      double2 *__restrict__ v, double *__restrict__ Pout) {
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
  put_partials<4>(acc, Pout);
}

// Vector and matrix precision of a BiCGStab solve: T = double (the FP64 solve) or float (the inner
// solve of FP32 iterative refinement); scalars, dot products and the arithmetic are FP64 either way.
template <typename T> struct v2_of;
template <> struct v2_of<double> { using type = double2; };
template <> struct v2_of<float> { using type = float2; };
template <typename T>
__device__ __forceinline__ typename v2_of<T>::type mk2(double a, double b) {
  return typename v2_of<T>::type{(T)a, (T)b};
}

// Iteration `it` start: reduce (r.r, r^.r) of the previous iteration (or the
// init partials), test convergence, rho_it = r^.r, beta = (rho_it /
// rho_{it-1}) (alpha_{it-1} / omega_{it-1}); p = r + beta (p - omega v), p^ = D^-1 p.
// The loop launches it for iteration 0 only (p = r0); k_bi_xp forms the later directions.
template <typename T>
__global__ void __launch_bounds__(kMaxBlock) k_bi_p(int Gin, int it, int n, const typename v2_of<T>::type *__restrict__ r,
                                                   typename v2_of<T>::type *__restrict__ p,
                                                   const typename v2_of<T>::type *__restrict__ v,
                                                   const T *__restrict__ dinv, typename v2_of<T>::type *__restrict__ ph,
                                                   const double *__restrict__ Pin, KrylovState *__restrict__ st) {
  using V2 = typename v2_of<T>::type;
  if (st->status || all_done<2>(st)) return;
  double t4[4];
  sum_partials<4>(Pin, Gin, t4);
  double rr[2], rho[2], bb[2], beta[2], om[2];
  bool done[2], all = true, bad = false, brk = false;
  const double tol = st->tol;
  for (int c = 0; c < 2; c++) {
    rr[c] = t4[c];
    if (it == 0) {
      bb[c] = t4[2 + c];
      rho[c] = rr[c];  // r^ = r0
    } else {
      bb[c] = st->bnorm[c] * st->bnorm[c];
      rho[c] = t4[2 + c];
    }
    done[c] = st->done[c] || bb[c] == 0.0 || sqrt(rr[c]) <= tol * sqrt(bb[c]);
    all = all && done[c];
    bad = bad || !is_finite(rr[c]);
    beta[c] = 0.0;
    om[c] = 0.0;
    if (it > 0 && !done[c]) {
      const int pp = (it - 1) & 1;
      om[c] = st->omega[pp][c];
      if (om[c] == 0.0) brk = true;  // breakdown
      beta[c] = (rho[c] / st->rho[pp][c]) * (st->alpha[pp][c] / om[c]);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int c = 0; c < 2; c++) {
      if (it == 0) {
        st->bnorm[c] = sqrt(bb[c]);
        st->zero_b[c] = (bb[c] == 0.0);
      }
      st->rho[it & 1][c] = rho[c];
      st->done[c] = done[c];
      st->rnorm[c] = sqrt(rr[c]);
    }
    st->iters = it;
    if (bad) st->status = CGP_E_NONFINITE;
    else if (brk && !all) st->status = CGP_E_NOCONV;
  }
  if (all || bad || brk) return;
  const bool a0 = !done[0], a1 = !done[1];
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    const V2 rr2 = r[i], vv = v[i];
    V2 pp = p[i];
    if (a0) pp.x = (T)((double)rr2.x + beta[0] * ((double)pp.x - om[0] * (double)vv.x));
    if (a1) pp.y = (T)((double)rr2.y + beta[1] * ((double)pp.y - om[1] * (double)vv.y));
    p[i] = pp;
    const double d = dinv[i];
    ph[i] = mk2<T>(d * (double)pp.x, d * (double)pp.y);
  }
}

// Iterations after the first run as three kernels instead of four: the update of x and r and the
// next search direction share one pass over the nodes.  The direction needs rho_{i+1} = r^.r_{i+1},
// and with r_{i+1} = s - omega t that is r^.s - omega r^.t, both of which the t kernel can sum on
// its own rows; the convergence test of r_{i+1} (its r.r summed directly) moves to the start of the
// next v kernel.  A direction formed for a component that then tests converged is never used.

// Iteration `it` start: for it > 0 reduce r.r of r_it (from k_bi_xp of it - 1) and test each
// component, as k_bi_p does at it = 0; then v = A p^ with partials r^.v.
template <typename T, int L>
__global__ void __launch_bounds__(kMaxBlock) k_bi_vc(int Gin, int it, int n, const int *__restrict__ rp,
                                                    const int *__restrict__ col, const T *__restrict__ A,
                                                    const typename v2_of<T>::type *__restrict__ ph,
                                                    typename v2_of<T>::type *__restrict__ v,
                                                    const typename v2_of<T>::type *__restrict__ rh,
                                                    const double *__restrict__ Pin, double *__restrict__ Pout,
                                                    KrylovState *__restrict__ st) {
  using V2 = typename v2_of<T>::type;
  if (st->status || all_done<2>(st)) return;
  if (it > 0) {
    double rr[2];
    sum_partials<2>(Pin, Gin, rr);
    bool done[2], all = true, bad = false, brk = false;
    const double tol = st->tol;
    for (int c = 0; c < 2; c++) {
      const double bb = st->bnorm[c] * st->bnorm[c];
      done[c] = st->done[c] || bb == 0.0 || sqrt(rr[c]) <= tol * sqrt(bb);
      all = all && done[c];
      bad = bad || !is_finite(rr[c]);
      if (!done[c] && st->omega[(it - 1) & 1][c] == 0.0) brk = true;  // breakdown
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      for (int c = 0; c < 2; c++) {
        st->done[c] = done[c];
        st->rnorm[c] = sqrt(rr[c]);
      }
      st->iters = it;
      if (bad) st->status = CGP_E_NONFINITE;
      else if (brk && !all) st->status = CGP_E_NOCONV;
    }
    if (all || bad || brk) return;
  }
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[2] = {0.0, 0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sx = 0.0, sy = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const double a = A[k];
      const V2 xc = ph[col[k]];
      sx += a * (double)xc.x;
      sy += a * (double)xc.y;
    }
    sx = group_sum<L>(sx);
    sy = group_sum<L>(sy);
    if (lane == 0) {
      const V2 vw = mk2<T>(sx, sy);
      v[row] = vw;
      const V2 h = rh[row];
      acc[0] += (double)h.x * (double)vw.x;
      acc[1] += (double)h.y * (double)vw.y;
    }
  }
  put_partials<2>(acc, Pout);
}

// alpha = rho / (r^.v); s = r - alpha v formed on the fly; t = A (D^-1 s); partials (t.s, t.t, r^.s,
// r^.t) per component
template <typename T, int L>
__global__ void __launch_bounds__(kMaxBlock) k_bi_t(int Gin, int it, int n, const int *__restrict__ rp,
                                                   const int *__restrict__ col, const T *__restrict__ A,
                                                   const typename v2_of<T>::type *__restrict__ r,
                                                   const typename v2_of<T>::type *__restrict__ v,
                                                   const typename v2_of<T>::type *__restrict__ rh,
                                                   const T *__restrict__ dinv, typename v2_of<T>::type *__restrict__ t,
                                                   const double *__restrict__ Pin, double *__restrict__ Pout,
                                                   KrylovState *__restrict__ st) {
  using V2 = typename v2_of<T>::type;
  if (st->status || all_done<2>(st)) return;
  double rv[2];
  sum_partials<2>(Pin, Gin, rv);
  double al[2];
  bool bad = false;
  for (int c = 0; c < 2; c++) {
    al[c] = st->done[c] ? 0.0 : st->rho[it & 1][c] / rv[c];
    bad = bad || !is_finite(al[c]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->alpha[it & 1][0] = al[0];
    st->alpha[it & 1][1] = al[1];
    if (bad) st->status = CGP_E_NONFINITE;
  }
  if (bad) return;
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sx = 0.0, sy = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const int j = col[k];
      const double a = (double)A[k] * (double)dinv[j];
      const V2 rr = r[j], vv = v[j];
      sx += a * ((double)rr.x - al[0] * (double)vv.x);
      sy += a * ((double)rr.y - al[1] * (double)vv.y);
    }
    sx = group_sum<L>(sx);
    sy = group_sum<L>(sy);
    if (lane == 0) {
      const V2 tw = mk2<T>(sx, sy);
      t[row] = tw;
      const V2 rr = r[row], vv = v[row], h = rh[row];
      const double s0 = (double)rr.x - al[0] * (double)vv.x, s1 = (double)rr.y - al[1] * (double)vv.y;
      const double tx = tw.x, ty = tw.y;
      acc[0] += tx * s0;
      acc[1] += ty * s1;
      acc[2] += tx * tx;
      acc[3] += ty * ty;
      acc[4] += (double)h.x * s0;
      acc[5] += (double)h.y * s1;
      acc[6] += (double)h.x * tx;
      acc[7] += (double)h.y * ty;
    }
  }
  put_partials<8>(acc, Pout);
}

// omega = (t.s)/(t.t); x += alpha p^ + omega D^-1 s, r = s - omega t; rho_{it+1} = r^.s - omega r^.t,
// beta = (rho_{it+1} / rho_it)(alpha / omega); p = r + beta (p - omega v), p^ = D^-1 p; partials r.r
template <typename T>
__global__ void __launch_bounds__(kMaxBlock) k_bi_xp(int Gin, int it, int n, typename v2_of<T>::type *__restrict__ x,
                                                    typename v2_of<T>::type *__restrict__ r,
                                                    typename v2_of<T>::type *__restrict__ p,
                                                    const typename v2_of<T>::type *__restrict__ v,
                                                    const typename v2_of<T>::type *__restrict__ t,
                                                    const T *__restrict__ dinv, typename v2_of<T>::type *__restrict__ ph,
                                                    const double *__restrict__ Pin, double *__restrict__ Pout,
                                                    KrylovState *__restrict__ st) {
  using V2 = typename v2_of<T>::type;
  if (st->status || all_done<2>(st)) return;
  double t8[8];
  sum_partials<8>(Pin, Gin, t8);
  double w[2], al[2], be[2], rho_next[2];
  bool act[2];
  for (int c = 0; c < 2; c++) {
    act[c] = !st->done[c];
    w[c] = (act[c] && t8[2 + c] > 0.0) ? t8[c] / t8[2 + c] : 0.0;
    al[c] = st->alpha[it & 1][c];
    rho_next[c] = t8[4 + c] - w[c] * t8[6 + c];
    // omega = 0 is a breakdown, reported by the next v kernel unless the component has converged
    be[c] = (act[c] && w[c] != 0.0) ? (rho_next[c] / st->rho[it & 1][c]) * (al[c] / w[c]) : 0.0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int c = 0; c < 2; c++) {
      st->omega[it & 1][c] = w[c];
      st->rho[(it + 1) & 1][c] = rho_next[c];
    }
  }
  double acc[2] = {0.0, 0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    V2 xx = x[i], rr = r[i], pp = p[i];
    const V2 vv = v[i], tt = t[i];
    const double d = dinv[i];
    if (act[0]) {
      const double s = (double)rr.x - al[0] * (double)vv.x;
      xx.x = (T)((double)xx.x + (al[0] * (d * (double)pp.x) + w[0] * (d * s)));
      rr.x = (T)(s - w[0] * (double)tt.x);
      pp.x = (T)((double)rr.x + be[0] * ((double)pp.x - w[0] * (double)vv.x));
    }
    if (act[1]) {
      const double s = (double)rr.y - al[1] * (double)vv.y;
      xx.y = (T)((double)xx.y + (al[1] * (d * (double)pp.y) + w[1] * (d * s)));
      rr.y = (T)(s - w[1] * (double)tt.y);
      pp.y = (T)((double)rr.y + be[1] * ((double)pp.y - w[1] * (double)vv.y));
    }
    x[i] = xx;
    r[i] = rr;
    p[i] = pp;
    ph[i] = mk2<T>(d * (double)pp.x, d * (double)pp.y);
    const double rx = rr.x, ry = rr.y;
    acc[0] += rx * rx;
    acc[1] += ry * ry;
  }
  put_partials<2>(acc, Pout);
}

__global__ void __launch_bounds__(kMaxBlock) k_bi_finish(int it_end, int G, const double *__restrict__ Pin,
                                                        KrylovState *__restrict__ st) {
  if (st->status || all_done<2>(st)) return;
  double t2[2];
  sum_partials<2>(Pin, G, t2);  // r.r per component (the first two arrays of the init partials too)
  if (threadIdx.x != 0) return;
  bool bad = false;
  for (int c = 0; c < 2; c++) {
    const double rn = sqrt(t2[c]);
    st->rnorm[c] = rn;
    bad = bad || !is_finite(rn);
    if (!st->done[c] && rn <= st->tol * st->bnorm[c]) st->done[c] = 1;
  }
  st->iters = it_end;
  if (bad) st->status = CGP_E_NONFINITE;
}

// ---- FP32 inner BiCGStab inside FP64 iterative refinement of the momentum solve (both components)
// FP32 copies of the eliminated momentum matrix and its Jacobi inverse (once per solve).
__global__ void k_mir_convert(long nnz, int n, const double *__restrict__ A, const double *__restrict__ dinv,
                              float *__restrict__ A32, float *__restrict__ dinv32) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += stride) {
    A32[k] = (float)A[k];
    if (k < n) dinv32[k] = (float)dinv[k];
  }
}

// r64 = b - A x in FP64 (both components); partials (r.r, b.b) per component.
template <int L>
__global__ void __launch_bounds__(kMaxBlock) k_mir_residual(int n, const int *__restrict__ rp,
                                                           const int *__restrict__ col, const double *__restrict__ A,
                                                           const double2 *__restrict__ b, const double2 *__restrict__ x,
                                                           double2 *__restrict__ r64, double *__restrict__ Pout) {
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
      r64[row] = rr;
      acc[0] += rr.x * rr.x;
      acc[1] += rr.y * rr.y;
      acc[2] += bb.x * bb.x;
      acc[3] += bb.y * bb.y;
    }
  }
  put_partials<4>(acc, Pout);
}

// Outer test on the FP64 residual (per component: done when ||r|| <= tol ||b||), then the inner
// solve's start: r = r^ = r64 / ||r64|| in FP32 for the components still refining (zero for the
// others, which the inner solve then marks done at once), d = p = v = 0; inner tolerance = what the
// outer tolerance still needs (the smaller over the refining components), at least inner_tol.
// Partials (r.r, r.r) per component in the layout of the FP64 init, so that the first iteration
// reads them the same way.
__global__ void __launch_bounds__(kMaxBlock) k_mir_init(int Gin, int n, double inner_tol,
                                                       const double2 *__restrict__ r64, float2 *__restrict__ r,
                                                       float2 *__restrict__ rh, float2 *__restrict__ p,
                                                       float2 *__restrict__ v, float2 *__restrict__ d,
                                                       const double *__restrict__ Pin, double *__restrict__ Pout,
                                                       KrylovState *__restrict__ so, KrylovState *__restrict__ si) {
  double t4[4];
  sum_partials<4>(Pin, Gin, t4);
  double rn[2], bn[2], sc[2];
  bool act[2], bad = false;
  double need = 1.0;
  for (int c = 0; c < 2; c++) {
    rn[c] = sqrt(t4[c]);
    bn[c] = sqrt(t4[2 + c]);
    bad = bad || !is_finite(rn[c]);
    act[c] = !(bn[c] == 0.0 || rn[c] <= so->tol * bn[c]);
    sc[c] = act[c] && rn[c] > 0.0 ? 1.0 / rn[c] : 0.0;
    if (act[c]) need = fmin(need, inner_tol_for(inner_tol, so->tol, rn[c], bn[c]));
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int c = 0; c < 2; c++) {
      so->bnorm[c] = bn[c];
      so->rnorm[c] = rn[c];
      so->zero_b[c] = (bn[c] == 0.0);
      so->done[c] = !act[c];
    }
    if (bad) so->status = CGP_E_NONFINITE;
    KrylovState t{};
    t.tol = need;
    t.maxit = si->maxit;
    t.ncomp = 2;
    for (int c = 0; c < 2; c++) t.done[c] = !act[c] || bad;
    *si = t;
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int stride = gridDim.x * blockDim.x;
  for (int i = xcd_block() * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double2 q = r64[i];
    const float2 z = make_float2((float)(q.x * sc[0]), (float)(q.y * sc[1]));
    r[i] = z;
    rh[i] = z;
    p[i] = make_float2(0.0f, 0.0f);
    v[i] = make_float2(0.0f, 0.0f);
    d[i] = make_float2(0.0f, 0.0f);
    const double zx = z.x, zy = z.y;
    acc[0] += zx * zx;
    acc[1] += zy * zy;
    acc[2] += zx * zx;
    acc[3] += zy * zy;
  }
  put_partials<4>(acc, Pout);
}

// out = a + s b over `count` values (the mass solve's extrapolated start and its difference update)
__global__ void k_axpy_into(long count, const double *__restrict__ a, double sb, const double *__restrict__ b,
                            double *__restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = a[i] + sb * b[i];
}

// x += ||r64|| d on the components that refined (FP64).
__global__ void k_mir_update(int n, double2 *__restrict__ x, const float2 *__restrict__ d,
                             const KrylovState *__restrict__ so) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float2 dd = d[i];
  double2 xx = x[i];
  if (!so->done[0]) xx.x += so->rnorm[0] * (double)dd.x;
  if (!so->done[1]) xx.y += so->rnorm[1] * (double)dd.y;
  x[i] = xx;
}

// ------------------------------------------------------------------ projected momentum guess
// The momentum solutions of the last kProj consecutive steps are kept per node, hist[j][i] =
// (U_i,x, U_i,y) of ring slot i at node j: 128 bytes a node, so one gathered column brings all
// of them.  The initial guess is, per component, the combination x0 = sum_i c_i U_i that
// minimises ||b - A x0||_2 over the free rows (A and b after the Dirichlet elimination, whose
// free rows do not read the Dirichlet columns): the normal equations (AU)^T (AU) c = (AU)^T b.

// Per block: partial sums of the two Gram matrices (upper triangles) and right-hand sides over
// its row tiles, one array of gridDim.x partials per entry.  Entry e of component c sits at
// c * kProjPer + e: the triangle row by row (i <= j), then (AU_i)^T b for i < kProj.
template <int L>
__global__ void __launch_bounds__(256) k_proj_gram(int n, const int *__restrict__ rp, const int *__restrict__ col,
                                                  const double *__restrict__ A, const unsigned char *__restrict__ vdir,
                                                  const double2 *__restrict__ hist, const double2 *__restrict__ b,
                                                  double *__restrict__ P) {
  constexpr int R = 256 / L;  // rows per tile
  __shared__ double sw[R][2 * kProj + 3];
  const int lane = threadIdx.x & (L - 1), g = threadIdx.x / L;
  int ci = -1, cj = -1;  // the two LDS columns whose product this thread accumulates
  if (threadIdx.x < 2 * kProjPer) {
    const int c = threadIdx.x / kProjPer;
    int e = threadIdx.x % kProjPer;
    if (e < kProjTri) {
      int i = 0;
      while (e >= kProj - i) {
        e -= kProj - i;
        i++;
      }
      ci = c * kProj + i;
      cj = c * kProj + i + e;
    } else {
      ci = c * kProj + (e - kProjTri);
      cj = 2 * kProj + c;
    }
  }
  double acc = 0.0;
  const int tiles = (n + R - 1) / R;
  for (int tile = xcd_block(); tile < tiles; tile += gridDim.x) {
    const int row = tile * R + g;
    double wx[kProj], wy[kProj];
#pragma unroll
    for (int i = 0; i < kProj; i++) wx[i] = wy[i] = 0.0;
    if (row < n) {
      for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
        const double a = A[k];
        const double2 *h = hist + (size_t)col[k] * kProj;
#pragma unroll
        for (int i = 0; i < kProj; i++) {
          const double2 v = h[i];
          wx[i] += a * v.x;
          wy[i] += a * v.y;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kProj; i++) {
      wx[i] = group_sum<L>(wx[i]);
      wy[i] = group_sum<L>(wy[i]);
    }
    if (lane == 0) {
      const bool fr = row < n && !vdir[row];
      const double2 bb = fr ? b[row] : make_double2(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < kProj; i++) {
        sw[g][i] = fr ? wx[i] : 0.0;
        sw[g][kProj + i] = fr ? wy[i] : 0.0;
      }
      sw[g][2 * kProj] = bb.x;
      sw[g][2 * kProj + 1] = bb.y;
    }
    __syncthreads();
    if (ci >= 0) {  // four independent chains over the tile's rows
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < R; r += 4) {
#pragma unroll
        for (int q = 0; q < 4; q++) a4[q] += sw[r + q][ci] * sw[r + q][cj];
      }
      acc += (a4[0] + a4[1]) + (a4[2] + a4[3]);
    }
    __syncthreads();
  }
  if (ci >= 0) P[threadIdx.x * gridDim.x + blockIdx.x] = acc;
}

// One block per Gram entry: the G block partials summed in a fixed order into S[entry].
__global__ void __launch_bounds__(256) k_proj_sum(int G, const double *__restrict__ P, double *__restrict__ S) {
  const double *p = P + (size_t)blockIdx.x * G;
  double a[4] = {0.0, 0.0, 0.0, 0.0};  // four chains, so that the loads overlap
  int q = threadIdx.x;
  for (; q + 3 * (int)blockDim.x < G; q += 4 * blockDim.x)
#pragma unroll
    for (int r = 0; r < 4; r++) a[r] += p[q + r * blockDim.x];
  for (; q < G; q += blockDim.x) a[0] += p[q];
  double v[1] = {(a[0] + a[1]) + (a[2] + a[3])};
  double tot[1];
  block_sum<1>(v, tot);
  if (threadIdx.x == 0) S[blockIdx.x] = tot[0];
}

// One thread per component solves the normal equations over the k filled ring slots: diagonal
// scaling to a unit diagonal, a ridge of kProjRidge (the solutions of consecutive steps are close
// to collinear; the ridge keeps every direction with a damped weight), Cholesky.  Unfilled slots
// and zero columns become identity rows with a zero right-hand side, and a pivot that does not
// stay above half the ridge drops its direction, so their coefficients are 0.  If anything is not
// finite the guess falls back to the newest solution alone.  Every loop has a constant trip count,
// so the arrays live in registers.
__global__ void __launch_bounds__(64) k_proj_solve(int k, int newest, const double *__restrict__ S,
                                                  double *__restrict__ coef) {
  if (threadIdx.x >= 2) return;
  const int c = threadIdx.x;
  const double *T = S + c * kProjPer;
  double a[kProj][kProj], h[kProj], sc[kProj], y[kProj];
  bool use[kProj];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < kProj; i++) {
#pragma unroll
    for (int j = 0; j < kProj; j++) {
      const int lo = i < j ? i : j, hi = i < j ? j : i;
      a[i][j] = T[lo * kProj - lo * (lo - 1) / 2 + (hi - lo)];  // upper triangle, row by row
    }
    h[i] = T[kProjTri + i];
  }
#pragma unroll
  for (int i = 0; i < kProj; i++) {
    const bool live = i < k;
    ok = ok && (!live || (is_finite(a[i][i]) && is_finite(h[i])));
    sc[i] = (live && a[i][i] > 0.0) ? 1.0 / sqrt(a[i][i]) : 0.0;
  }
#pragma unroll
  for (int i = 0; i < kProj; i++) {
#pragma unroll
    for (int j = 0; j < kProj; j++)
      a[i][j] = (sc[i] > 0.0 && sc[j] > 0.0) ? a[i][j] * sc[i] * sc[j] : (i == j ? 1.0 : 0.0);
    a[i][i] += sc[i] > 0.0 ? kProjRidge : 0.0;
    h[i] = sc[i] > 0.0 ? h[i] * sc[i] : 0.0;
  }
  // L L^T in the lower triangle
#pragma unroll
  for (int j = 0; j < kProj; j++) {
    double d = a[j][j];
#pragma unroll
    for (int q = 0; q < j; q++) d -= a[j][q] * a[j][q];
    use[j] = d > 0.5 * kProjRidge;
    const double lj = use[j] ? sqrt(d) : 1.0;
    a[j][j] = lj;
#pragma unroll
    for (int i = j + 1; i < kProj; i++) {
      double v = a[i][j];
#pragma unroll
      for (int q = 0; q < j; q++) v -= a[i][q] * a[j][q];
      a[i][j] = use[j] ? v / lj : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < kProj; i++) {  // L z = h
    double v = h[i];
#pragma unroll
    for (int q = 0; q < i; q++) v -= a[i][q] * y[q];
    y[i] = use[i] ? v / a[i][i] : 0.0;
  }
#pragma unroll
  for (int i = kProj - 1; i >= 0; i--) {  // L^T w = z
    double v = y[i];
#pragma unroll
    for (int q = i + 1; q < kProj; q++) v -= a[q][i] * y[q];
    y[i] = use[i] ? v / a[i][i] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < kProj; i++) {
    y[i] *= sc[i];
    ok = ok && is_finite(y[i]);
  }
#pragma unroll
  for (int i = 0; i < kProj; i++) coef[c * kProj + i] = ok ? y[i] : (i == newest ? 1.0 : 0.0);
}

// x0 = sum_{i<k} c_i U_i per component
__global__ void k_proj_x0(int n, int k, const double2 *__restrict__ hist, const double *__restrict__ coef,
                          double2 *__restrict__ x) {
  __shared__ double cs[2 * kProj];
  if (threadIdx.x < 2 * kProj) cs[threadIdx.x] = coef[threadIdx.x];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2 *h = hist + (size_t)i * kProj;
  double sx = 0.0, sy = 0.0;
  for (int s = 0; s < k; s++) {
    const double2 v = h[s];
    sx += cs[s] * v.x;
    sy += cs[kProj + s] * v.y;
  }
  x[i] = make_double2(sx, sy);
}

// ring slot `slot` of every node <- the new solution
__global__ void k_proj_push(int n, const double2 *__restrict__ ut, double2 *__restrict__ hist, int slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  hist[(size_t)i * kProj + slot] = ut[i];
}

// ------------------------------------------------------------------ iterative refinement (FP32 inner PCG)
// r64 = b - K x in FP64; partials (r.r, b.b)
template <int L>
__global__ void __launch_bounds__(kMaxBlock) k_ir_residual(int n, const int *__restrict__ rp,
                                                          const int *__restrict__ col, const double *__restrict__ A,
                                                          const double *__restrict__ b, const double *__restrict__ x,
                                                          double *__restrict__ r, double *__restrict__ Pout) {
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
  put_partials<2>(acc, Pout);
}

// Outer convergence test and start of the inner solve K32 d = r64 / ||r64||:
// r = r64/||r64|| (FP32), z = D^-1 r, d = 0, p0 = p1 = 0; partials (r.z, r.r, r.r).
__global__ void __launch_bounds__(kMaxBlock) k_ir_inner_init(int Gin, int n, double inner_tol,
                                                            const double *__restrict__ r64,
                                                            const float *__restrict__ dinv, float *__restrict__ r,
                                                            float *__restrict__ z, float *__restrict__ d,
                                                            float *__restrict__ p0, float *__restrict__ p1,
                                                            const double *__restrict__ Pin, double *__restrict__ Pout,
                                                            KrylovState *__restrict__ so, KrylovState *__restrict__ si) {
  double t2[2];
  sum_partials<2>(Pin, Gin, t2);
  const double rn = sqrt(t2[0]), bn = sqrt(t2[1]);
  const bool bad = !is_finite(rn) || !is_finite(bn);
  const bool done = bn == 0.0 || rn <= so->tol * bn;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    so->rnorm[0] = rn;
    so->bnorm[0] = bn;
    so->zero_b[0] = (bn == 0.0);
    so->done[0] = done;
    if (bad) so->status = CGP_E_NONFINITE;
    si->done[0] = done || bad;
    si->status = 0;
    si->iters = 0;
    si->tol = inner_tol_for(inner_tol, so->tol, rn, bn);
  }
  if (done || bad) return;
  const double inv = 1.0 / rn;
  double acc[3] = {0.0, 0.0, 0.0};
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
    acc[2] += (double)rr * (double)rr;
  }
  put_partials<3>(acc, Pout);
}

// x += ||r64|| d (FP64 update of the outer iterate)
__global__ void k_ir_update(int n, double *__restrict__ x, const float *__restrict__ d,
                            const KrylovState *__restrict__ so, const KrylovState *__restrict__ si) {
  if (so->done[0] || so->status || si->status) return;
  const double s = so->rnorm[0];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] += s * (double)d[i];
}

// ------------------------------------------------------------------ Chebyshev iteration (mass solve)
// For P1 triangles the Jacobi-scaled consistent mass matrix has its spectrum in [1/2, 2] on every mesh
// (Wathen 1987: each element's D_e^-1 M_e has the eigenvalues 1/2, 1/2 and 2, and the assembled
// Rayleigh quotient x^T M x / x^T D x lies between the elements' extremes); an eliminated Dirichlet
// row keeps only its diagonal (eigenvalue 1).  With those bounds the Chebyshev iteration needs no
// inner products: one SpMV and a three-term update per step (Saad, Iterative Methods for Sparse
// Linear Systems, 2nd ed., Algorithm 12.1).
constexpr double kChebLo = 0.5, kChebHi = 2.0;

// r = b - M x (the true residual), d = D^-1 r / theta; partials (r.r, b.b) per component
template <int L>
__global__ void __launch_bounds__(kMaxBlock) k_cheb_init(int n, const int *__restrict__ rp,
                                                        const int *__restrict__ col, const double *__restrict__ A,
                                                        const double *__restrict__ dinv, const double2 *__restrict__ b,
                                                        const double2 *__restrict__ x, double2 *__restrict__ r,
                                                        double2 *__restrict__ d, double inv_theta,
                                                        double *__restrict__ Pout) {
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
      const double rx = bb.x - sx, ry = bb.y - sy, di = dinv[row] * inv_theta;
      r[row] = make_double2(rx, ry);
      d[row] = make_double2(di * rx, di * ry);
      acc[0] += rx * rx;
      acc[1] += ry * ry;
      acc[2] += bb.x * bb.x;
      acc[3] += bb.y * bb.y;
    }
  }
  put_partials<4>(acc, Pout);
}

// one step: x += d_k, r -= M d_k, d_{k+1} = c1 d_k + c2 D^-1 r
template <int L>
__global__ void __launch_bounds__(kMaxBlock) k_cheb_step(int n, const int *__restrict__ rp,
                                                        const int *__restrict__ col, const double *__restrict__ A,
                                                        const double *__restrict__ dinv, double2 *__restrict__ x,
                                                        double2 *__restrict__ r, const double2 *__restrict__ dk,
                                                        double2 *__restrict__ dk1, double c1, double c2) {
  const int lane = threadIdx.x & (L - 1);
  const int rows_per_grid = gridDim.x * blockDim.x / L;
  for (int row = (xcd_block() * blockDim.x + threadIdx.x) / L; row < n; row += rows_per_grid) {
    double sx = 0.0, sy = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const double a = A[k];
      const double2 dc = dk[col[k]];
      sx += a * dc.x;
      sy += a * dc.y;
    }
    sx = group_sum<L>(sx);
    sy = group_sum<L>(sy);
    if (lane == 0) {
      const double2 dd = dk[row], xx = x[row], rr = r[row];
      const double di = dinv[row];
      const double rx = rr.x - sx, ry = rr.y - sy;
      x[row] = make_double2(xx.x + dd.x, xx.y + dd.y);
      r[row] = make_double2(rx, ry);
      dk1[row] = make_double2(c1 * dd.x + c2 * (di * rx), c1 * dd.y + c2 * (di * ry));
    }
  }
}

// the init partials into the state: norms, zero right-hand sides (first call), convergence per component
__global__ void __launch_bounds__(256) k_cheb_state(int G, const double *__restrict__ Pin,
                                                   KrylovState *__restrict__ st, int first) {
  double t4[4];
  sum_partials<4>(Pin, G, t4);
  if (threadIdx.x != 0) return;
  for (int c = 0; c < 2; c++) {
    if (first) {
      st->bnorm[c] = sqrt(t4[2 + c]);
      st->zero_b[c] = (t4[2 + c] == 0.0);
    }
    const double rn = sqrt(t4[c]);
    st->rnorm[c] = rn;
    if (!is_finite(rn)) st->status = CGP_E_NONFINITE;
    st->done[c] = st->zero_b[c] || rn <= st->tol * st->bnorm[c];
  }
}

__global__ void k_state_init(KrylovState *st, double tol, int maxit, int ncomp) {
  KrylovState s{};
  s.tol = tol;
  s.maxit = maxit;
  s.ncomp = ncomp;
  *st = s;
}

}  // namespace dev

// ====================================================================== host drivers
using namespace dev;

namespace {

enum { SLOT_MOM = 0, SLOT_P = 1, SLOT_PIN = 2, SLOT_MASS = 3, SLOT_MOMIN = 4 };
// partial-sum regions (each holds up to 8 arrays of kMaxRedGrid doubles)
enum { R_INIT = 0, R_A = 1, R_B = 2, R_C = 3 };

inline double *region(cgp_mesh *m, int k) { return m->red.partials + size_t(k) * 8 * kMaxRedGrid; }

cgp_status poll(cgp_mesh *m, int slot, int count = 1) {
  guess_progress(m);  // host work of a pending online rebuild, while the queued kernels run
  CGP_HIP(hipMemcpyAsync(&m->h_state[slot], m->d_state + slot, sizeof(KrylovState) * count, hipMemcpyDeviceToHost,
                         m->stream));
  CGP_HIP(hipStreamSynchronize(m->stream));
  return CGP_OK;
}

bool host_all_done(const KrylovState &s) {
  for (int c = 0; c < s.ncomp; c++)
    if (!s.done[c]) return false;
  return true;
}

cgp_status status_of(const KrylovState &s, int slot) {
  static const char *names[4] = {"momentum BiCGStab", "Poisson PCG", "Poisson inner PCG", "mass PCG"};
  const std::string what = std::string(names[slot & 3]) + " at iteration " + std::to_string(s.iters);
  if (s.status == CGP_E_NONFINITE) {
    set_error(what + ": non-finite residual or step length");
    return CGP_E_NONFINITE;
  }
  if (s.status == CGP_E_DEVICE) {
    set_error(what + ": persistent Krylov kernel aborted at a grid barrier");
    return CGP_E_DEVICE;
  }
  if (s.status == CGP_E_NOCONV || !host_all_done(s)) {
    set_error(what + ": iteration limit reached (or breakdown)");
    return CGP_E_NOCONV;
  }
  return CGP_OK;
}

// ---- optional HIP-event bracketing of the dominant Poisson kernel
cgp_status kt_harvest(cgp_mesh *m, int done_iters) {
  for (int i = 0; i < m->kt_used; i++) {
    if (m->kt_iter[i] >= done_iters) continue;  // launched after convergence: returned at once
    float ms = 0.0f;
    CGP_HIP(hipEventElapsedTime(&ms, m->kt_ev[2 * i], m->kt_ev[2 * i + 1]));
    m->kt_ms += ms;
    m->kt_count++;
    m->kt_iters++;
  }
  m->kt_used = 0;
  return CGP_OK;
}

void kt_begin(cgp_mesh *m, int iter) {
  if (!m->kt_on) return;
  if (m->kt_used * 2 + 2 > (int)m->kt_ev.size()) {
    const size_t old = m->kt_ev.size();
    m->kt_ev.resize(std::max<size_t>(512, 2 * old));
    m->kt_iter.resize(m->kt_ev.size() / 2);
    for (size_t i = old; i < m->kt_ev.size(); i++) (void)hipEventCreate(&m->kt_ev[i]);
  }
  m->kt_iter[m->kt_used] = iter;
  (void)hipEventRecord(m->kt_ev[2 * m->kt_used], m->stream);
}

void kt_end(cgp_mesh *m) {
  if (!m->kt_on) return;
  (void)hipEventRecord(m->kt_ev[2 * m->kt_used + 1], m->stream);
  m->kt_used++;
}

// Event pair for one launch of the dominant kernel, recorded by the dispatch itself
// (hipExtLaunchKernelGGL), so that it brackets the kernel's own execution; false when not timing.
bool kt_slot(cgp_mesh *m, int iter, hipEvent_t *e0, hipEvent_t *e1) {
  if (!m->kt_on) return false;
  if (m->kt_used * 2 + 2 > (int)m->kt_ev.size()) {
    const size_t old = m->kt_ev.size();
    m->kt_ev.resize(std::max<size_t>(512, 2 * old));
    m->kt_iter.resize(m->kt_ev.size() / 2);
    for (size_t i = old; i < m->kt_ev.size(); i++) (void)hipEventCreate(&m->kt_ev[i]);
  }
  m->kt_iter[m->kt_used] = iter;
  *e0 = m->kt_ev[2 * m->kt_used];
  *e1 = m->kt_ev[2 * m->kt_used + 1];
  m->kt_used++;
  return true;
}

// Launch shapes of one PCG/BiCGStab iteration on a mesh level.
struct LoopShapes {
  Shape rows;   // SpMV-type kernels (lanes per row)
  Shape elem;   // vector kernels (one lane per entry)
};
LoopShapes loop_shapes(const cgp_tuning_knobs &t, int n) {
  return LoopShapes{shape_rows(t, n, t.lanes), shape_rows(t, n, 1)};
}

// Jacobi-PCG loop (init done by the caller, with its partials in R_INIT from a
// grid of G0 blocks): T = double or float vectors.
template <typename T, int NC>
cgp_status pcg_loop(cgp_mesh *m, int slot, int n, const int *rp, const int *col, const T *A, const T *dinv, T *x,
                    T *r, T *z, T *p0, T *p1, T *q, const cgp_tuning_knobs &tk, int G0, int maxit, int *chunk_hint,
                    bool timed, KrylovState *out) {
  KrylovState *st = m->d_state + slot;
  hipStream_t s = m->stream;
  const LoopShapes sh = loop_shapes(tk, n);
  double *Pinit = region(m, R_INIT), *Ppq = region(m, R_A), *Pupd = region(m, R_B);
  int it = 0, chunk = std::max(1, std::min(*chunk_hint, maxit));
  for (;;) {
    dispatch_L(tk.lanes, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      for (int c = 0; c < chunk && it < maxit; c++, it++) {
        T *po = (it & 1) ? p1 : p0, *pn = (it & 1) ? p0 : p1;
        hipEvent_t e0, e1;
        if (timed && kt_slot(m, it, &e0, &e1))
          hipExtLaunchKernelGGL((k_cg_spmv<T, NC, LL>), dim3(sh.rows.grid), dim3(sh.rows.block), 0, s, e0, e1, 0,
                                it == 0 ? G0 : sh.elem.grid, it, n, rp, col, A, (const T *)z, (const T *)po, pn, q,
                                (const double *)(it == 0 ? Pinit : Pupd), Ppq, st);
        else
          hipLaunchKernelGGL((k_cg_spmv<T, NC, LL>), dim3(sh.rows.grid), dim3(sh.rows.block), 0, s,
                             it == 0 ? G0 : sh.elem.grid, it, n, rp, col, A, (const T *)z, (const T *)po, pn, q,
                             (const double *)(it == 0 ? Pinit : Pupd), Ppq, st);
        hipLaunchKernelGGL((k_cg_update<T, NC>), dim3(sh.elem.grid), dim3(sh.elem.block), 0, s, sh.rows.grid, it, n,
                           x, r, z, dinv, (const T *)pn, (const T *)q, (const double *)Ppq, Pupd, st);
      }
    });
    hipLaunchKernelGGL((k_cg_finish<NC>), dim3(1), dim3(256), 0, s, it, it == 0 ? G0 : sh.elem.grid,
                       (const double *)(it == 0 ? Pinit : Pupd), st);
    CGP_HIP(hipGetLastError());
    cgp_status ps = poll(m, slot);
    if (ps) return ps;
    const KrylovState &h = m->h_state[slot];
    if (timed && m->kt_on && (ps = kt_harvest(m, h.iters))) return ps;
    if (h.status || host_all_done(h) || it >= maxit) break;
    chunk = std::max(8, it / 16);  // later chunks grow: fewer polls, bounded overshoot
  }
  *out = m->h_state[slot];
  *chunk_hint = out->iters + 1;  // stable counts (mass solves): the next solve usually needs one poll
  return CGP_OK;
}

template <int NC>
cgp_status run_pcg64(cgp_mesh *m, int slot, int n, const int *rp, const int *col, const double *A,
                     const double *dinv, const double *b, double *x, double **w, const cgp_tuning_knobs &tk,
                     double tol, int maxit, int *chunk_hint, bool timed, KrylovState *out) {
  KrylovState *st = m->d_state + slot;
  hipStream_t s = m->stream;
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, tol, maxit, NC);
  const Shape init = shape_rows(tk, n, tk.lanes);
  dispatch_L(tk.lanes, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    hipLaunchKernelGGL((k_cg_init<NC, LL>), dim3(init.grid), dim3(init.block), 0, s, n, rp, col, A, b,
                       (const double *)x, dinv, w[0], w[1], w[2], w[3], region(m, R_INIT));
  });
  cgp_status ls = pcg_loop<double, NC>(m, slot, n, rp, col, A, dinv, x, w[0], w[1], w[2], w[3], w[4], tk, init.grid,
                                       maxit, chunk_hint, timed, out);
  if (ls) return ls;
  hipLaunchKernelGGL((k_zero_b_fix<NC>), dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const KrylovState *)st);
  return status_of(*out, slot);
}

// Single-kernel PCG loop.  Precondition: records of slot 0 hold {r0, -, 0, D^-1} with
// r0 = b - K x0 (or the normalised refinement residual), slot 1 holds D^-1, p = 0, and the
// b.b partials are in R_INIT from a grid of g_first blocks.
constexpr int kCg1DirectGrid = 256;  // largest grid whose partials every wave of the next iteration sums itself

// Kernel variant for a launch shape: lanes L, rows per lane group P (1 or 2, more by looping), partial
// sums read U per lane ahead, E entries per lane ahead of the scalars.  `tree`: the partials arrive
// summed (one value per total) and the sizes are bandwidth-bound, so nothing is loaded ahead and the
// kernel keeps its registers low for occupancy.
template <typename F>
void dispatch_cg1(int lanes, int passes, int grid, bool tree, F &&f) {
  auto with_LP = [&](auto LC, auto PC) {
    constexpr int LL = decltype(LC)::value;
    if (tree) f(LC, PC, std::integral_constant<int, 1>{}, std::integral_constant<int, 0>{});
    else if (grid > 256) f(LC, PC, std::integral_constant<int, 8>{}, std::integral_constant<int, cg1_ahead<LL>()>{});
    else f(LC, PC, std::integral_constant<int, 4>{}, std::integral_constant<int, cg1_ahead<LL>()>{});
  };
  auto with_L = [&](auto LC) {
    if (passes >= 2) with_LP(LC, std::integral_constant<int, 2>{});
    else with_LP(LC, std::integral_constant<int, 1>{});
  };
  switch (lanes) {
    case 2: with_L(std::integral_constant<int, 2>{}); break;
    case 4: with_L(std::integral_constant<int, 4>{}); break;
    case 16: with_L(std::integral_constant<int, 16>{}); break;
    default: with_L(std::integral_constant<int, 8>{}); break;
  }
}

// The graph entry of this argument set, created empty (captured on first use); at most 8 are kept, the
// oldest replaced after the stream has drained (one of its graphs may still be queued).
cgp_status cg1_graph_for(cgp_mesh *m, const uintptr_t (&key)[Cg1Graph::kKey], Cg1Graph **out) {
  for (Cg1Graph &g : m->cg1_graphs)
    if (std::equal(key, key + Cg1Graph::kKey, g.key)) {
      *out = &g;
      return CGP_OK;
    }
  if (!m->cap_stream) CGP_HIP(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
  if (m->cg1_graphs.size() >= 8) {
    CGP_HIP(hipStreamSynchronize(m->stream));
    for (hipGraphExec_t &x : m->cg1_graphs.front().gx)
      if (x) (void)hipGraphExecDestroy(x);
    m->cg1_graphs.erase(m->cg1_graphs.begin());
  }
  m->cg1_graphs.emplace_back();
  std::copy(key, key + Cg1Graph::kKey, m->cg1_graphs.back().key);
  *out = &m->cg1_graphs.back();
  return CGP_OK;
}

template <typename T>
cgp_status cg1_loop(cgp_mesh *m, int slot, int n, const int *rp, const int *col, const T *A, T *x, T *p,
                    rec_t<T> *const R[2], const cgp_tuning_knobs &tk, int g_first, int maxit, int *chunk_hint,
                    bool timed, KrylovState *out) {
  KrylovState *st = m->d_state + slot;
  hipStream_t s = m->stream;
  const Shape sh = shape_rows(tk, n, tk.lanes);
  double *Pw = region(m, R_A);
  // above 256 blocks the partials of each iteration are first summed by one block (k_cg1_total)
  const bool tree = sh.grid > kCg1DirectGrid;
  double *Ptot = region(m, R_INIT) + 4 * kMaxRedGrid;  // 3 totals, clear of the init partials
  const int gin = tree ? 1 : sh.grid;
  auto pin = [&](int it) {
    if (tree) return Ptot;
    return it == 0 ? Pw : region(m, ((it - 1) & 1) ? R_C : R_B);
  };
  auto pout = [&](int it) { return region(m, (it & 1) ? R_C : R_B); };
  dispatch_L(tk.lanes, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    hipLaunchKernelGGL((k_cg1_init_w<T, LL>), dim3(sh.grid), dim3(sh.block), 0, s, g_first, n, rp, col, A, R[0],
                       (const double *)region(m, R_INIT), Pw, st);
  });
  if (tree) hipLaunchKernelGGL(k_cg1_total, dim3(1), dim3(1024), 0, s, sh.grid, (const double *)Pw, Ptot, st);
  // one iteration (and its total when the grid is large) enqueued on stream q; e0/e1: event pair
  auto launch_one = [&](hipStream_t q, int i, hipEvent_t e0, hipEvent_t e1) {
    dispatch_cg1(tk.lanes, tk.passes, sh.grid, tree, [&](auto LC, auto PC, auto UC, auto EC) {
      constexpr int LL = decltype(LC)::value, PP = decltype(PC)::value, UU = decltype(UC)::value;
      constexpr int EE = decltype(EC)::value;
      const int cur = i & 1, nxt = cur ^ 1;
      if (e0)
        hipExtLaunchKernelGGL((k_cg1_iter<T, LL, PP, UU, EE>), dim3(sh.grid), dim3(sh.block), 0, q, e0, e1, 0, gin, i,
                              n, rp, col, A, x, p, (const rec_t<T> *)R[cur], R[nxt], (const double *)pin(i),
                              pout(i), st);
      else
        hipLaunchKernelGGL((k_cg1_iter<T, LL, PP, UU, EE>), dim3(sh.grid), dim3(sh.block), 0, q, gin, i, n, rp, col,
                           A, x, p, (const rec_t<T> *)R[cur], R[nxt], (const double *)pin(i), pout(i), st);
    });
    if (tree) hipLaunchKernelGGL(k_cg1_total, dim3(1), dim3(1024), 0, q, sh.grid, (const double *)pout(i), Ptot, st);
  };
  // Without event timing, runs of kCg1GraphChunk iterations go out as one launch of a captured graph:
  // the chunk from iteration 0, or the one captured at iterations kCg1GraphChunk.. (even length, so a
  // replay at any even iteration reads and writes the same slots).  Graphs are kept per argument set.
  Cg1Graph *gr = nullptr;
  if (m->tune.pcg_graph && !(timed && m->kt_on)) {
    const uintptr_t key[Cg1Graph::kKey] = {sizeof(T), (uintptr_t)n, (uintptr_t)rp, (uintptr_t)col, (uintptr_t)A,
                                           (uintptr_t)x, (uintptr_t)p, (uintptr_t)R[0], (uintptr_t)R[1],
                                           (uintptr_t)st, (uintptr_t)Pw, (uintptr_t)sh.grid, (uintptr_t)sh.block,
                                           (uintptr_t)(tk.lanes * 64 + tk.passes)};
    cgp_status gs = cg1_graph_for(m, key, &gr);
    if (gs) return gs;
  }
  auto graph_exec = [&](int which) -> hipGraphExec_t {
    if (!gr->gx[which]) {
      hipGraph_t g = nullptr;
      hipStream_t q = m->cap_stream;
      if (hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
      const int i0 = which == 0 ? 0 : kCg1GraphChunk;
      for (int c = 0; c < kCg1GraphChunk; c++) launch_one(q, i0 + c, nullptr, nullptr);
      if (hipStreamEndCapture(q, &g) != hipSuccess || !g) return nullptr;
      if (hipGraphInstantiate(&gr->gx[which], g, nullptr, nullptr, 0) != hipSuccess) gr->gx[which] = nullptr;
      (void)hipGraphDestroy(g);
    }
    return gr->gx[which];
  };
  int it = 0, chunk = std::max(1, std::min(*chunk_hint, maxit));
  for (;;) {
    const int end = std::min(maxit, it + chunk);
    while (it < end) {
      if (gr && end - it >= kCg1GraphChunk && (it & 1) == 0) {
        hipGraphExec_t gx = graph_exec(it == 0 ? 0 : 1);
        if (!gx) {
          set_error("cg1_loop: capturing the PCG iteration graph failed");
          return CGP_E_DEVICE;
        }
        CGP_HIP(hipGraphLaunch(gx, s));
        it += kCg1GraphChunk;
        continue;
      }
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timed) kt_slot(m, it, &e0, &e1);
      launch_one(s, it, e0, e1);
      it++;
    }
    hipLaunchKernelGGL(k_cg1_finish, dim3(1), dim3(256), 0, s, gin, (const double *)pin(it), st);
    CGP_HIP(hipGetLastError());
    cgp_status ps = poll(m, slot);
    if (ps) return ps;
    const KrylovState &h = m->h_state[slot];
    if (timed && m->kt_on && (ps = kt_harvest(m, h.iters))) return ps;
    if (h.status || h.done[0] || it >= maxit) break;
    chunk = std::max(8, it / 16);  // later chunks grow: fewer polls, bounded overshoot
  }
  *out = m->h_state[slot];
  *chunk_hint = std::max(1, out->iters - 2);
  return CGP_OK;
}

}  // namespace

// BiCGStab iterations (both components) from the state and partials an init kernel left: T = double
// (the FP64 solve; x is the solution) or float (the inner solve of the refinement; x is its
// correction).  Chunks of iterations, each followed by a state poll; *chunk_hint is the next solve's
// first chunk (its count + 1: momentum counts are stable, so usually one poll per solve).
template <typename T>
cgp_status bicg_loop(cgp_mesh *m, int slot, int n, const T *A, const T *dinv, typename v2_of<T>::type *x,
                     typename v2_of<T>::type *r, typename v2_of<T>::type *rh, typename v2_of<T>::type *p,
                     typename v2_of<T>::type *v, typename v2_of<T>::type *t, typename v2_of<T>::type *ph,
                     int g_init, int maxit, int *chunk_hint) {
  using V2 = typename v2_of<T>::type;
  hipStream_t s = m->stream;
  KrylovState *st = m->d_state + slot;
  const cgp_tuning_knobs &tk = m->tune.fine;
  const LoopShapes sh = loop_shapes(tk, n);
  const int *rp = m->d_rp_f, *col = m->d_col_f;
  double *Pinit = region(m, R_INIT), *Pv = region(m, R_A), *Pt = region(m, R_B), *Px = region(m, R_C);
  int it = 0, chunk = std::max(1, std::min(*chunk_hint, maxit));
  for (;;) {
    dispatch_L(tk.lanes, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      for (int c = 0; c < chunk && it < maxit; c++, it++) {
        // the first direction p = r0 (and the first convergence test); later ones come with the update
        if (it == 0)
          hipLaunchKernelGGL(k_bi_p<T>, dim3(sh.elem.grid), dim3(sh.elem.block), 0, s, g_init, 0, n, (const V2 *)r,
                             p, (const V2 *)v, dinv, ph, (const double *)Pinit, st);
        hipLaunchKernelGGL((k_bi_vc<T, LL>), dim3(sh.rows.grid), dim3(sh.rows.block), 0, s, sh.elem.grid, it, n, rp,
                           col, A, (const V2 *)ph, v, (const V2 *)rh, (const double *)Px, Pv, st);
        hipLaunchKernelGGL((k_bi_t<T, LL>), dim3(sh.rows.grid), dim3(sh.rows.block), 0, s, sh.rows.grid, it, n, rp,
                           col, A, (const V2 *)r, (const V2 *)v, (const V2 *)rh, dinv, t, (const double *)Pv, Pt,
                           st);
        hipLaunchKernelGGL(k_bi_xp<T>, dim3(sh.elem.grid), dim3(sh.elem.block), 0, s, sh.rows.grid, it, n, x, r, p,
                           (const V2 *)v, (const V2 *)t, dinv, ph, (const double *)Pt, Px, st);
      }
    });
    hipLaunchKernelGGL(k_bi_finish, dim3(1), dim3(256), 0, s, it, it == 0 ? g_init : sh.elem.grid,
                       (const double *)(it == 0 ? Pinit : Px), st);
    CGP_HIP(hipGetLastError());
    cgp_status ps = poll(m, slot);
    if (ps) return ps;
    const KrylovState &h = m->h_state[slot];
    if (h.status || host_all_done(h) || it >= maxit) break;
    chunk = 2;
  }
  *chunk_hint = std::max(1, m->h_state[slot].iters + 1);
  return CGP_OK;
}

// FP32 inner BiCGStab inside FP64 iterative refinement (outer state SLOT_MOM, inner SLOT_MOMIN):
// r64 = b - A x, outer test, inner solve of A d = r64 / ||r64|| in FP32 to the reduction still
// needed, x += ||r64|| d, until both components meet the tolerance.  The FP32 matrix and vectors
// are allocated at the first such solve.
cgp_status momentum_ir(cgp_mesh *m, const cgp_solver_opts *o, const double2 *b, double2 *x, int *inner_total) {
  hipStream_t s = m->stream;
  const int n = m->pf.n;
  const long nnz = m->pf.nnz;
  if (!m->d_A32) {
    void *q = nullptr;
    CGP_HIP(hipMalloc(&q, sizeof(float) * ((size_t)nnz + (size_t)n)));
    m->allocations.push_back(q);
    m->d_A32 = (float *)q;
    m->d_dinvA32 = m->d_A32 + nnz;
    CGP_HIP(hipMalloc(&q, sizeof(float2) * 7 * (size_t)n));
    m->allocations.push_back(q);
    m->d_wf32 = (float2 *)q;
  }
  const cgp_tuning_knobs &tk = m->tune.fine;
  const LoopShapes sh = loop_shapes(tk, n);
  hipLaunchKernelGGL(k_mir_convert, dim3(std::min<long>(4096, (nnz + 255) / 256)), dim3(256), 0, s, nnz, n,
                     (const double *)m->d_A, (const double *)m->d_dinvA, m->d_A32, m->d_dinvA32);
  float2 *w = m->d_wf32;
  float2 *r = w, *rh = w + n, *p = w + 2 * (size_t)n, *v = w + 3 * (size_t)n, *t = w + 4 * (size_t)n,
         *ph = w + 5 * (size_t)n, *d = w + 6 * (size_t)n;
  double2 *r64 = (double2 *)m->d_wf[1];
  KrylovState *so = m->d_state + SLOT_MOM, *si = m->d_state + SLOT_MOMIN;
  const double inner_tol = o->inner_tol > 0 ? o->inner_tol : 1e-5;
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, si, inner_tol, o->max_iter, 2);
  *inner_total = 0;
  for (int outer = 0; outer < 50; outer++) {
    dispatch_L(tk.lanes, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_mir_residual<LL>), dim3(sh.rows.grid), dim3(sh.rows.block), 0, s, n, m->d_rp_f,
                         m->d_col_f, (const double *)m->d_A, b, (const double2 *)x, r64, region(m, R_C));
    });
    hipLaunchKernelGGL(k_mir_init, dim3(sh.elem.grid), dim3(sh.elem.block), 0, s, sh.rows.grid, n, inner_tol,
                       (const double2 *)r64, r, rh, p, v, d, (const double *)region(m, R_C), region(m, R_INIT), so,
                       si);
    const int budget = std::max(1, o->max_iter - *inner_total);
    cgp_status ls = bicg_loop<float>(m, SLOT_MOMIN, n, m->d_A32, m->d_dinvA32, d, r, rh, p, v, t, ph, sh.elem.grid,
                                     budget, &m->mom32_chunk);
    if (ls) return ls;
    cgp_status ps = poll(m, SLOT_MOM);
    if (ps) return ps;
    const KrylovState ho = m->h_state[SLOT_MOM], hi = m->h_state[SLOT_MOMIN];
    if (ho.status || host_all_done(ho)) break;
    if (hi.status) {
      m->h_state[SLOT_MOM].status = hi.status;
      break;
    }
    *inner_total += hi.iters;
    hipLaunchKernelGGL(k_mir_update, dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const float2 *)d,
                       (const KrylovState *)so);
    if (*inner_total >= o->max_iter) {  // the residual of the last iterate, for the report
      dispatch_L(tk.lanes, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_mir_residual<LL>), dim3(sh.rows.grid), dim3(sh.rows.block), 0, s, n, m->d_rp_f,
                           m->d_col_f, (const double *)m->d_A, b, (const double2 *)x, r64, region(m, R_C));
      });
      hipLaunchKernelGGL(k_mir_init, dim3(sh.elem.grid), dim3(sh.elem.block), 0, s, sh.rows.grid, n, inner_tol,
                         (const double2 *)r64, r, rh, p, v, d, (const double *)region(m, R_C), region(m, R_INIT),
                         so, si);
      if ((ps = poll(m, SLOT_MOM))) return ps;
      if (!host_all_done(m->h_state[SLOT_MOM])) m->h_state[SLOT_MOM].status = CGP_E_NOCONV;
      break;
    }
  }
  CGP_HIP(hipGetLastError());
  return CGP_OK;
}

// ------------------------------------------------------------------ step 1
cgp_status drv_momentum(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *f, const double *u,
                        double *ut, cgp_stats *stats, const double *pn) {
  hipStream_t s = m->stream;
  const int n = m->pf.n;
  launch_conv_assembly(m, u);  // A = S + dt N(U^n), every entry
  double2 *rhs = (double2 *)m->d_wf[0];
  launch_mom_rhs(m, g, u, f, pn, (double *)rhs);
  const bool extrap = (o->x0_mode == CGP_X0_EXTRAP && ut == m->d_ut);
  const bool project = (o->x0_mode == CGP_X0_PROJECT && ut == m->d_ut);
  if (project && !m->d_uhist) {
    const size_t hb = (size_t)kProj * 2 * n * sizeof(double);
    const size_t pb = (2 * (size_t)kProjPer * kProjGrid + 2 * kProj + 2 * kProjPer) * sizeof(double);
    void *q = nullptr;
    CGP_HIP(hipMalloc(&q, hb));
    m->allocations.push_back(q);
    m->d_uhist = (double *)q;
    CGP_HIP(hipMalloc(&q, pb));
    m->allocations.push_back(q);
    m->d_proj = (double *)q;
    CGP_HIP(hipMemsetAsync(m->d_uhist, 0, hb, s));  // unused slots hold finite values
    m->uh_count = m->uh_head = 0;
  }
  if (!project) m->uh_count = m->uh_head = 0;  // the ring fills from slot 0 again
  if (project && m->uh_count > 0) {
    // x0 from the ring (A and rhs above are the eliminated system of this step)
    const int k = m->uh_count, newest = (m->uh_head + kProj - 1) % kProj;
    const int tiles = (n + 63) / 64;
    const int G = std::max(8, std::min(kProjGrid, (tiles + 7) / 8 * 8));
    double *coef = m->d_proj + 2 * (size_t)kProjPer * kProjGrid;
    hipLaunchKernelGGL((k_proj_gram<4>), dim3(G), dim3(256), 0, s, n, m->d_rp_f, m->d_col_f, (const double *)m->d_A,
                       m->d_vdir, (const double2 *)m->d_uhist, (const double2 *)rhs, m->d_proj);
    double *sums = coef + 2 * kProj;
    hipLaunchKernelGGL(k_proj_sum, dim3(2 * kProjPer), dim3(256), 0, s, G, (const double *)m->d_proj, sums);
    hipLaunchKernelGGL(k_proj_solve, dim3(1), dim3(64), 0, s, k, newest, (const double *)sums, coef);
    hipLaunchKernelGGL(k_proj_x0, dim3(blocks_1d(n)), dim3(256), 0, s, n, k, (const double2 *)m->d_uhist,
                       (const double *)coef, (double2 *)ut);
  } else if (project) {
    CGP_HIP(hipMemcpyAsync(ut, u, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else if (extrap && m->ut_hist >= 3) {
    // d_ut, d_ut_prev, d_ut_prev2 hold U~^n, U~^(n-1), U~^(n-2): x0 = 3 U~^n - 3 U~^(n-1) + U~^(n-2)
    // (quadratic in time), and the history shifts by one step
    launch_extrapolate3(m, 2 * n, m->d_ut, m->d_ut_prev, m->d_ut_prev2);
  } else if (extrap && m->ut_hist == 2) {
    // x0 = 2 U~^n - U~^(n-1); U~^(n-1) moves to d_ut_prev2, U~^n to d_ut_prev
    CGP_HIP(hipMemcpyAsync(m->d_ut_prev2, m->d_ut_prev, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_extrapolate(m, 2 * n, m->d_ut, m->d_ut_prev);
  } else {
    if (extrap && m->ut_hist == 1)
      CGP_HIP(hipMemcpyAsync(m->d_ut_prev, m->d_ut, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if (o->x0_mode == CGP_X0_ZERO)
      CGP_HIP(hipMemsetAsync(ut, 0, 2 * n * sizeof(double), s));
    else
      CGP_HIP(hipMemcpyAsync(ut, u, 2 * n * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  m->ut_hist = extrap ? std::min(m->ut_hist + 1, 3) : 0;
  // known values in the initial guess: the eliminated Dirichlet rows then start (and stay) exact
  launch_set_dirichlet(m, g, ut);
  KrylovState *st = m->d_state + SLOT_MOM;
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, o->tol, o->max_iter, 2);
  const cgp_tuning_knobs &tk = m->tune.fine;
  const LoopShapes sh = loop_shapes(tk, n);
  double2 *x = (double2 *)ut;
  int mom_iters = 0;
  if (o->precision == CGP_PREC_FP32_IR) {
    cgp_status ls = momentum_ir(m, o, (const double2 *)rhs, x, &mom_iters);
    if (ls) return ls;
  } else {
    double2 *r = (double2 *)m->d_wf[1], *rh = (double2 *)m->d_wf[2], *p = (double2 *)m->d_wf[3];
    double2 *v = (double2 *)m->d_wf[4], *t = (double2 *)m->d_wf[5], *ph = (double2 *)m->d_wf[6];
    double *Pinit = region(m, R_INIT);
    dispatch_L(tk.lanes, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_bi_init<LL>), dim3(sh.rows.grid), dim3(sh.rows.block), 0, s, n, m->d_rp_f, m->d_col_f,
                         (const double *)m->d_A, (const double2 *)rhs, (const double2 *)x, r, rh, p, v, Pinit);
    });
    cgp_status ls = bicg_loop<double>(m, SLOT_MOM, n, m->d_A, m->d_dinvA, x, r, rh, p, v, t, ph, sh.rows.grid,
                                      o->max_iter, &m->mom_chunk);
    if (ls) return ls;
    mom_iters = m->h_state[SLOT_MOM].iters;
  }
  hipLaunchKernelGGL((k_zero_b_fix<2>), dim3(blocks_1d(n)), dim3(256), 0, s, n, ut, (const KrylovState *)st);
  KrylovState h = m->h_state[SLOT_MOM];
  h.iters = mom_iters;
  if (project && status_of(h, SLOT_MOM) == CGP_OK) {
    hipLaunchKernelGGL(k_proj_push, dim3(blocks_1d(n)), dim3(256), 0, s, n, (const double2 *)ut,
                       (double2 *)m->d_uhist, m->uh_head);
    m->uh_head = (m->uh_head + 1) % kProj;
    m->uh_count = std::min(m->uh_count + 1, kProj);
  } else {
    m->uh_count = m->uh_head = 0;
  }
  if (stats) {
    stats->mom_iters = mom_iters;
    stats->mom_relres = 0.0;
    for (int c = 0; c < 2; c++)
      stats->mom_relres = std::max(stats->mom_relres, h.bnorm[c] > 0 ? h.rnorm[c] / h.bnorm[c] : 0.0);
  }
  return status_of(h, SLOT_MOM);
}

// ------------------------------------------------------------------ step 3
namespace {

// FP32 Jacobi-PCG inside FP64 iterative refinement, launch-per-phase loop or persistent inner kernel.
cgp_status poisson_ir(cgp_mesh *m, const double *b, double *x, const cgp_solver_opts *o, bool persistent, bool fused,
                      KrylovState *fin, int *total_iters, int *outer_out) {
  hipStream_t s = m->stream;
  const int n = m->pc.n;
  const cgp_tuning_knobs &tk = m->tune.coarse;
  const LoopShapes sh = loop_shapes(tk, n);
  KrylovState *so = m->d_state + SLOT_P, *si = m->d_state + SLOT_PIN;
  double *r64 = m->d_wc[1];
  float *r = m->d_wc32[0], *z = m->d_wc32[1], *d = m->d_wc32[2], *p0 = m->d_wc32[3], *p1 = m->d_wc32[4],
        *q = m->d_wc32[5];
  float4 *f1R[2] = {reinterpret_cast<float4 *>(m->d_rec), reinterpret_cast<float4 *>(m->d_rec) + n};
  float *f1p = m->d_wc32[7];
  const double inner_tol = o->inner_tol > 0 ? o->inner_tol : 1e-4;
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, so, o->tol, o->max_iter, 1);
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, si, inner_tol, o->max_iter, 1);
  auto residual = [&]() {
    dispatch_L(tk.lanes, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_ir_residual<LL>), dim3(sh.rows.grid), dim3(sh.rows.block), 0, s, n, m->d_rp_c,
                         m->d_col_c, (const double *)m->d_Kbc, b, (const double *)x, r64, region(m, R_C));
    });
    if (fused)
      hipLaunchKernelGGL(k_cg1_ir_init, dim3(sh.elem.grid), dim3(sh.elem.block), 0, s, sh.rows.grid, n, inner_tol,
                         (const double *)r64, (const float *)m->d_dinvK32, f1R[0], f1R[1], d, f1p,
                         (const double *)region(m, R_C), region(m, R_INIT), so, si);
    else
      hipLaunchKernelGGL(k_ir_inner_init, dim3(sh.elem.grid), dim3(sh.elem.block), 0, s, sh.rows.grid, n,
                         inner_tol, (const double *)r64, (const float *)m->d_dinvK32, r, z, d, p0, p1,
                         (const double *)region(m, R_C), region(m, R_INIT), so, si);
  };
  int outer = 0;
  *total_iters = 0;
  for (outer = 0; outer < 200; outer++) {
    residual();
    const int budget = std::max(1, o->max_iter - *total_iters);
    KrylovState hi{};
    if (persistent) {
      void *w[5] = {r, z, p0, p1, q};
      kt_begin(m, 0);
      cgp_status ls = persistent_pcg(m, true, nullptr, d, w, inner_tol, budget, si, so, r64);
      kt_end(m);
      if (ls) return ls;
      cgp_status ps = poll(m, SLOT_P, 2);
      if (ps) return ps;
      hi = m->h_state[SLOT_PIN];
      if (m->kt_on) {
        const int used = m->kt_used;
        if ((ps = kt_harvest(m, m->h_state[SLOT_P].done[0] ? 0 : 1))) return ps;
        if (!m->h_state[SLOT_P].done[0]) m->kt_iters += (long)hi.iters - used;
      }
    } else if (fused) {
      cgp_status ls = cg1_loop<float>(m, SLOT_PIN, n, m->d_rp_c, m->d_col_c, (const float *)m->d_Kbc32, d, f1p, f1R,
                                      tk, sh.elem.grid, budget, &m->p32_chunk[std::min(outer, 3)], true, &hi);
      if (ls) return ls;
      cgp_status ps = poll(m, SLOT_P);
      if (ps) return ps;
    } else {
      cgp_status ls = pcg_loop<float, 1>(m, SLOT_PIN, n, m->d_rp_c, m->d_col_c, (const float *)m->d_Kbc32,
                                         (const float *)m->d_dinvK32, d, r, z, p0, p1, q, tk, sh.elem.grid, budget,
                                         &m->p32_chunk[std::min(outer, 3)], true, &hi);
      if (ls) return ls;
      cgp_status ps = poll(m, SLOT_P);
      if (ps) return ps;
    }
    const KrylovState ho = m->h_state[SLOT_P];
    if (ho.done[0] || ho.status) {
      *fin = ho;
      break;
    }
    if (hi.status) {
      *fin = hi;
      break;
    }
    *total_iters += hi.iters;
    hipLaunchKernelGGL(k_ir_update, dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const float *)d,
                       (const KrylovState *)so, (const KrylovState *)si);
    if (*total_iters >= o->max_iter) {
      residual();  // residual of the last iterate, for the report
      cgp_status ps = poll(m, SLOT_P);
      if (ps) return ps;
      *fin = m->h_state[SLOT_P];
      outer++;
      break;
    }
  }
  hipLaunchKernelGGL((k_zero_b_fix<1>), dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const KrylovState *)so);
  *outer_out = outer + 1;
  return status_of(*fin, SLOT_P);
}

}  // namespace

cgp_status drv_poisson(cgp_mesh *m, const double *b_in, double *x, const cgp_solver_opts *o, cgp_stats *stats) {
  hipStream_t s = m->stream;
  const int n = m->pc.n;
  double *b = m->d_wc[0];
  CGP_HIP(hipMemcpyAsync(b, b_in, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (o->x0_mode == CGP_X0_ZERO) CGP_HIP(hipMemsetAsync(x, 0, n * sizeof(double), s));
  if (m->n_pdir > 0) {
    launch_pdir_zero(m, b, x);
  } else {
    // pure Neumann (Eq. 13 on all of the boundary): project b onto the range of Kbar
    launch_mean_shift(m, b, nullptr, double(n), region(m, R_A));
  }
  if (o->x0_mode >= CGP_X0_LEARNED) {
    cgp_status gs = guess_initial(m, o->x0_mode, b, x);
    if (gs) return gs;
    if (m->n_pdir > 0) launch_pdir_zero(m, b, x);  // the guess knows nothing of p = 0 on the outflow
  }
  const bool persistent = (o->launch == CGP_LAUNCH_PERSISTENT);
  const bool fused = (o->launch == CGP_LAUNCH_FUSED || o->launch == CGP_LAUNCH_AUTO);
  if (persistent) {
    cgp_status ss = persistent_setup(m);
    if (ss) return ss;
  }
  KrylovState fin{};
  cgp_status rs = CGP_OK;
  int total_iters = 0, outer = 1;
  if (o->method == CGP_METHOD_ILU_GMRES) {
    cgp_status gs = gmres_solve(m, b, x, o, &fin);
    if (gs) return gs;
    rs = status_of(fin, SLOT_P);
    total_iters = fin.iters;
  } else if (o->precision == CGP_PREC_FP64) {
    if (persistent) {
      void *w[5] = {m->d_wc[1], m->d_wc[2], m->d_wc[3], m->d_wc[4], m->d_wc[5]};
      KrylovState *so = m->d_state + SLOT_P;
      hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, so, o->tol, o->max_iter, 1);
      kt_begin(m, 0);
      cgp_status ls = persistent_pcg(m, false, b, x, w, o->tol, o->max_iter, so, nullptr, nullptr);
      kt_end(m);
      if (ls) return ls;
      hipLaunchKernelGGL((k_zero_b_fix<1>), dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const KrylovState *)so);
      cgp_status ps = poll(m, SLOT_P);
      if (ps) return ps;
      fin = m->h_state[SLOT_P];
      if (m->kt_on) {
        const int used = m->kt_used;
        if ((ps = kt_harvest(m, 1))) return ps;
        m->kt_iters += (long)fin.iters - used;
      }
      rs = status_of(fin, SLOT_P);
    } else if (fused) {
      KrylovState *so = m->d_state + SLOT_P;
      const cgp_tuning_knobs &tk = m->tune.coarse;
      const Shape sh = shape_rows(tk, n, tk.lanes);
      double4 *R[2] = {reinterpret_cast<double4 *>(m->d_rec), reinterpret_cast<double4 *>(m->d_rec) + n};
      double *p = m->d_wc[7];
      hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, so, o->tol, o->max_iter, 1);
      dispatch_L(tk.lanes, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_cg1_init_r<LL>), dim3(sh.grid), dim3(sh.block), 0, s, n, m->d_rp_c, m->d_col_c,
                           (const double *)m->d_Kbc, (const double *)m->d_dinvK, (const double *)b,
                           (const double *)x, p, R[0], R[1], region(m, R_INIT));
      });
      cgp_status ls = cg1_loop<double>(m, SLOT_P, n, m->d_rp_c, m->d_col_c, (const double *)m->d_Kbc, x, p, R, tk,
                                       sh.grid, o->max_iter, &m->p_chunk, true, &fin);
      if (ls) return ls;
      hipLaunchKernelGGL((k_zero_b_fix<1>), dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const KrylovState *)so);
      rs = status_of(fin, SLOT_P);
    } else {
      double *w[5] = {m->d_wc[1], m->d_wc[2], m->d_wc[3], m->d_wc[4], m->d_wc[5]};
      rs = run_pcg64<1>(m, SLOT_P, n, m->d_rp_c, m->d_col_c, m->d_Kbc, m->d_dinvK, b, x, w, m->tune.coarse, o->tol,
                        o->max_iter, &m->p_chunk, true, &fin);
    }
    total_iters = fin.iters;
  } else {
    rs = poisson_ir(m, b, x, o, persistent, fused && !persistent, &fin, &total_iters, &outer);
  }
  if (rs != CGP_OK && rs != CGP_E_NOCONV) return rs;
  if (m->n_pdir == 0) launch_mean_shift(m, x, m->d_mc, m->mc_sum, region(m, R_A));  // zero weighted mean
  CGP_HIP(hipGetLastError());
  if (rs == CGP_OK) {
    cgp_status gs = guess_record(m, x);
    if (gs) return gs;
  }
  if (stats) {
    stats->p_iters = total_iters;
    stats->p_outer = outer;
    stats->p_relres = fin.bnorm[0] > 0 ? fin.rnorm[0] / fin.bnorm[0] : 0.0;
  }
  return rs;
}

// ------------------------------------------------------------------ step 5
// Chebyshev iteration for the consistent mass matrix (two components), from x: cycles of steps,
// each closed by the true residual and one poll.  The first cycle runs as many steps as the last solve
// needed (*hint); a later one as many as the bound 2 q^k on the M-norm error (q = 1/3 for kappa = 4)
// asks for the remaining reduction, plus two for the residual's 2-norm.
cgp_status cheb_mass(cgp_mesh *m, int n, const double *b, double *x, double **w, const cgp_tuning_knobs &tk,
                     double tol, int maxit, int *hint, KrylovState *out) {
  KrylovState *st = m->d_state + SLOT_MASS;
  hipStream_t s = m->stream;
  double2 *r = reinterpret_cast<double2 *>(w[0]);
  double2 *d[2] = {reinterpret_cast<double2 *>(w[1]), reinterpret_cast<double2 *>(w[2])};
  const Shape sh = shape_rows(tk, n, tk.lanes);
  const double theta = 0.5 * (kChebHi + kChebLo), delta = 0.5 * (kChebHi - kChebLo), sigma = theta / delta;
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, tol, maxit, 2);
  auto check = [&](bool first) {
    dispatch_L(tk.lanes, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_cheb_init<LL>), dim3(sh.grid), dim3(sh.block), 0, s, n, m->d_rp_f, m->d_col_f,
                         (const double *)m->d_Mbc, (const double *)m->d_dinvM, (const double2 *)b,
                         (const double2 *)x, r, d[0], 1.0 / theta, region(m, R_INIT));
    });
    hipLaunchKernelGGL(k_cheb_state, dim3(1), dim3(256), 0, s, sh.grid, (const double *)region(m, R_INIT), st,
                       first ? 1 : 0);
  };
  check(true);
  int used = 0, k = std::max(1, std::min(*hint, maxit));
  for (;;) {
    double rho = 1.0 / sigma;
    for (int j = 0; j < k; j++) {
      const double rho1 = 1.0 / (2.0 * sigma - rho);
      const double c1 = rho1 * rho, c2 = 2.0 * rho1 / delta;
      dispatch_L(tk.lanes, [&](auto LC) {
        constexpr int LL = decltype(LC)::value;
        hipLaunchKernelGGL((k_cheb_step<LL>), dim3(sh.grid), dim3(sh.block), 0, s, n, m->d_rp_f, m->d_col_f,
                           (const double *)m->d_Mbc, (const double *)m->d_dinvM, reinterpret_cast<double2 *>(x), r,
                           (const double2 *)d[j & 1], d[(j + 1) & 1], c1, c2);
      });
      rho = rho1;
    }
    used += k;
    check(false);
    CGP_HIP(hipGetLastError());
    cgp_status ps = poll(m, SLOT_MASS);
    if (ps) return ps;
    const KrylovState &h = m->h_state[SLOT_MASS];
    if (h.status || host_all_done(h) || used >= maxit) break;
    double need = 1.0;
    for (int c = 0; c < 2; c++)
      if (!h.done[c]) need = std::max(need, h.rnorm[c] / (tol * h.bnorm[c]));
    k = std::max(1, std::min(maxit - used, (int)std::ceil(std::log(2.0 * need) / std::log(3.0)) + 2));
  }
  *out = m->h_state[SLOT_MASS];
  out->iters = used;
  *hint = std::max(1, used);
  hipLaunchKernelGGL((k_zero_b_fix<2>), dim3(blocks_1d(n)), dim3(256), 0, s, n, x, (const KrylovState *)st);
  return status_of(*out, SLOT_MASS);
}

cgp_status drv_correct(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *ut, const double *pf,
                       double *u, cgp_stats *stats) {
  hipStream_t s = m->stream;
  const int n = m->pf.n;
  if (m->params.mass_mode == CGP_MASS_LUMPED) {
    launch_correct_lumped(m, g, ut, pf, u);
    CGP_HIP(hipGetLastError());
    if (stats) {
      stats->mass_iters = 0;
      stats->mass_relres = 0.0;
    }
    return CGP_OK;
  }
  double *rhs = m->d_wf[0];
  launch_correct_rhs(m, g, ut, pf, rhs);
  // CGP_X0_EXTRAP inside cgp_step: the lumped correction plus the last step's consistent-minus-lumped
  // difference, which changes slowly from step to step
  const bool extrap = (o->x0_mode == CGP_X0_EXTRAP && ut == m->d_ut);
  double *ul = m->d_wf[6];  // the lumped correction (free here: the momentum solve is done)
  const long cnt = 2L * n;
  if (extrap && !m->d_mdelta) {
    void *q = nullptr;
    CGP_HIP(hipMalloc(&q, sizeof(double) * cnt));
    m->allocations.push_back(q);
    m->d_mdelta = (double *)q;
    m->mdelta_ok = false;
  }
  if (!extrap) m->mdelta_ok = false;
  if (o->x0_mode == CGP_X0_ZERO) {
    CGP_HIP(hipMemsetAsync(u, 0, 2 * n * sizeof(double), s));
    launch_set_dirichlet(m, g, u);
  } else if (extrap && m->mdelta_ok) {
    launch_correct_lumped(m, g, ut, pf, ul);
    hipLaunchKernelGGL(k_axpy_into, dim3((cnt + 255) / 256), dim3(256), 0, s, cnt, (const double *)ul, 1.0,
                       (const double *)m->d_mdelta, u);
    launch_set_dirichlet(m, g, u);
  } else {
    // start from the lumped-mass correction (g on the Dirichlet rows): the consistent solve then
    // only removes the difference between the two mass matrices
    launch_correct_lumped(m, g, ut, pf, extrap ? ul : u);
    if (extrap) CGP_HIP(hipMemcpyAsync(u, ul, sizeof(double) * cnt, hipMemcpyDeviceToDevice, s));
  }
  double *w[5] = {m->d_wf[1], m->d_wf[2], m->d_wf[3], m->d_wf[4], m->d_wf[5]};
  KrylovState fin{};
  cgp_status rs = o->method == CGP_METHOD_CHEBYSHEV
                       ? cheb_mass(m, n, rhs, u, w, m->tune.fine, o->tol, o->max_iter, &m->cheb_steps, &fin)
                       : run_pcg64<2>(m, SLOT_MASS, n, m->d_rp_f, m->d_col_f, m->d_Mbc, m->d_dinvM, rhs, u, w,
                                      m->tune.fine, o->tol, o->max_iter, &m->mass_chunk, false, &fin);
  launch_set_dirichlet(m, g, u);
  if (extrap) {
    hipLaunchKernelGGL(k_axpy_into, dim3((cnt + 255) / 256), dim3(256), 0, s, cnt, (const double *)u, -1.0,
                       (const double *)ul, m->d_mdelta);
    m->mdelta_ok = (rs == CGP_OK);
  }
  CGP_HIP(hipGetLastError());
  if (stats) {
    stats->mass_iters = fin.iters;
    stats->mass_relres = 0.0;
    for (int c = 0; c < 2; c++)
      stats->mass_relres = std::max(stats->mass_relres, fin.bnorm[c] > 0 ? fin.rnorm[c] / fin.bnorm[c] : 0.0);
  }
  return rs;
}

}  // namespace cgp
