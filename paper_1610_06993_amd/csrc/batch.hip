// Many independent CGP simulations on one GPU: the coarse pressure Poisson
// solves (Eq. 21) of all instances run as one Jacobi-PCG whose every
// iteration is one kernel launch over all instances' rows.
//
// The instances' coarse systems are concatenated (block-diagonal CSR with
// global int32 indices).  Rows are cut into tiles that never straddle two
// instances; a block works on one tile and writes one partial per tile, and
// each instance sums its own tiles' partials in a fixed order, so every
// instance keeps its own Krylov scalars and convergence flag (a converged
// instance's tiles return at once).  The iteration is the single-kernel
// Chronopoulos-Gear form of the single-mesh solver, with the same node records
// {r, w, s, D^-1} (a gathered column is one 32-byte load).  At the batch's
// size the iteration streams from HBM, and each instance's partials are summed
// per block: a per-wave sum, as in the single-mesh kernel, would read them 16
// times over.  Chunks of iterations are
// captured once into HIP graphs and replayed, with one poll of the instance
// states per chunk.  Launch shapes (lanes per row, block, rows per lane group)
// come from cgp_batch_set_tuning or from the autotuner, which times each
// candidate on the batch's own system and caches the choice in a JSON file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "devutil.h"
#include "kernels.h"
#include "learn.h"

constexpr int kBatchLanes = 4;  // host threads / streams for the per-instance phases of a batch step

struct cgp_batch {
  std::vector<cgp_mesh *> meshes;
  hipStream_t mstream = nullptr;     // the meshes' stream
  hipStream_t stream = nullptr;      // the batch's own stream (graphs are captured on it)
  // per-instance phases of cgp_batch_step run on these streams from as many host threads, so that the
  // small instances' latency-bound solves overlap (default priority, like every stream here)
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> aux_ev;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  int ninst = 0;
  long rows = 0, nnz = 0;
  std::vector<long> row_off, nnz_off;
  // concatenated coarse operators
  int *d_rp = nullptr, *d_col = nullptr;
  double *d_A = nullptr, *d_dinv = nullptr;
  // work vectors over all rows
  double *d_x = nullptr, *d_b = nullptr, *d_p = nullptr;
  // FP32 refinement: operator and D^-1 in FP32, FP64 residual, FP32 inner iterate and direction
  float *d_A32 = nullptr, *d_dinv32 = nullptr, *d_d32 = nullptr, *d_p32 = nullptr;
  double *d_r64 = nullptr;
  double4 *d_rec[2] = {};             // records {r, w, s, D^-1}, double-buffered
  // tiles
  cgp_batch_tuning tune{4, 512, 1, 1, 16, 0};
  int ntiles = 0;
  int4 *d_tiles = nullptr;            // {instance, first row, end row, -}
  int4 *d_tinfo = nullptr;            // per tile: {first tile, tile count} of its instance
  int *d_t0 = nullptr, *d_nt = nullptr;
  double *d_part = nullptr;           // 4 regions of [3][ntiles]
  cgp::KrylovState *d_state = nullptr, *h_state = nullptr;
  // graphs of one chunk starting at iteration 0 and at iteration `chunk`
  hipGraphExec_t gx[2] = {nullptr, nullptr};
  std::vector<void *> allocations;
};

namespace cgp {
namespace bdev {
using namespace dev;

// store this block's K sums as P[k * G + t]
template <int K>
__device__ __forceinline__ void put_at(const double (&v)[K], double *__restrict__ P, int G, int t) {
  double tot[K];
  block_sum<K>(v, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; k++) P[(long)k * G + t] = tot[k];
  }
}

// fixed-order totals of K partial arrays over one instance's tiles [t0, t0 + nt)
template <int K>
__device__ __forceinline__ void inst_sum(const double *__restrict__ P, int G, int t0, int nt, double (&tot)[K]) {
  double v[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nt; b += blockDim.x) s += P[(long)k * G + t0 + b];
    v[k] = s;
  }
  block_sum<K>(v, tot);
}

// put_at with a single barrier: must be the block's last reduction
template <int K>
__device__ __forceinline__ void put_at_last(const double (&v)[K], double *__restrict__ P, int G, int t) {
  __shared__ double sh[K][kMaxBlock / 64];
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
    P[(long)threadIdx.x * G + t] = s;
  }
}

__global__ void k_bt_state_init(int ninst, double tol, int maxit, KrylovState *st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ninst) return;
  KrylovState s{};
  s.tol = tol;
  s.maxit = maxit;
  s.ncomp = 1;
  st[i] = s;
}

// r0 = b - A x, p = s = 0: records {r0, -, 0, D^-1} in slot 0, {-, -, -, D^-1} in slot 1; partial
// b.b per tile
template <int L>
__global__ void __launch_bounds__(kMaxBlock) k_bt_init_r(int G, const int4 *__restrict__ tiles,
                                                        const int *__restrict__ rp, const int *__restrict__ col,
                                                        const double *__restrict__ A, const double *__restrict__ dinv,
                                                        const double *__restrict__ b, const double *__restrict__ x,
                                                        double *__restrict__ p, double4 *__restrict__ R0,
                                                        double4 *__restrict__ R1, double *__restrict__ Pout) {
  const int t = xcd_block();
  const int4 T = tiles[t];
  const int lane = threadIdx.x & (L - 1), groups = blockDim.x / L;
  double acc[1] = {0.0};
  for (int row = T.y + (int)threadIdx.x / L; row < T.z; row += groups) {
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
  put_at<1>(acc, Pout, G, t);
}

// w0 = A D^-1 r0 into the records' w field (fields r and D^-1 gathered); partials (gamma, delta,
// r.r); publishes ||b|| per instance.  T = double (the FP64 solve) or float (an FP32 inner solve).
template <typename T, int L>
__global__ void __launch_bounds__(kMaxBlock) k_bt_init_w(int G, const int4 *__restrict__ tiles,
                                                        const int *__restrict__ t0s, const int *__restrict__ nts,
                                                        const int *__restrict__ rp, const int *__restrict__ col,
                                                        const T *__restrict__ A, rec_t<T> *__restrict__ R0,
                                                        const double *__restrict__ Pin, double *__restrict__ Pout,
                                                        KrylovState *__restrict__ st) {
  const int t = xcd_block();
  const int4 Tl = tiles[t];
  KrylovState *S = st + Tl.x;
  if (S->status || S->done[0]) return;
  const int t0 = t0s[Tl.x];
  double tb[1];
  inst_sum<1>(Pin, G, t0, nts[Tl.x], tb);
  if (t == t0 && threadIdx.x == 0) {
    S->bnorm[0] = sqrt(tb[0]);
    S->zero_b[0] = (tb[0] == 0.0);
    if (!is_finite(tb[0])) S->status = CGP_E_NONFINITE;
  }
  const int lane = threadIdx.x & (L - 1), groups = blockDim.x / L;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int row = Tl.y + (int)threadIdx.x / L; row < Tl.z; row += groups) {
    double sum = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const int j = col[k];
      sum += (double)(A[k] * (R0[j].w * R0[j].x));
    }
    sum = group_sum<L>(sum);
    if (lane == 0) {
      const T w = (T)sum, r0 = R0[row].x;
      const double r = (double)r0, u = (double)(R0[row].w * r0);
      R0[row].y = w;
      acc[0] += r * u;
      acc[1] += (double)w * u;
      acc[2] += r * r;
    }
  }
  put_at<3>(acc, Pout, G, t);
}

// One PCG iteration of every unconverged instance (recurrences as in the single-mesh kernel).
// The first tile's block of each instance publishes its scalars and counts its updates.
template <typename T, int L>
__global__ void __launch_bounds__(kMaxBlock)
    k_bt_iter(int it, int G, const int4 *__restrict__ tiles, const int4 *__restrict__ tinfo,
              const int *__restrict__ rp, const int *__restrict__ col, const T *__restrict__ A,
              T *__restrict__ x, T *__restrict__ p, const rec_t<T> *__restrict__ Rc,
              rec_t<T> *__restrict__ Rn, const double *__restrict__ Pin, double *__restrict__ Pout,
              KrylovState *__restrict__ st) {
  using R4 = rec_t<T>;
  const int t = xcd_block();
  const int4 Tl = tiles[t], I = tinfo[t];
  KrylovState *S = st + Tl.x;
  if (S->status || S->done[0]) return;
  double t3[3];
  inst_sum<3>(Pin, G, I.x, I.y, t3);
  const double gam = t3[0], del = t3[1], rr = t3[2];
  const double bb = S->bnorm[0] * S->bnorm[0];
  const bool done = bb == 0.0 || sqrt(rr) <= S->tol * sqrt(bb);
  double beta = 0.0, alpha = 0.0;
  if (it == 0) {
    alpha = gam / del;
  } else {
    beta = gam / S->rz[(it - 1) & 1][0];
    alpha = gam / (del - beta * gam / S->alpha[(it - 1) & 1][0]);
  }
  const bool bad = !is_finite(rr) || (!done && (!is_finite(alpha) || !is_finite(beta)));
  if (t == I.x && threadIdx.x == 0) {
    S->rz[it & 1][0] = gam;
    S->alpha[it & 1][0] = alpha;
    S->rnorm[0] = sqrt(rr);
    if (done) S->done[0] = 1;
    if (bad) S->status = CGP_E_NONFINITE;
    if (!done && !bad) S->iters += 1;
  }
  if (done || bad) return;
  const T al = (T)alpha, bt = (T)beta;
  const int lane = threadIdx.x & (L - 1), groups = blockDim.x / L;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int row = Tl.y + (int)threadIdx.x / L; row < Tl.z; row += groups) {
    double sum = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) {
      const R4 g = Rc[col[k]];
      sum += (double)(A[k] * (g.w * (g.x - al * (g.y + bt * g.z))));
    }
    sum = group_sum<L>(sum);
    if (lane == 0) {
      const R4 o = Rc[row];
      const T d = o.w, rc = o.x, wc = o.y, sc = o.z;
      const T si = wc + bt * sc;
      const T pi = d * rc + bt * p[row];
      const T rn = rc - al * si;
      const T un = d * (rc - al * (wc + bt * sc));
      const T wn = (T)sum;
      x[row] = x[row] + al * pi;
      p[row] = pi;
      store_rws(&Rn[row], rn, wn, si);
      acc[0] += (double)rn * (double)un;
      acc[1] += (double)wn * (double)un;
      acc[2] += (double)rn * (double)rn;
    }
  }
  put_at_last<3>(acc, Pout, G, t);
}

// The same iteration with every load of the tile issued before the instance's scalars are known
// (cgp_batch_tuning.ahead = 1).  The gathered column's next u_j = D^-1_j (r_j - alpha (w_j + beta s_j))
// is linear in (1, alpha, alpha beta), so a row's SpMV splits into three sums that need no scalars,
//   sum_k A_jk u_j = S_r - alpha S_w - alpha beta S_s,  S_f = sum_k A_jk D^-1_j f_j,
// which each lane accumulates as its gathered records arrive, while the instance's partials of the
// previous iteration are still being summed.  A tile is P passes of blockDim/L rows: every lane group
// streams P rows one after the other (only three accumulators per row stay live), and lane q of the
// group holds row q's own record, x and p for the update.  The sums are combined in FP64; the result
// differs from the single-mesh kernel's only in rounding.
template <int L> constexpr int bt_ahead() { return (10 + L - 1) / L; }  // entries per lane issued together

template <typename T, int L, int P, bool JOINT>
__global__ void __launch_bounds__(kMaxBlock)
    k_bt_iter_ahead(int it, int G, const int4 *__restrict__ tiles, const int4 *__restrict__ tinfo,
                    const int *__restrict__ rp, const int *__restrict__ col, const T *__restrict__ A,
                    T *__restrict__ x, T *__restrict__ p, const rec_t<T> *__restrict__ Rc,
                    rec_t<T> *__restrict__ Rn, const double *__restrict__ Pin, double *__restrict__ Pout,
                    KrylovState *__restrict__ st) {
  static_assert(P <= L, "one row update per lane of a group");
  using R4 = rec_t<T>;
  constexpr int E = bt_ahead<L>();
  const int t = xcd_block();
  const int4 Tl = tiles[t], I = tinfo[t];
  KrylovState *S = st + Tl.x;
  if (S->status || S->done[0]) return;
  const int lane = threadIdx.x & (L - 1), rpb = blockDim.x / L, gid = threadIdx.x / L;
  const int my_row = Tl.y + lane * rpb + gid;  // the row this lane updates (lane < P)
  const bool mine = lane < P && my_row < Tl.z;
  R4 own{};
  T xo = T(0), po = T(0);
  if (mine) {
    own = Rc[my_row];
    xo = x[my_row];
    po = p[my_row];
  }
  int k0[P], k1[P];
#pragma unroll
  for (int q = 0; q < P; q++) {
    const int row = Tl.y + q * rpb + gid;
    k0[q] = row < Tl.z ? rp[row] : 0;
    k1[q] = row < Tl.z ? rp[row + 1] : 0;
  }
  double sr[P], sw[P], ss[P];
  // JOINT: the columns and values of all P rows are loaded before the first gather (more loads in
  // flight, more registers); otherwise row by row
  int jj[JOINT ? P : 1][E];
  T aa[JOINT ? P : 1][E];
  auto load_cols = [&](int q, int slot) {
#pragma unroll
    for (int e = 0; e < E; e++) {
      const int k = k0[q] + lane + e * L;
      jj[slot][e] = k < k1[q] ? col[k] : -1;
      aa[slot][e] = k < k1[q] ? A[k] : T(0);
    }
  };
  if (JOINT) {
#pragma unroll
    for (int q = 0; q < P; q++) load_cols(q, q);
  }
#pragma unroll
  for (int q = 0; q < P; q++) {
    // the row's first E entries per lane: columns and values, then the gathered records, together
    const int slot = JOINT ? q : 0;
    if (!JOINT) load_cols(q, 0);
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int e = 0; e < E; e++)
      if (jj[slot][e] >= 0) {
        const R4 g = Rc[jj[slot][e]];
        const T ad = aa[slot][e] * g.w;
        a += (double)(ad * g.x);
        b += (double)(ad * g.y);
        c += (double)(ad * g.z);
      }
    for (int k = k0[q] + lane + E * L; k < k1[q]; k += L) {  // longer rows
      const R4 g = Rc[col[k]];
      const T ad = A[k] * g.w;
      a += (double)(ad * g.x);
      b += (double)(ad * g.y);
      c += (double)(ad * g.z);
    }
    sr[q] = a;
    sw[q] = b;
    ss[q] = c;
  }
  double t3[3];
  inst_sum<3>(Pin, G, I.x, I.y, t3);
  const double gam = t3[0], del = t3[1], rr = t3[2];
  const double bb = S->bnorm[0] * S->bnorm[0];
  const bool done = bb == 0.0 || sqrt(rr) <= S->tol * sqrt(bb);
  double beta = 0.0, alpha = 0.0;
  if (it == 0) {
    alpha = gam / del;
  } else {
    beta = gam / S->rz[(it - 1) & 1][0];
    alpha = gam / (del - beta * gam / S->alpha[(it - 1) & 1][0]);
  }
  const bool bad = !is_finite(rr) || (!done && (!is_finite(alpha) || !is_finite(beta)));
  if (t == I.x && threadIdx.x == 0) {
    S->rz[it & 1][0] = gam;
    S->alpha[it & 1][0] = alpha;
    S->rnorm[0] = sqrt(rr);
    if (done) S->done[0] = 1;
    if (bad) S->status = CGP_E_NONFINITE;
    if (!done && !bad) S->iters += 1;
  }
  if (done || bad) return;
  const T al = (T)alpha, bt = (T)beta;
  const double ab = (double)al * (double)bt;
  double my_sum = 0.0;
#pragma unroll
  for (int q = 0; q < P; q++) {
    const double sum = group_sum<L>(sr[q] - (double)al * sw[q] - ab * ss[q]);
    if (lane == q) my_sum = sum;
  }
  double acc[3] = {0.0, 0.0, 0.0};
  if (mine) {
    const T d = own.w, rc = own.x, wc = own.y, sc = own.z;
    const T si = wc + bt * sc;
    const T pi = d * rc + bt * po;
    const T rn = rc - al * si;
    const T un = d * (rc - al * (wc + bt * sc));
    const T wn = (T)my_sum;
    x[my_row] = xo + al * pi;
    p[my_row] = pi;
    store_rws(&Rn[my_row], rn, wn, si);
    acc[0] = (double)rn * (double)un;
    acc[1] = (double)wn * (double)un;
    acc[2] = (double)rn * (double)rn;
  }
  put_at_last<3>(acc, Pout, G, t);
}

// ---- FP32 inner solves inside FP64 iterative refinement, per instance (as the single-mesh solve)
// r64 = b - A x in FP64; partials (r.r, b.b) per tile
template <int L>
__global__ void __launch_bounds__(kMaxBlock) k_bt_ir_residual(int G, const int4 *__restrict__ tiles,
                                                             const int *__restrict__ rp, const int *__restrict__ col,
                                                             const double *__restrict__ A,
                                                             const double *__restrict__ b, const double *__restrict__ x,
                                                             double *__restrict__ r64, double *__restrict__ Pout) {
  const int t = xcd_block();
  const int4 Tl = tiles[t];
  const int lane = threadIdx.x & (L - 1), groups = blockDim.x / L;
  double acc[2] = {0.0, 0.0};
  for (int row = Tl.y + (int)threadIdx.x / L; row < Tl.z; row += groups) {
    double sum = 0.0;
    for (int k = rp[row] + lane; k < rp[row + 1]; k += L) sum += A[k] * x[col[k]];
    sum = group_sum<L>(sum);
    if (lane == 0) {
      const double bb = b[row], rr = bb - sum;
      r64[row] = rr;
      acc[0] += rr * rr;
      acc[1] += bb * bb;
    }
  }
  put_at<2>(acc, Pout, G, t);
}

// Outer convergence test of each instance and the start of its inner solve K32 d = r64/||r64||:
// records {r0, -, 0, D^-1} (FP32) in slot 0 and D^-1 in slot 1, d = p = 0; partial r0.r0 per tile.
// The instance's first tile publishes the outer state and resets the inner one, whose tolerance is
// the reduction still needed (at least inner_tol).
__global__ void __launch_bounds__(kMaxBlock) k_bt_ir_init(int G, const int4 *__restrict__ tiles,
                                                         const int4 *__restrict__ tinfo, double inner_tol,
                                                         const double *__restrict__ r64,
                                                         const float *__restrict__ dinv, float4 *__restrict__ R0,
                                                         float4 *__restrict__ R1, float *__restrict__ d,
                                                         float *__restrict__ p, const double *__restrict__ Pin,
                                                         double *__restrict__ Pout, KrylovState *__restrict__ so,
                                                         KrylovState *__restrict__ si) {
  const int t = xcd_block();
  const int4 Tl = tiles[t], I = tinfo[t];
  KrylovState *O = so + Tl.x, *S = si + Tl.x;
  double t2[2];
  inst_sum<2>(Pin, G, I.x, I.y, t2);
  const double rn = sqrt(t2[0]), bn = sqrt(t2[1]);
  const bool bad = !is_finite(rn) || !is_finite(bn) || O->status;
  const bool done = bn == 0.0 || rn <= O->tol * bn;
  if (t == I.x && threadIdx.x == 0) {
    O->rnorm[0] = rn;
    O->bnorm[0] = bn;
    O->zero_b[0] = (bn == 0.0);
    O->done[0] = done;
    if (bad && !O->status) O->status = CGP_E_NONFINITE;
    S->done[0] = done || bad;
    S->status = 0;
    S->iters = 0;
    const double need = 0.5 * O->tol * bn / rn;
    S->tol = need > inner_tol ? need : inner_tol;
  }
  if (done || bad) return;
  const double inv = 1.0 / rn;
  const int groups = blockDim.x;
  double acc[1] = {0.0};
  for (int row = Tl.y + (int)threadIdx.x; row < Tl.z; row += groups) {
    const float rr = (float)(r64[row] * inv), di = dinv[row];
    R0[row] = make_float4(rr, 0.0f, 0.0f, di);
    R1[row] = make_float4(0.0f, 0.0f, 0.0f, di);
    d[row] = 0.0f;
    p[row] = 0.0f;
    acc[0] += (double)rr * (double)rr;
  }
  put_at<1>(acc, Pout, G, t);
}

// x += ||r64|| d for every instance whose outer solve goes on and whose inner solve ended cleanly
__global__ void k_bt_ir_update(const int4 *__restrict__ tiles, const KrylovState *__restrict__ so,
                               const KrylovState *__restrict__ si, double *__restrict__ x,
                               const float *__restrict__ d) {
  const int4 Tl = tiles[blockIdx.x];
  const KrylovState *O = so + Tl.x, *S = si + Tl.x;
  if (O->done[0] || O->status || S->status) return;
  const double s = O->rnorm[0];
  for (int row = Tl.y + (int)threadIdx.x; row < Tl.z; row += blockDim.x) x[row] += s * (double)d[row];
}

// after a chunk (one block per instance): convergence from the last iteration's partials
__global__ void __launch_bounds__(256) k_bt_finish(int G, const int *__restrict__ t0s, const int *__restrict__ nts,
                                                   const double *__restrict__ Pin, KrylovState *__restrict__ st) {
  KrylovState *S = st + blockIdx.x;
  if (S->status || S->done[0]) return;
  double t3[3];
  inst_sum<3>(Pin, G, t0s[blockIdx.x], nts[blockIdx.x], t3);
  if (threadIdx.x != 0) return;
  const double rn = sqrt(t3[2]);
  S->rnorm[0] = rn;
  if (!is_finite(rn)) S->status = CGP_E_NONFINITE;
  else if (rn <= S->tol * S->bnorm[0]) S->done[0] = 1;
}

// instances with a zero right-hand side get x = 0
__global__ void k_bt_zero_b(const int4 *__restrict__ tiles, const KrylovState *__restrict__ st,
                            double *__restrict__ x) {
  const int4 T = tiles[blockIdx.x];
  if (!st[T.x].zero_b[0]) return;
  for (int row = T.y + (int)threadIdx.x; row < T.z; row += blockDim.x) x[row] = 0.0;
}

// synthetic right-hand side for the autotuner: a hash of the row index in [-1, 1)
__global__ void k_bt_fill(long n, double *__restrict__ b, double *__restrict__ x) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = (unsigned long long)i * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  b[i] = double(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  x[i] = 0.0;
}

}  // namespace bdev

namespace {
using namespace bdev;

template <typename T>
cgp_status balloc(cgp_batch *B, T **p, size_t count) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? CGP_E_OOM : CGP_E_DEVICE;
  }
  B->allocations.push_back(q);
  *p = static_cast<T *>(q);
  return CGP_OK;
}

#define BTRY(x)                  \
  do {                           \
    cgp_status s_ = (x);         \
    if (s_ != CGP_OK) return s_; \
  } while (0)

enum { B_INIT = 0, B_A = 1, B_B = 2, B_C = 3 };
double *bregion(cgp_batch *B, int k) { return B->d_part + (size_t)k * 3 * B->ntiles; }
double *bpin(cgp_batch *B, int it) { return it == 0 ? bregion(B, B_A) : bregion(B, ((it - 1) & 1) ? B_C : B_B); }
double *bpout(cgp_batch *B, int it) { return bregion(B, (it & 1) ? B_C : B_B); }

void drop_graphs(cgp_batch *B) {
  for (auto &g : B->gx)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// tiles of `per` rows that never straddle instances; (re)allocates tile-sized buffers
cgp_status build_tiles(cgp_batch *B) {
  const cgp_batch_tuning &t = B->tune;
  const int per = t.block * t.passes / t.lanes;
  std::vector<int4> tiles;
  std::vector<int> t0(B->ninst), nt(B->ninst);
  for (int i = 0; i < B->ninst; i++) {
    t0[i] = (int)tiles.size();
    for (long r = B->row_off[i]; r < B->row_off[i + 1]; r += per)
      tiles.push_back(make_int4(i, (int)r, (int)std::min<long>(r + per, B->row_off[i + 1]), 0));
    nt[i] = (int)tiles.size() - t0[i];
  }
  // pad to a multiple of 8 with empty tiles of the last instance (rows [end, end)), so that the XCD
  // remapping applies; they contribute zero partials
  const int last = B->ninst - 1;
  while (tiles.size() % 8) {
    const int e = (int)B->row_off[B->ninst];
    tiles.push_back(make_int4(last, e, e, 0));
    nt[last]++;
  }
  std::vector<int4> tinfo(tiles.size());
  for (size_t k = 0; k < tiles.size(); k++) tinfo[k] = make_int4(t0[tiles[k].x], nt[tiles[k].x], 0, 0);
  if ((int)tiles.size() > B->ntiles) {
    BTRY(balloc(B, &B->d_tiles, tiles.size()));
    BTRY(balloc(B, &B->d_tinfo, tiles.size()));
    BTRY(balloc(B, &B->d_part, 4 * 3 * tiles.size()));
  }
  B->ntiles = (int)tiles.size();
  CGP_HIP(hipMemcpyAsync(B->d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, B->stream));
  CGP_HIP(hipMemcpyAsync(B->d_tinfo, tinfo.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice, B->stream));
  CGP_HIP(hipMemcpyAsync(B->d_t0, t0.data(), sizeof(int) * B->ninst, hipMemcpyHostToDevice, B->stream));
  CGP_HIP(hipMemcpyAsync(B->d_nt, nt.data(), sizeof(int) * B->ninst, hipMemcpyHostToDevice, B->stream));
  CGP_HIP(hipStreamSynchronize(B->stream));
  drop_graphs(B);
  return CGP_OK;
}

// the loads-ahead kernel's instantiations: lanes 4 or 8 per row, passes 1, 2 or 4 rows per lane group
// (8 with 8 lanes),
// columns row by row or of all rows first
template <typename F>
void dispatch_ahead(int L, int P, bool joint, F &&f) {
  auto with_LP = [&](auto LC, auto PC) {
    if (joint) f(LC, PC, std::true_type{});
    else f(LC, PC, std::false_type{});
  };
  auto with_L = [&](auto LC) {
    switch (P) {
      case 1: with_LP(LC, std::integral_constant<int, 1>{}); break;
      case 2: with_LP(LC, std::integral_constant<int, 2>{}); break;
      default: with_LP(LC, std::integral_constant<int, 4>{}); break;
    }
  };
  if (L == 8 && P == 8) with_LP(std::integral_constant<int, 8>{}, std::integral_constant<int, 8>{});
  else if (L == 8) with_L(std::integral_constant<int, 8>{});
  else with_L(std::integral_constant<int, 4>{});
}

// enqueue `count` iterations starting at `it0`, then the chunk's convergence check: the FP64 solve
// (fp32 = false) or the FP32 inner solves of the refinement (states si = d_state + ninst)
void enqueue_chunk(cgp_batch *B, int it0, int count, bool fp32 = false) {
  const int G = B->ntiles, blk = B->tune.block;
  hipStream_t s = B->stream;
  KrylovState *st = fp32 ? B->d_state + B->ninst : B->d_state;
  float4 *R32[2] = {reinterpret_cast<float4 *>(B->d_rec[0]), reinterpret_cast<float4 *>(B->d_rec[0]) + B->rows};
  if (B->tune.ahead) {
    dispatch_ahead(B->tune.lanes, B->tune.passes, B->tune.ahead == 2, [&](auto LC, auto PC, auto JC) {
      constexpr int LL = decltype(LC)::value, PP = decltype(PC)::value;
      constexpr bool JJ = decltype(JC)::value;
      for (int it = it0; it < it0 + count; it++) {
        const int cur = it & 1, nxt = cur ^ 1;
        if (fp32)
          hipLaunchKernelGGL((k_bt_iter_ahead<float, LL, PP, JJ>), dim3(G), dim3(blk), 0, s, it, G,
                             (const int4 *)B->d_tiles, (const int4 *)B->d_tinfo, (const int *)B->d_rp,
                             (const int *)B->d_col, (const float *)B->d_A32, B->d_d32, B->d_p32,
                             (const float4 *)R32[cur], R32[nxt], (const double *)bpin(B, it), bpout(B, it), st);
        else
          hipLaunchKernelGGL((k_bt_iter_ahead<double, LL, PP, JJ>), dim3(G), dim3(blk), 0, s, it, G,
                             (const int4 *)B->d_tiles, (const int4 *)B->d_tinfo, (const int *)B->d_rp,
                             (const int *)B->d_col, (const double *)B->d_A, B->d_x, B->d_p,
                             (const double4 *)B->d_rec[cur], B->d_rec[nxt], (const double *)bpin(B, it),
                             bpout(B, it), st);
      }
    });
  } else
  dispatch_L(B->tune.lanes, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    for (int it = it0; it < it0 + count; it++) {
      const int cur = it & 1, nxt = cur ^ 1;
      if (fp32)
        hipLaunchKernelGGL((k_bt_iter<float, LL>), dim3(G), dim3(blk), 0, s, it, G, (const int4 *)B->d_tiles,
                           (const int4 *)B->d_tinfo, (const int *)B->d_rp, (const int *)B->d_col,
                           (const float *)B->d_A32, B->d_d32, B->d_p32, (const float4 *)R32[cur], R32[nxt],
                           (const double *)bpin(B, it), bpout(B, it), st);
      else
        hipLaunchKernelGGL((k_bt_iter<double, LL>), dim3(G), dim3(blk), 0, s, it, G, (const int4 *)B->d_tiles,
                           (const int4 *)B->d_tinfo, (const int *)B->d_rp, (const int *)B->d_col,
                           (const double *)B->d_A, B->d_x, B->d_p, (const double4 *)B->d_rec[cur], B->d_rec[nxt],
                           (const double *)bpin(B, it), bpout(B, it), st);
    }
  });
  hipLaunchKernelGGL(k_bt_finish, dim3(B->ninst), dim3(256), 0, s, G, (const int *)B->d_t0, (const int *)B->d_nt,
                     (const double *)bpin(B, it0 + count), st);
}

cgp_status run_chunk(cgp_batch *B, int which) {
  const int K = B->tune.chunk;
  const int it0 = which == 0 ? 0 : K;
  if (!B->tune.use_graph) {
    enqueue_chunk(B, it0, K);
    CGP_HIP(hipGetLastError());
    return CGP_OK;
  }
  if (!B->gx[which]) {
    hipGraph_t g = nullptr;
    CGP_HIP(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
    enqueue_chunk(B, it0, K);
    CGP_HIP(hipStreamEndCapture(B->stream, &g));
    hipError_t e = hipGraphInstantiate(&B->gx[which], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      B->gx[which] = nullptr;
      set_error(std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
      return CGP_E_DEVICE;
    }
  }
  CGP_HIP(hipGraphLaunch(B->gx[which], B->stream));
  return CGP_OK;
}

// copy both state arrays (the FP64 or outer states, then the inner ones) to the host; report on the
// array that starts at `first` (0 or ninst)
cgp_status poll_states(cgp_batch *B, bool *all_done, int *bad, int first = 0) {
  CGP_HIP(hipMemcpyAsync(B->h_state, B->d_state, sizeof(KrylovState) * 2 * B->ninst, hipMemcpyDeviceToHost,
                         B->stream));
  CGP_HIP(hipStreamSynchronize(B->stream));
  *all_done = true;
  *bad = -1;
  for (int i = 0; i < B->ninst; i++) {
    const KrylovState &h = B->h_state[first + i];
    if (h.status && *bad < 0) *bad = i;
    if (!h.done[0]) *all_done = false;
  }
  return CGP_OK;
}

// the PCG on the concatenated system, from b, x already in place; returns iterations launched
cgp_status solve(cgp_batch *B, double tol, int maxit, int *launched) {
  hipStream_t s = B->stream;
  const int G = B->ntiles, blk = B->tune.block;
  hipLaunchKernelGGL(k_bt_state_init, dim3((B->ninst + 255) / 256), dim3(256), 0, s, B->ninst, tol, maxit,
                     B->d_state);
  dispatch_L(B->tune.lanes, [&](auto LC) {
    constexpr int LL = decltype(LC)::value;
    hipLaunchKernelGGL((k_bt_init_r<LL>), dim3(G), dim3(blk), 0, s, G, (const int4 *)B->d_tiles,
                       (const int *)B->d_rp, (const int *)B->d_col, (const double *)B->d_A,
                       (const double *)B->d_dinv, (const double *)B->d_b, (const double *)B->d_x, B->d_p,
                       B->d_rec[0], B->d_rec[1], bregion(B, B_INIT));
    hipLaunchKernelGGL((k_bt_init_w<double, LL>), dim3(G), dim3(blk), 0, s, G, (const int4 *)B->d_tiles,
                       (const int *)B->d_t0, (const int *)B->d_nt, (const int *)B->d_rp, (const int *)B->d_col,
                       (const double *)B->d_A, B->d_rec[0], (const double *)bregion(B, B_INIT), bregion(B, B_A),
                       B->d_state);
  });
  CGP_HIP(hipGetLastError());
  const int K = B->tune.chunk;
  int n = 0;
  bool all = false;
  int bad = -1;
  for (int c = 0; n < maxit; c++) {
    BTRY(run_chunk(B, c == 0 ? 0 : 1));
    n += K;
    BTRY(poll_states(B, &all, &bad));
    if (all || bad >= 0) break;
  }
  hipLaunchKernelGGL(k_bt_zero_b, dim3(G), dim3(256), 0, s, (const int4 *)B->d_tiles,
                     (const KrylovState *)B->d_state, B->d_x);
  CGP_HIP(hipGetLastError());
  *launched = n;
  if (bad >= 0) {
    set_error("batched Poisson PCG: instance " + std::to_string(bad) + " produced a non-finite residual");
    return CGP_E_NONFINITE;
  }
  if (!all) {
    set_error("batched Poisson PCG: iteration limit reached before every instance converged");
    return CGP_E_NOCONV;
  }
  return CGP_OK;
}

// FP32 Jacobi-PCG inside FP64 iterative refinement for every instance at once (as the single-mesh
// refinement): per refinement step one FP64 residual launch, one init launch, then the FP32 inner
// iterations of all instances whose outer solve goes on, and one update launch.  iters[i]: inner
// iterations of instance i; outers[i]: residual checks it took.
cgp_status solve_ir(cgp_batch *B, const cgp_solver_opts *o, int *launched, std::vector<int> &iters,
                    std::vector<int> &outers) {
  hipStream_t s = B->stream;
  const int G = B->ntiles, blk = B->tune.block, n = B->ninst, K = B->tune.chunk;
  const double inner_tol = o->inner_tol > 0 ? o->inner_tol : 1e-4;
  KrylovState *so = B->d_state, *si = B->d_state + n;
  float4 *R32[2] = {reinterpret_cast<float4 *>(B->d_rec[0]), reinterpret_cast<float4 *>(B->d_rec[0]) + B->rows};
  hipLaunchKernelGGL(k_bt_state_init, dim3((n + 255) / 256), dim3(256), 0, s, n, o->tol, o->max_iter, so);
  hipLaunchKernelGGL(k_bt_state_init, dim3((n + 255) / 256), dim3(256), 0, s, n, inner_tol, o->max_iter, si);
  iters.assign(n, 0);
  outers.assign(n, 0);
  int total = 0;
  bool all = false;
  int bad = -1;
  for (int outer = 0; outer < 200; outer++) {
    dispatch_L(B->tune.lanes, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_bt_ir_residual<LL>), dim3(G), dim3(blk), 0, s, G, (const int4 *)B->d_tiles,
                         (const int *)B->d_rp, (const int *)B->d_col, (const double *)B->d_A,
                         (const double *)B->d_b, (const double *)B->d_x, B->d_r64, bregion(B, B_B));
      hipLaunchKernelGGL(k_bt_ir_init, dim3(G), dim3(blk), 0, s, G, (const int4 *)B->d_tiles,
                         (const int4 *)B->d_tinfo, inner_tol, (const double *)B->d_r64, (const float *)B->d_dinv32,
                         R32[0], R32[1], B->d_d32, B->d_p32, (const double *)bregion(B, B_B), bregion(B, B_INIT),
                         so, si);
    });
    CGP_HIP(hipGetLastError());
    BTRY(poll_states(B, &all, &bad, 0));
    for (int i = 0; i < n; i++)
      if (!outers[i] && (B->h_state[i].done[0] || B->h_state[i].status)) outers[i] = outer + 1;
    if (all || bad >= 0 || total >= o->max_iter) break;
    dispatch_L(B->tune.lanes, [&](auto LC) {
      constexpr int LL = decltype(LC)::value;
      hipLaunchKernelGGL((k_bt_init_w<float, LL>), dim3(G), dim3(blk), 0, s, G, (const int4 *)B->d_tiles,
                         (const int *)B->d_t0, (const int *)B->d_nt, (const int *)B->d_rp, (const int *)B->d_col,
                         (const float *)B->d_A32, R32[0], (const double *)bregion(B, B_INIT), bregion(B, B_A), si);
    });
    bool inner_all = false;
    int inner_bad = -1;
    for (int it0 = 0; total < o->max_iter; it0 += K) {
      enqueue_chunk(B, it0, K, true);
      CGP_HIP(hipGetLastError());
      total += K;
      BTRY(poll_states(B, &inner_all, &inner_bad, n));
      if (inner_all || inner_bad >= 0) break;
    }
    for (int i = 0; i < n; i++) iters[i] += B->h_state[n + i].iters;
    if (inner_bad >= 0) {
      bad = inner_bad;
      break;
    }
    hipLaunchKernelGGL(k_bt_ir_update, dim3(G), dim3(256), 0, s, (const int4 *)B->d_tiles,
                       (const KrylovState *)so, (const KrylovState *)si, B->d_x, (const float *)B->d_d32);
    CGP_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(k_bt_zero_b, dim3(G), dim3(256), 0, s, (const int4 *)B->d_tiles, (const KrylovState *)so,
                     B->d_x);
  CGP_HIP(hipGetLastError());
  *launched = total;
  if (bad >= 0) {
    set_error("batched FP32-refinement Poisson solve: instance " + std::to_string(bad) +
              " produced a non-finite residual");
    return CGP_E_NONFINITE;
  }
  if (!all) {
    set_error("batched FP32-refinement Poisson solve: iteration limit reached before every instance converged");
    return CGP_E_NOCONV;
  }
  return CGP_OK;
}

}  // namespace
}  // namespace cgp

using namespace cgp;

extern "C" {

void cgp_batch_destroy(cgp_batch *B) {
  if (!B) return;
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  drop_graphs(B);
  for (void *p : B->allocations) (void)hipFree(p);
  if (B->h_state) (void)hipHostFree(B->h_state);
  if (B->ev_in) (void)hipEventDestroy(B->ev_in);
  if (B->ev_out) (void)hipEventDestroy(B->ev_out);
  for (hipStream_t a : B->aux) (void)hipStreamDestroy(a);
  for (hipEvent_t e : B->aux_ev) (void)hipEventDestroy(e);
  if (B->stream) (void)hipStreamDestroy(B->stream);
  delete B;
}

cgp_status cgp_batch_create(cgp_mesh *const *meshes, int32_t n, cgp_batch **out) {
  if (!meshes || !out || n < 1) {
    set_error("cgp_batch_create: need at least one mesh");
    return CGP_E_ARG;
  }
  long rows = 0, nnz = 0;
  for (int i = 0; i < n; i++) {
    cgp_mesh *m = meshes[i];
    if (!m || m->host_only || !m->assembled) {
      set_error("cgp_batch_create: every mesh must be a device mesh that has been assembled");
      return CGP_E_STATE;
    }
    if (m->stream != meshes[0]->stream) {
      set_error("cgp_batch_create: all meshes must use the same stream");
      return CGP_E_ARG;
    }
    rows += m->pc.n;
    nnz += m->pc.nnz;
  }
  if (nnz >= (1L << 31) - 1) {
    set_error("cgp_batch_create: more than 2^31 coarse nonzeros in total");
    return CGP_E_ARG;
  }
  cgp_batch *B = new cgp_batch();
  auto fail = [&](cgp_status st) {
    std::string msg = cgp_last_error();
    cgp_batch_destroy(B);
    set_error(msg);
    return st;
  };
  B->meshes.assign(meshes, meshes + n);
  B->ninst = n;
  B->rows = rows;
  B->nnz = nnz;
  B->mstream = meshes[0]->stream;
  const int naux = std::min(n, kBatchLanes);
  B->aux.assign(naux, nullptr);
  B->aux_ev.assign(naux + 1, nullptr);
  for (int k = 0; k < naux; k++)
    if (hipStreamCreateWithFlags(&B->aux[k], hipStreamNonBlocking) != hipSuccess) {
      set_error("cgp_batch_create: stream creation failed");
      return fail(CGP_E_DEVICE);
    }
  for (auto &e : B->aux_ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      set_error("cgp_batch_create: event creation failed");
      return fail(CGP_E_DEVICE);
    }
  if (hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming) != hipSuccess) {
    set_error("cgp_batch_create: stream or event creation failed");
    return fail(CGP_E_DEVICE);
  }
  cgp_status st;
  if ((st = balloc(B, &B->d_rp, rows + 1)) || (st = balloc(B, &B->d_col, nnz)) || (st = balloc(B, &B->d_A, nnz)) ||
      (st = balloc(B, &B->d_dinv, rows)) || (st = balloc(B, &B->d_x, rows)) || (st = balloc(B, &B->d_b, rows)) ||
      (st = balloc(B, &B->d_p, rows)) || (st = balloc(B, &B->d_rec[0], rows)) ||
      (st = balloc(B, &B->d_rec[1], rows)) ||
      (st = balloc(B, &B->d_A32, nnz)) || (st = balloc(B, &B->d_dinv32, rows)) ||
      (st = balloc(B, &B->d_d32, rows)) || (st = balloc(B, &B->d_p32, rows)) || (st = balloc(B, &B->d_r64, rows)) ||
      (st = balloc(B, &B->d_t0, n)) || (st = balloc(B, &B->d_nt, n)) || (st = balloc(B, &B->d_state, 2 * n)))
    return fail(st);
  if (hipMemset(B->d_state, 0, sizeof(KrylovState) * 2 * n) != hipSuccess) {
    set_error("cgp_batch_create: state initialisation failed");
    return fail(CGP_E_DEVICE);
  }
  if (hipHostMalloc((void **)&B->h_state, sizeof(KrylovState) * 2 * n, hipHostMallocDefault) != hipSuccess) {
    set_error("cgp_batch_create: pinned allocation failed");
    return fail(CGP_E_OOM);
  }
  // concatenated CSR with global indices; values copied from each mesh's coarse operator
  std::vector<int> rp(rows + 1), col(nnz);
  B->row_off.assign(n + 1, 0);
  B->nnz_off.assign(n + 1, 0);
  for (int i = 0; i < n; i++) {
    const HostCSR &c = meshes[i]->pc;
    const long r0 = B->row_off[i], z0 = B->nnz_off[i];
    for (int r = 0; r < c.n; r++) rp[r0 + r] = (int)(z0 + c.rp[r]);
    for (int k = 0; k < c.nnz; k++) col[z0 + k] = (int)(r0 + c.col[k]);
    B->row_off[i + 1] = r0 + c.n;
    B->nnz_off[i + 1] = z0 + c.nnz;
  }
  rp[rows] = (int)nnz;
  if (hipMemcpy(B->d_rp, rp.data(), sizeof(int) * rp.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(B->d_col, col.data(), sizeof(int) * col.size(), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("cgp_batch_create: upload failed");
    return fail(CGP_E_DEVICE);
  }
  if (hipStreamSynchronize(B->mstream) != hipSuccess) {
    set_error("cgp_batch_create: mesh stream failed");
    return fail(CGP_E_DEVICE);
  }
  for (int i = 0; i < n; i++) {
    cgp_mesh *m = meshes[i];
    if (hipMemcpyAsync(B->d_A + B->nnz_off[i], m->d_Kbc, sizeof(double) * m->pc.nnz, hipMemcpyDeviceToDevice,
                       B->stream) != hipSuccess ||
        hipMemcpyAsync(B->d_dinv + B->row_off[i], m->d_dinvK, sizeof(double) * m->pc.n, hipMemcpyDeviceToDevice,
                       B->stream) != hipSuccess ||
        hipMemcpyAsync(B->d_A32 + B->nnz_off[i], m->d_Kbc32, sizeof(float) * m->pc.nnz, hipMemcpyDeviceToDevice,
                       B->stream) != hipSuccess ||
        hipMemcpyAsync(B->d_dinv32 + B->row_off[i], m->d_dinvK32, sizeof(float) * m->pc.n, hipMemcpyDeviceToDevice,
                       B->stream) != hipSuccess) {
      set_error("cgp_batch_create: operator copy failed");
      return fail(CGP_E_DEVICE);
    }
  }
  if ((st = build_tiles(B))) return fail(st);
  *out = B;
  return CGP_OK;
}

cgp_status cgp_batch_get_tuning(const cgp_batch *B, cgp_batch_tuning *out) {
  if (!B || !out) {
    set_error("cgp_batch_get_tuning: null argument");
    return CGP_E_ARG;
  }
  *out = B->tune;
  return CGP_OK;
}

cgp_status cgp_batch_set_tuning(cgp_batch *B, const cgp_batch_tuning *t) {
  if (!B || !t || (t->lanes != 2 && t->lanes != 4 && t->lanes != 8 && t->lanes != 16) || t->block < 64 || t->block > 1024 ||
      (t->block & (t->block - 1)) || t->passes < 1 || t->passes > 64 || t->chunk < 2 || t->chunk > 256 ||
      (t->chunk & 1) || (t->use_graph != 0 && t->use_graph != 1) || t->ahead < 0 || t->ahead > 2 ||
      (t->ahead && ((t->lanes != 4 && t->lanes != 8) ||
                    (t->passes != 1 && t->passes != 2 && t->passes != 4 && !(t->passes == 8 && t->lanes == 8))))) {
    set_error("cgp_batch_set_tuning: lanes 2/4/8/16, block a power of two in 64..1024, passes 1..64, "
              "chunk even in 2..256, use_graph 0/1, ahead 0/1/2 (ahead 1, 2: lanes 4/8, passes 1/2/4, or 8 with 8 lanes)");
    return CGP_E_ARG;
  }
  const bool shape = t->lanes != B->tune.lanes || t->block != B->tune.block || t->passes != B->tune.passes;
  const bool chunk = t->chunk != B->tune.chunk || t->use_graph != B->tune.use_graph || t->ahead != B->tune.ahead;
  B->tune = *t;
  if (shape) return build_tiles(B);
  if (chunk) drop_graphs(B);
  return CGP_OK;
}

cgp_status cgp_batch_poisson_solve(cgp_batch *B, const double *const *rhs, double *const *x,
                                   const cgp_solver_opts *o, cgp_stats *stats) {
  if (!B || !rhs || !x || !o || !(o->tol > 0.0) || o->max_iter < 1 ||
      (o->precision != CGP_PREC_FP64 && o->precision != CGP_PREC_FP32_IR) || o->x0_mode < CGP_X0_ZERO ||
      o->x0_mode > CGP_X0_POD_GALERKIN || o->method != CGP_METHOD_DEFAULT) {
    set_error("cgp_batch_poisson_solve: bad argument (Jacobi-PCG in FP64 or FP32_IR; x0 zero, previous, learned or "
              "POD-Galerkin)");
    return CGP_E_ARG;
  }
  for (int i = 0; i < B->ninst; i++)
    if (!rhs[i] || !x[i]) {
      set_error("cgp_batch_poisson_solve: null vector");
      return CGP_E_ARG;
    }
  // gather on the meshes' stream, with each instance's boundary conditions (as in the single solve)
  hipStream_t ms = B->mstream;
  for (int i = 0; i < B->ninst; i++) {
    cgp_mesh *m = B->meshes[i];
    const long off = B->row_off[i];
    const size_t bytes = sizeof(double) * m->pc.n;
    CGP_HIP(hipMemcpyAsync(B->d_b + off, rhs[i], bytes, hipMemcpyDeviceToDevice, ms));
    if (o->x0_mode == CGP_X0_ZERO) CGP_HIP(hipMemsetAsync(B->d_x + off, 0, bytes, ms));
    else CGP_HIP(hipMemcpyAsync(B->d_x + off, x[i], bytes, hipMemcpyDeviceToDevice, ms));
    if (m->n_pdir > 0) launch_pdir_zero(m, B->d_b + off, B->d_x + off);
    else launch_mean_shift(m, B->d_b + off, nullptr, double(m->pc.n), m->red.partials);
    if (o->x0_mode >= CGP_X0_LEARNED) {
      // the instance's own attached model or online basis, as in its single solve
      BTRY(guess_initial(m, o->x0_mode, B->d_b + off, B->d_x + off));
      if (m->n_pdir > 0) launch_pdir_zero(m, B->d_b + off, B->d_x + off);
    }
  }
  CGP_HIP(hipGetLastError());
  CGP_HIP(hipEventRecord(B->ev_in, ms));
  CGP_HIP(hipStreamWaitEvent(B->stream, B->ev_in, 0));
  int launched = 0;
  const auto t0 = std::chrono::steady_clock::now();
  const bool ir = (o->precision == CGP_PREC_FP32_IR);
  std::vector<int> ir_iters, ir_outers;
  cgp_status rs = ir ? solve_ir(B, o, &launched, ir_iters, ir_outers) : solve(B, o->tol, o->max_iter, &launched);
  const double ms_solve = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (rs != CGP_OK && rs != CGP_E_NOCONV) return rs;
  CGP_HIP(hipEventRecord(B->ev_out, B->stream));
  CGP_HIP(hipStreamWaitEvent(ms, B->ev_out, 0));
  for (int i = 0; i < B->ninst; i++) {
    cgp_mesh *m = B->meshes[i];
    const long off = B->row_off[i];
    if (m->n_pdir == 0) launch_mean_shift(m, B->d_x + off, m->d_mc, m->mc_sum, m->red.partials);
    CGP_HIP(hipMemcpyAsync(x[i], B->d_x + off, sizeof(double) * m->pc.n, hipMemcpyDeviceToDevice, ms));
    const KrylovState &h = B->h_state[i];
    if (h.done[0] && !h.status) BTRY(guess_record(m, x[i]));  // online window of a converged instance
  }
  CGP_HIP(hipGetLastError());
  if (stats)
    for (int i = 0; i < B->ninst; i++) {
      const KrylovState &h = B->h_state[i];
      stats[i] = cgp_stats{};
      stats[i].p_iters = ir ? ir_iters[i] : h.iters;
      stats[i].p_outer = ir ? ir_outers[i] : 1;
      stats[i].p_relres = h.bnorm[0] > 0 ? h.rnorm[0] / h.bnorm[0] : 0.0;
      stats[i].ms_poisson = (float)ms_solve;
      stats[i].n_dominant = launched;  // launches of the batched iteration kernel (all instances)
    }
  return rs;
}

cgp_status cgp_batch_step(cgp_batch *B, const cgp_step_opts *o, const double *const *g, const double *const *f,
                          double *const *u, double *const *pf, double *const *pc, cgp_stats *stats) {
  if (!B || !o || !g || !u || !pf || !pc) {
    set_error("cgp_batch_step: null argument");
    return CGP_E_ARG;
  }
  const int n = B->ninst;
  for (int i = 0; i < n; i++)
    if (B->meshes[i]->params.pressure_mode != CGP_PRESSURE_NONINCREMENTAL) {
      set_error("cgp_batch_step: the incremental pressure modes are served by cgp_step only");
      return CGP_E_ARG;
    }
  std::vector<cgp_stats> S(n);
  std::vector<const double *> bc(n);
  // phases 1-2 and 4-5 per instance, on the auxiliary streams from one host thread per stream (each
  // mesh is touched by one thread; its stream is swapped for the phase and restored)
  auto per_instance = [&](auto &&body) -> cgp_status {
    const int T = (int)B->aux.size();
    CGP_HIP(hipEventRecord(B->aux_ev[T], B->mstream));
    for (int k = 0; k < T; k++) CGP_HIP(hipStreamWaitEvent(B->aux[k], B->aux_ev[T], 0));
    std::vector<cgp_status> st(T, CGP_OK);
    std::vector<std::string> msg(T);
    int dev = 0;
    CGP_HIP(hipGetDevice(&dev));
    auto work = [&](int k) {
      if (hipSetDevice(dev) != hipSuccess) {  // the current device is per host thread
        st[k] = CGP_E_DEVICE;
        msg[k] = "cgp_batch_step: hipSetDevice failed in a worker thread";
        return;
      }
      for (int i = k; i < n; i += T) {
        cgp_mesh *m = B->meshes[i];
        m->stream = B->aux[k];
        const cgp_status r = body(i, m);
        m->stream = B->mstream;
        if (r != CGP_OK && (st[k] == CGP_OK || st[k] == CGP_E_NOCONV)) {
          st[k] = r;
          msg[k] = cgp_last_error();
        }
        if (r != CGP_OK && r != CGP_E_NOCONV) return;
      }
    };
    std::vector<std::thread> pool;
    int started = 1;
    try {
      for (int k = 1; k < T; k++, started++) pool.emplace_back(work, k);
    } catch (const std::exception &) {  // no more threads: the rest run on this one
    }
    work(0);
    for (int k = started; k < T; k++) work(k);
    for (auto &t : pool) t.join();
    for (int k = 0; k < T; k++) {
      CGP_HIP(hipEventRecord(B->aux_ev[k], B->aux[k]));
      CGP_HIP(hipStreamWaitEvent(B->mstream, B->aux_ev[k], 0));
    }
    cgp_status worst = CGP_OK;
    for (int k = 0; k < T; k++)
      if (st[k] != CGP_OK && (worst == CGP_OK || worst == CGP_E_NOCONV)) {
        worst = st[k];
        set_error(msg[k]);
      }
    return worst;
  };
  cgp_status worst = CGP_OK;
  auto note = [&](cgp_status s) {
    if (s == CGP_E_NOCONV && worst == CGP_OK) worst = s;
    return s == CGP_OK || s == CGP_E_NOCONV;
  };
  // phase times (timing >= 1): host wall clock around each phase, whose calls return after their polls
  using clk = std::chrono::steady_clock;
  auto ms_since = [](clk::time_point t0) {
    return (float)std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  };
  clk::time_point t0 = clk::now();
  float ms_mom = 0.0f, ms_p = 0.0f, ms_cor = 0.0f;
  // steps 1-2 (Eqs. 19-21) per instance
  cgp_status s = per_instance([&](int i, cgp_mesh *m) {
    cgp_status r = drv_momentum(m, &o->momentum, g[i], f ? f[i] : nullptr, u[i], m->d_ut, &S[i]);
    if (r != CGP_OK && r != CGP_E_NOCONV) return r;
    const cgp_status r2 = drv_restrict(m, m->d_ut, m->d_bc);
    return r2 != CGP_OK ? r2 : r;
  });
  if (!note(s)) return s;
  if (o->timing >= 1) {
    CGP_HIP(hipStreamSynchronize(B->mstream));
    ms_mom = ms_since(t0);
    t0 = clk::now();
  }
  for (int i = 0; i < n; i++) bc[i] = B->meshes[i]->d_bc;
  // step 3 (Eq. 21): every instance's Poisson solve in one PCG
  std::vector<cgp_stats> P(n);
  s = cgp_batch_poisson_solve(B, bc.data(), pc, &o->poisson, P.data());
  if (!note(s)) return s;
  if (o->timing >= 1) {
    CGP_HIP(hipStreamSynchronize(B->mstream));
    ms_p = ms_since(t0);
    t0 = clk::now();
  }
  // steps 4-5 (Eqs. 22-23) per instance
  s = per_instance([&](int i, cgp_mesh *m) {
    const cgp_status r = drv_prolong(m, pc[i], pf[i]);
    if (r != CGP_OK) return r;
    return drv_correct(m, &o->mass, g[i], m->d_ut, pf[i], u[i], &S[i]);
  });
  if (!note(s)) return s;
  if (o->timing >= 1) {
    CGP_HIP(hipStreamSynchronize(B->mstream));
    ms_cor = ms_since(t0);
  }
  for (int i = 0; i < n; i++) {
    S[i].p_iters = P[i].p_iters;
    S[i].p_outer = P[i].p_outer;
    S[i].p_relres = P[i].p_relres;
    S[i].ms_poisson = P[i].ms_poisson;
    S[i].n_dominant = P[i].n_dominant;
    if (o->timing >= 1) {  // the batch's phase wall times, the same for every instance
      S[i].ms_momentum = ms_mom;  // momentum and restriction of all instances
      S[i].ms_poisson = ms_p;
      S[i].ms_correct = ms_cor;   // prolongation and correction of all instances
    }
  }
  CGP_HIP(hipStreamSynchronize(B->mstream));
  if (stats) std::copy(S.begin(), S.end(), stats);
  return worst;
}

// Time `iters` iterations of each candidate shape on a synthetic right-hand side (tolerance 0, so no
// instance converges) and keep the fastest.  The choice is cached in `cache_path` (JSON, one entry per
// batch size class: rows and nonzeros rounded to two significant digits) and reused when present.
cgp_status cgp_batch_autotune(cgp_batch *B, const char *cache_path, cgp_batch_tuning *chosen) {
  if (!B) {
    set_error("cgp_batch_autotune: null batch");
    return CGP_E_ARG;
  }
  auto round2 = [](long v) {
    long p = 1;
    while (v >= 100 * p) p *= 10;
    return (v + p / 2) / p * p;
  };
  char key[96];
  std::snprintf(key, sizeof(key), "v2_rows%ld_nnz%ld_inst%d", round2(B->rows), round2(B->nnz), B->ninst);
  // cache lookup: lines of the form  "key": {"lanes": L, "block": B, "passes": P, ...}
  std::string text;
  if (cache_path) {
    std::ifstream in(cache_path);
    std::stringstream ss;
    ss << in.rdbuf();
    text = ss.str();
    const std::string needle = std::string("\"") + key + "\"";
    const size_t at = text.find(needle);
    if (at != std::string::npos) {
      cgp_batch_tuning t = B->tune;
      if (std::sscanf(text.c_str() + at + needle.size(),
                      ": {\"lanes\": %d, \"block\": %d, \"passes\": %d, \"ahead\": %d", &t.lanes, &t.block,
                      &t.passes, &t.ahead) == 4) {
        BTRY(cgp_batch_set_tuning(B, &t));
        if (chosen) *chosen = B->tune;
        return CGP_OK;
      }
    }
  }
  const cgp_batch_tuning keep = B->tune;
  const int lanes[3] = {2, 4, 8}, blocks[3] = {256, 512, 1024}, passes[4] = {1, 2, 4, 8};
  cgp_batch_tuning best = keep;
  double best_us = 1e30;
  std::string table;
  hipEvent_t e0, e1;
  CGP_HIP(hipEventCreate(&e0));
  CGP_HIP(hipEventCreate(&e1));
  for (int ah = 0; ah < 3; ah++)
  for (int L : lanes)
    for (int blk : blocks)
      for (int ps : passes) {
        if (ah && L == 2) continue;  // the loads-ahead kernels are built for 4 and 8 lanes
        if (ps == 8 && !(ah && L == 8)) continue;  // 8 rows per lane group: loads ahead with 8 lanes only
        cgp_batch_tuning t = keep;
        t.lanes = L;
        t.block = blk;
        t.passes = ps;
        t.ahead = ah;
        t.use_graph = 1;
        t.chunk = 16;
        BTRY(cgp_batch_set_tuning(B, &t));
        double us = 0.0;
        for (int rep = 0; rep < 2; rep++) {  // the first repetition also captures the graphs
          hipLaunchKernelGGL(k_bt_fill, dim3((B->rows + 255) / 256), dim3(256), 0, B->stream, B->rows, B->d_b,
                             B->d_x);
          int launched = 0;
          CGP_HIP(hipEventRecord(e0, B->stream));
          cgp_status s = solve(B, 0.0, 64, &launched);
          CGP_HIP(hipEventRecord(e1, B->stream));
          if (s != CGP_OK && s != CGP_E_NOCONV) return s;
          CGP_HIP(hipEventSynchronize(e1));
          float ms = 0.0f;
          CGP_HIP(hipEventElapsedTime(&ms, e0, e1));
          us = 1e3 * ms / launched;
        }
        char line[160];
        std::snprintf(line, sizeof(line),
                      "%s{\"lanes\": %d, \"block\": %d, \"passes\": %d, \"ahead\": %d, \"us_per_iteration\": %.3f}",
                      table.empty() ? "" : ", ", L, blk, ps, ah, us);
        table += line;
        if (us < best_us) {
          best_us = us;
          best = t;
        }
      }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  best.use_graph = keep.use_graph;
  best.chunk = keep.chunk;
  BTRY(cgp_batch_set_tuning(B, &best));
  if (chosen) *chosen = B->tune;
  if (cache_path) {
    char head[256];
    std::snprintf(head, sizeof(head),
                  "\"%s\": {\"lanes\": %d, \"block\": %d, \"passes\": %d, \"ahead\": %d, \"us_per_iteration\": %.3f, ",
                  key, best.lanes, best.block, best.passes, best.ahead, best_us);
    const std::string entry = std::string(head) + "\"candidates\": [" + table + "]}";
    // append the entry to the JSON object (the file holds one object of entries and a log of timings)
    std::string body = text;
    const size_t close = body.rfind('}');
    if (body.empty() || close == std::string::npos) body = std::string("{\n  ") + entry + "\n}\n";
    else body = body.substr(0, close) + (body.find('"') != std::string::npos ? ",\n  " : "  ") + entry + "\n}\n";
    std::ofstream out(cache_path, std::ios::trunc);
    out << body;
    if (!out) {
      set_error(std::string("cgp_batch_autotune: cannot write ") + cache_path);
      return CGP_E_ARG;
    }
  }
  return CGP_OK;
}

}  // extern "C"
