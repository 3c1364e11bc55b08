// Device helpers shared by libcgp's kernels (gfx950, wave64).
//
// Grid-wide sums are deterministic and fence-free.  A producer kernel
// reduces each of its K values inside the block (wave64 butterfly, then LDS in
// wave order) and stores one partial per block, P[k][gridDim.x], with plain
// stores.  The next kernel in the stream sees them complete (kernel boundary)
// and every one of its blocks sums the G partials itself in the same fixed
// order, so all blocks hold bit-identical totals; block 0 publishes whatever
// later kernels or the host need.  No device-scope fence is executed inside a
// kernel: on a multi-XCD part such a fence writes back and invalidates the
// XCD's L2, which costs far more than one more kernel boundary.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace cgp {
namespace dev {

constexpr int kMaxBlock = 1024;  // largest block of a reducing kernel (sizes the LDS scratch)

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

template <int L>
__device__ __forceinline__ float group_sumf(float x) {
#pragma unroll
  for (int off = L / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, L);
  return x;
}

// A classification test, not x - x == 0: with floating-point contraction (the HIP default) a
// product's x - x can become fma(a, b, -(a b)), its rounding error, and reject finite values.
__device__ __forceinline__ bool is_finite(double x) { return __builtin_isfinite(x); }

// Sum K values over the block in a fixed order; every thread gets the totals.
template <int K>
__device__ __forceinline__ void block_sum(const double (&v)[K], double (&tot)[K]) {
  __shared__ double sh[K][kMaxBlock / 64];
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
    res[threadIdx.x] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; k++) tot[k] = res[k];
  __syncthreads();  // sh/res may be reused by the next call
}

// Producer side: store this block's K sums as P[k * gridDim.x + blockIdx.x].
template <int K>
__device__ __forceinline__ void put_partials(const double (&v)[K], double *__restrict__ P) {
  double tot[K];
  block_sum<K>(v, tot);
  if (threadIdx.x < K) {
#pragma unroll
    for (int k = 0; k < K; k++)
      if (threadIdx.x == k) P[k * gridDim.x + blockIdx.x] = tot[k];
  }
}

// Consumer side: totals of K partial arrays of length G written by the previous kernel.
template <int K>
__device__ __forceinline__ void sum_partials(const double *__restrict__ P, int G, double (&tot)[K]) {
  double v[K];
#pragma unroll
  for (int k = 0; k < K; k++) {
    double s = 0.0;
    for (int b = threadIdx.x; b < G; b += blockDim.x) s += P[k * G + b];
    v[k] = s;
  }
  block_sum<K>(v, tot);
}

// Per-node records of the single-kernel PCG: {r, w, s, D^-1} in double4 (FP64) or float4 (FP32).
template <typename T> struct rec_of;
template <> struct rec_of<double> { using type = double4; };
template <> struct rec_of<float> { using type = float4; };
template <typename T> using rec_t = typename rec_of<T>::type;

// store the r, w, s fields of a record (D^-1 stays)
__device__ __forceinline__ void store_rws(double4 *q, double r, double w, double s) {
  *reinterpret_cast<double2 *>(q) = make_double2(r, w);
  q->z = s;
}
__device__ __forceinline__ void store_rws(float4 *q, float r, float w, float s) {
  *reinterpret_cast<float2 *>(q) = make_float2(r, w);
  q->z = s;
}

// Consumer side without LDS or barriers: every wave sums the K partial arrays of length G
// itself (U loads per lane issued together, the rest in a loop, then the wave butterfly).  The
// order is fixed, so every wave of every block holds bit-identical totals, and a wave can start
// work that does not need them while its loads are in flight.
template <int K, int U>
__device__ __forceinline__ void wave_partials(const double *__restrict__ P, int G, double (&tot)[K]) {
  const int l = threadIdx.x & 63;
  double a[K][U];
#pragma unroll
  for (int u = 0; u < U; u++) {
    const int b = l + 64 * u;
#pragma unroll
    for (int k = 0; k < K; k++) a[k][u] = b < G ? P[k * G + b] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < K; k++) {
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < U; u++) s += a[k][u];
    for (int b = l + 64 * U; b < G; b += 64) s += P[k * G + b];
    tot[k] = wave_sum(s);
  }
}

// Producer side with a single barrier: the block's partials go straight from LDS to P.  It has
// its own LDS array and must be the block's last reduction.
template <int K>
__device__ __forceinline__ void put_partials_last(const double (&v)[K], double *__restrict__ P) {
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
    P[threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

}  // namespace dev
}  // namespace cgp
