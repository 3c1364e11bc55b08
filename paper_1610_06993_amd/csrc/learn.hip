// Learned initial guess for the coarse pressure Poisson solve.
//
// A proper-orthogonal-decomposition (POD) basis Phi [n_c][m] of pressure
// snapshots, orthonormal in the coarse lumped-mass inner product, and a
// multilayer perceptron m -> h -> h -> m (GELU) that maps the normalised modal
// projection of the Poisson right-hand side, Phi^T b, to the normalised modal
// coefficients of the pressure, Phi^T M p.  The guess is x0 = Phi c, or the
// previous pressure with its POD-subspace component replaced by Phi c.
//
// The network runs in BF16 with FP32 accumulation on the gfx950 matrix cores
// (v_mfma_f32_16x16x32_bf16): inputs, weights, activations and back-propagated
// deltas are rounded to BF16 (round to nearest even) where they enter a GEMM;
// pre-activations, outputs, gradients, biases and the Adam state stay in FP32.
// Projection and expansion against the basis are FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "devutil.h"
#include "kernels.h"
#include "learn.h"
#include "symeig.h"

namespace cgp {
// blocks of the POD projection (one partial per block and mode) and of the expansion
constexpr int kProjectGrid = 1024, kExpandGrid = 2048;
namespace {
cgp_status pod_events(cgp_guess *g);
cgp_status pod_finish(cgp_guess *g);
cgp_status pod_stage_gram(cgp_guess *g, hipStream_t st, const double *snaps, int S);
}  // namespace
namespace ldev {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) unsigned short u16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

// FP32 -> BF16, round to nearest even (NaN stays NaN)
__device__ __forceinline__ unsigned short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (unsigned short)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * expf(-0.5f * z * z);
  return cdf + z * pdf;
}

// C[M][N] = A[M][K] B[K][N] on the matrix cores.  Strides are in elements:
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn].  One wave computes a
// 16x16 tile with v_mfma_f32_16x16x32_bf16: lane l supplies row (l % 16) of A
// and column (l % 16) of B for the 8 values of k in slot (l / 16), and holds
// C rows 4*(l/16)..+3 of column l % 16.  Out-of-range entries are zero.
// Epilogues: EPI 0 stores C (+ bias[n]); EPI 1 stores z = C + bias[n] (FP32)
// and h = bf16(GELU(z)).
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_bf16(int M, int N, int K, const unsigned short *__restrict__ A, long sam,
                                                  long sak, const unsigned short *__restrict__ B, long sbk, long sbn,
                                                  const float *__restrict__ bias, float *__restrict__ C, long ldc,
                                                  unsigned short *__restrict__ H, long ldh) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tm = (blockIdx.y * 2 + (wave >> 1)) * 16, tn = (blockIdx.x * 2 + (wave & 1)) * 16;
  if (tm >= M || tn >= N) return;  // whole wave leaves together
  const int r = lane & 15, g = lane >> 4;
  const int am = tm + r, bn = tn + r;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    u16x8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int k = k0 + g * 8 + e;
      av[e] = (am < M && k < K) ? A[am * sam + k * sak] : (unsigned short)0;
      bv[e] = (bn < N && k < K) ? B[k * sbk + bn * sbn] : (unsigned short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av), __builtin_bit_cast(bf16x8, bv), acc,
                                                  0, 0, 0);
  }
  const int cn = tn + r;
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int cm = tm + g * 4 + i;
    if (cm >= M || cn >= N) continue;
    float v = acc[i] + (bias ? bias[cn] : 0.0f);
    C[cm * ldc + cn] = v;
    if (EPI == 1) H[cm * ldh + cn] = f2bf(gelu(v));
  }
}

// dY = 2 (Y - T) / (rows * cols); dYb = bf16(dY); per-block partial of sum (Y - T)^2
__global__ void k_mse(int count, float scale, const float *__restrict__ Y, const float *__restrict__ T,
                      float *__restrict__ dY, unsigned short *__restrict__ dYb, double *__restrict__ P) {
  double acc[1] = {0.0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const float e = Y[i] - T[i];
    const float d = scale * e;
    dY[i] = d;
    dYb[i] = f2bf(d);
    acc[0] += (double)e * (double)e;
  }
  dev::put_partials<1>(acc, P);
}

__global__ void k_sum_partials(int G, const double *__restrict__ P, double *__restrict__ out) {
  double t[1];
  dev::sum_partials<1>(P, G, t);
  if (threadIdx.x == 0) *out = t[0];
}

// dZ = dH * GELU'(Z) (FP32) and its BF16 copy
__global__ void k_gelu_back(int count, const float *__restrict__ dH, const float *__restrict__ Z, float *__restrict__ dZ,
                            unsigned short *__restrict__ dZb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float d = dH[i] * gelu_grad(Z[i]);
  dZ[i] = d;
  dZb[i] = f2bf(d);
}

// column sums of D[rows][cols] (bias gradients), one thread per column, fixed order
__global__ void k_colsum(int rows, int cols, const float *__restrict__ D, float *__restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int r = 0; r < rows; r++) s += D[r * cols + c];
  out[c] = s;
}

// Adam (Kingma & Ba) on FP32 master weights; refresh the BF16 copy
__global__ void k_adam(int count, float *__restrict__ w, unsigned short *__restrict__ wb, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wn = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wn;
  wb[i] = f2bf(wn);
}

__global__ void k_to_bf16(int count, const float *__restrict__ x, unsigned short *__restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) y[i] = f2bf(x[i]);
}

// rows of a feature table gathered by index: xb[r][:] = bf16(X[idx[r]][:]), t[r][:] = T[idx[r]][:]
__global__ void k_gather_batch(int rows, int cols, const int *__restrict__ idx, const float *__restrict__ X,
                               const float *__restrict__ T, unsigned short *__restrict__ xb, float *__restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int r = i / cols, c = i - r * cols;
  const int s = idx[r];
  xb[i] = f2bf(X[s * cols + c]);
  t[i] = T[s * cols + c];
}

// ---- basis kernels (FP64)
// Cpart[z][a][b] = sum over i in chunk z of P(a,i) w_i Y(i,b), with P(a,i) = P[a*spa + i*spi],
// Y(i,b) = Y[i*syi + b*syb]; 64x64 tile per block, each thread a 4x4 sub-tile, 32-row LDS stages.
// An operand stored along i (stride 1 in i, as the snapshot rows of a Gram matrix are) is staged by
// lanes walking i, so that a wave reads whole 256-byte runs; otherwise lanes walk the tile's columns.
__global__ void __launch_bounds__(256) k_gemm64(int M, int N, int K, int kchunk, const double *__restrict__ P,
                                                long spa, long spi, const double *__restrict__ w,
                                                const double *__restrict__ Y, long syi, long syb,
                                                double *__restrict__ Cpart) {
  __shared__ double sp[32][65], sy[32][65];
  const int ta = blockIdx.y * 64, tb = blockIdx.x * 64;
  const int i_beg = blockIdx.z * kchunk, i_end = min(K, i_beg + kchunk);
  // a thread's 4x4 outputs are rows tr + 16u and columns tc + 16v: the 16 column groups of a wave
  // then read 16 consecutive LDS words (no bank conflicts), where contiguous 4x4 blocks hit 4 banks
  const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
  double acc[4][4] = {};
  for (int i0 = i_beg; i0 < i_end; i0 += 32) {
    for (int e = threadIdx.x; e < 32 * 64; e += 256) {
      {
        const int ii = spi == 1 ? (e & 31) : (e >> 6), cc = spi == 1 ? (e >> 5) : (e & 63), i = i0 + ii;
        const int aa = ta + cc;
        sp[ii][cc] = (i < i_end && aa < M) ? P[aa * spa + (long)i * spi] * (w ? w[i] : 1.0) : 0.0;
      }
      {
        const int ii = syi == 1 ? (e & 31) : (e >> 6), cc = syi == 1 ? (e >> 5) : (e & 63), i = i0 + ii;
        const int bb = tb + cc;
        sy[ii][cc] = (i < i_end && bb < N) ? Y[(long)i * syi + bb * syb] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll 4
    for (int ii = 0; ii < 32; ii++) {
      double pa[4], yb[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        pa[u] = sp[ii][tr + 16 * u];
        yb[u] = sy[ii][tc + 16 * u];
      }
#pragma unroll
      for (int u = 0; u < 4; u++)
#pragma unroll
        for (int v = 0; v < 4; v++) acc[u][v] += pa[u] * yb[v];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; u++)
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int aa = ta + tr + 16 * u, bb = tb + tc + 16 * v;
      if (aa < M && bb < N) Cpart[((long)blockIdx.z * M + aa) * N + bb] = acc[u][v];
    }
}

// C[e] = sum over the chunks of Cpart[z][e], fixed order
__global__ void k_sum_chunks(long count, int chunks, const double *__restrict__ Cpart, double *__restrict__ C) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  double s = 0.0;
  for (int z = 0; z < chunks; z++) s += Cpart[z * count + e];
  C[e] = s;
}

// C[e] = sum over the chunks of Cpart[z][e], one block per output, fixed order
__global__ void __launch_bounds__(256) k_sum_chunks_blk(long count, int chunks, const double *__restrict__ Cpart,
                                                        double *__restrict__ C) {
  const long e = blockIdx.x;
  double v[1] = {0.0};
  for (int z = threadIdx.x; z < chunks; z += blockDim.x) v[0] += Cpart[(long)z * count + e];
  double t[1];
  dev::block_sum<1>(v, t);
  if (threadIdx.x == 0) C[e] = t[0];
}

// Y[i][k] = sum_j K[i][j] Phi[j][k]: a group of LPR lanes per row (lane = mode), 64 / LPR rows per wave
template <int LPR>
__global__ void __launch_bounds__(256) k_spmm_modes(int n, int nm, const int *__restrict__ rp,
                                                    const int *__restrict__ col, const double *__restrict__ val,
                                                    const double *__restrict__ Phi, double *__restrict__ Y) {
  constexpr int RPW = 64 / LPR;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sub = lane / LPR, l = lane % LPR;
  for (int i = (blockIdx.x * 4 + wave) * RPW + sub; i < n; i += gridDim.x * 4 * RPW) {
    double acc = 0.0;
    if (l < nm)
      for (int k = rp[i]; k < rp[i + 1]; k++) acc += val[k] * Phi[(long)col[k] * nm + l];
    if (l < nm) Y[(long)i * nm + l] = acc;
  }
}

// r = b - K x (one thread per row)
__global__ void k_residual(int n, const int *__restrict__ rp, const int *__restrict__ col,
                           const double *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
                           double *__restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = rp[i]; k < rp[i + 1]; k++) s += val[k] * x[col[k]];
  r[i] = b[i] - s;
}

// R[k][i] = B[k][i] - (K P[k])_i for every sample k (rows = samples); blockIdx.y = k
__global__ void k_pair_residual(int n, const int *__restrict__ rp, const int *__restrict__ col,
                                const double *__restrict__ val, const double *__restrict__ B,
                                const double *__restrict__ P, double *__restrict__ R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long k = blockIdx.y;
  const double *pk = P + k * n;
  double s = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; e++) s += val[e] * pk[col[e]];
  R[k * n + i] = B[k * n + i] - s;
}

// Lanes of a wave cover (row, mode) pairs of the row-major Phi [n][nm]: a span of 16, 32 or 64
// lanes per row (the next power of two >= nm), so one wave instruction reads 64 / span whole rows.
__device__ __forceinline__ int mode_span(int nm) { return nm <= 16 ? 16 : nm <= 32 ? 32 : 64; }

// per-block partials of out[k] = sum_i Phi[i][k] w_i v_i for the nm <= 64 modes; partials laid out
// [nm][grid]
__global__ void __launch_bounds__(256) k_project(int n, int nm, const double *__restrict__ Phi,
                                                 const double *__restrict__ w, const double *__restrict__ v,
                                                 double *__restrict__ P) {
  __shared__ double sh[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int span = mode_span(nm), sub = lane / span, k = lane % span, rpw = 64 / span;
  const long step = (long)gridDim.x * 4 * rpw;
  double acc = 0.0;
  if (k < nm) {
#pragma unroll 4
    for (long i = (long)(blockIdx.x * 4 + wave) * rpw + sub; i < n; i += step)
      acc += Phi[i * nm + k] * (w ? w[i] : 1.0) * v[i];
  }
  for (int off = span; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);  // the wave's rows of mode k
  sh[wave][lane] = acc;
  __syncthreads();
  if (threadIdx.x < nm) P[threadIdx.x * gridDim.x + blockIdx.x] = sh[0][threadIdx.x] + sh[1][threadIdx.x] +
                                                                     sh[2][threadIdx.x] + sh[3][threadIdx.x];
}

// out[k] = sum over the G partials of mode k (one block per mode, fixed order)
__global__ void __launch_bounds__(256) k_project_finish(int G, const double *__restrict__ P, double *__restrict__ out) {
  const double *p = P + (size_t)blockIdx.x * G;
  double v[1] = {0.0};
  for (int b = threadIdx.x; b < G; b += blockDim.x) v[0] += p[b];
  double tot[1];
  dev::block_sum<1>(v, tot);
  if (threadIdx.x == 0) out[blockIdx.x] = tot[0];
}

// x[i] = base[i] + sum_k Phi[i][k] c[k]  (base may be NULL or equal to x); the span of lanes of a row
// sums its modes
__global__ void __launch_bounds__(256) k_expand(int n, int nm, const double *__restrict__ Phi,
                                                const double *__restrict__ c, const double *base, double *x) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int span = mode_span(nm), sub = lane / span, k = lane % span, rpw = 64 / span;
  const double ck = k < nm ? c[k] : 0.0;
  const long step = (long)gridDim.x * 4 * rpw;
  for (long i0 = (long)(blockIdx.x * 4 + wave) * rpw; i0 < n; i0 += step) {  // uniform over the wave
    const long i = i0 + sub;
    double v = (k < nm && i < n) ? Phi[i * nm + k] * ck : 0.0;
    for (int off = span >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (k == 0 && i < n) x[i] = (base ? base[i] : 0.0) + v;
  }
}

// inference glue (one block): xb = bf16((a - mu_a) / sd_a)
__global__ void k_feat_in(int nm, const double *__restrict__ a, const double *__restrict__ mu,
                          const double *__restrict__ sd, unsigned short *__restrict__ xb) {
  const int k = threadIdx.x;
  if (k < nm) xb[k] = f2bf((float)((a[k] - mu[k]) / sd[k]));
}

// c = y * sd + mu
__global__ void k_feat_out(int nm, const float *__restrict__ y, const double *__restrict__ mu,
                           const double *__restrict__ sd, double *__restrict__ c) {
  const int k = threadIdx.x;
  if (k < nm) c[k] = (double)y[k] * sd[k] + mu[k];
}

// c = Kinv a (dense nm x nm, one thread per row)
__global__ void k_small_matvec(int nm, const double *__restrict__ Kinv, const double *__restrict__ a,
                               double *__restrict__ c) {
  const int k = threadIdx.x;
  if (k >= nm) return;
  double s = 0.0;
  for (int j = 0; j < nm; j++) s += Kinv[k * nm + j] * a[j];
  c[k] = s;
}

}  // namespace ldev

// ====================================================================== host side
using namespace ldev;

namespace {

template <typename T>
cgp_status galloc(cgp_guess *g, T **p, size_t count) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? CGP_E_OOM : CGP_E_DEVICE;
  }
  g->allocations.push_back(q);
  *p = static_cast<T *>(q);
  return CGP_OK;
}

// device scratch slot k of at least `count` doubles (kept and grown; freed with the guess)
cgp_status scratch(cgp_guess *g, int k, size_t count, double **out) {
  if (g->scr_cap[k] < count) {
    double *p = nullptr;
    cgp_status st = galloc(g, &p, count);
    if (st) return st;
    g->scr[k] = p;
    g->scr_cap[k] = count;
  }
  *out = g->scr[k];
  return CGP_OK;
}

// pinned host staging of at least `count` doubles
cgp_status pinned(cgp_guess *g, size_t count, double **out) {
  if (g->pin_cap < count) {
    if (g->h_pin) {
      CGP_HIP(hipStreamSynchronize(g->mesh->stream));  // a copy from the old staging may be in flight
      if (g->side) CGP_HIP(hipStreamSynchronize(g->side));
      (void)hipHostFree(g->h_pin);
    }
    g->h_pin = nullptr;
    g->pin_cap = 0;
    hipError_t e = hipHostMalloc((void **)&g->h_pin, sizeof(double) * count, hipHostMallocDefault);
    if (e != hipSuccess) {
      set_error(std::string("hipHostMalloc: ") + hipGetErrorString(e));
      return CGP_E_OOM;
    }
    g->pin_cap = count;
  }
  *out = g->h_pin;
  return CGP_OK;
}

#define GTRY(x)                  \
  do {                           \
    cgp_status s_ = (x);         \
    if (s_ != CGP_OK) return s_; \
  } while (0)

inline uint64_t splitmix(uint64_t &state) {
  uint64_t z = (state += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
inline double uniform01(uint64_t &state) { return double(splitmix(state) >> 11) * (1.0 / 9007199254740992.0); }

// parameter offsets
struct Layout {
  long w1, b1, w2, b2, w3, b3, total;
};
Layout layout(const cgp_guess *g) {
  Layout L{};
  const long m = g->nm, h = g->nh;
  L.w1 = 0;
  L.b1 = L.w1 + h * m;
  L.w2 = L.b1 + h;
  L.b2 = L.w2 + h * h;
  L.w3 = L.b2 + h;
  L.b3 = L.w3 + m * h;
  L.total = L.b3 + m;
  return L;
}

// C[M][N] (+)= A B with strided BF16 operands on the matrix cores
template <int EPI>
void gemm(hipStream_t s, int M, int N, int K, const unsigned short *A, long sam, long sak, const unsigned short *B,
          long sbk, long sbn, const float *bias, float *C, long ldc, unsigned short *H = nullptr, long ldh = 0) {
  dim3 grid((N + 31) / 32, (M + 31) / 32);
  hipLaunchKernelGGL((k_gemm_bf16<EPI>), grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, bias, C, ldc, H,
                     ldh);
}

// FP64 C[M][N] = sum_i P(a,i) w_i Y(i,b) through split-K partials
cgp_status gemm64(cgp_guess *g, hipStream_t s, int M, int N, int K, const double *P, long spa, long spi,
                  const double *w, const double *Y, long syi, long syb, double *C) {
  // split K so that about 512 blocks run, within 64 MB of partial sums
  const long tiles = (long)((N + 63) / 64) * ((M + 63) / 64);
  long chunks = std::max(1L, std::min((long)(K + 255) / 256, 512 / tiles));
  chunks = std::max(1L, std::min(chunks, (8L << 20) / ((long)M * N)));
  const int kchunk = (int)(((K + chunks - 1) / chunks + 31) / 32 * 32);
  chunks = (K + kchunk - 1) / kchunk;
  dim3 grid((N + 63) / 64, (M + 63) / 64, chunks);
  if (chunks == 1) {  // one K chunk: the partial is the result
    hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, s, M, N, K, kchunk, P, spa, spi, w, Y, syi, syb, C);
    CGP_HIP(hipGetLastError());
    return CGP_OK;
  }
  double *part = nullptr;
  cgp_status st = scratch(g, 4, (size_t)chunks * M * N, &part);
  if (st) return st;
  hipLaunchKernelGGL(k_gemm64, grid, dim3(256), 0, s, M, N, K, kchunk, P, spa, spi, w, Y, syi, syb, part);
  const long count = (long)M * N;
  if (count <= 65536)  // few outputs, many chunks: one block per output
    hipLaunchKernelGGL(k_sum_chunks_blk, dim3(count), dim3(256), 0, s, count, (int)chunks, (const double *)part, C);
  else
    hipLaunchKernelGGL(k_sum_chunks, dim3((count + 255) / 256), dim3(256), 0, s, count, (int)chunks,
                       (const double *)part, C);
  CGP_HIP(hipGetLastError());
  return CGP_OK;
}

void forward(cgp_guess *g, hipStream_t s, int B) {
  const Layout L = layout(g);
  const int m = g->nm, h = g->nh;
  const unsigned short *wb = g->d_wb;
  const float *w = g->d_w;
  gemm<1>(s, B, h, m, g->d_xb, m, 1, wb + L.w1, 1, m, w + L.b1, g->d_z1, h, g->d_h1b, h);
  gemm<1>(s, B, h, h, g->d_h1b, h, 1, wb + L.w2, 1, h, w + L.b2, g->d_z2, h, g->d_h2b, h);
  gemm<0>(s, B, m, h, g->d_h2b, h, 1, wb + L.w3, 1, h, w + L.b3, g->d_y, m);
}

// loss partials in d_part, gradients in d_g
void backward(cgp_guess *g, hipStream_t s, int B) {
  const Layout L = layout(g);
  const int m = g->nm, h = g->nh;
  const unsigned short *wb = g->d_wb;
  float *gr = g->d_g;
  const float scale = 2.0f / float(B * m);
  hipLaunchKernelGGL(k_mse, dim3(16), dim3(256), 0, s, B * m, scale, (const float *)g->d_y, (const float *)g->d_t,
                     g->d_dy, g->d_dyb, g->d_part);
  // layer 3
  gemm<0>(s, m, h, B, g->d_dyb, 1, m, g->d_h2b, h, 1, nullptr, gr + L.w3, h);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, B, m, (const float *)g->d_dy, gr + L.b3);
  gemm<0>(s, B, h, m, g->d_dyb, m, 1, wb + L.w3, h, 1, nullptr, g->d_dh2, h);
  hipLaunchKernelGGL(k_gelu_back, dim3((B * h + 255) / 256), dim3(256), 0, s, B * h, (const float *)g->d_dh2,
                     (const float *)g->d_z2, g->d_dz2, g->d_dz2b);
  // layer 2
  gemm<0>(s, h, h, B, g->d_dz2b, 1, h, g->d_h1b, h, 1, nullptr, gr + L.w2, h);
  hipLaunchKernelGGL(k_colsum, dim3((h + 255) / 256), dim3(256), 0, s, B, h, (const float *)g->d_dz2, gr + L.b2);
  gemm<0>(s, B, h, h, g->d_dz2b, h, 1, wb + L.w2, h, 1, nullptr, g->d_dh1, h);
  hipLaunchKernelGGL(k_gelu_back, dim3((B * h + 255) / 256), dim3(256), 0, s, B * h, (const float *)g->d_dh1,
                     (const float *)g->d_z1, g->d_dz1, g->d_dz1b);
  // layer 1
  gemm<0>(s, h, m, B, g->d_dz1b, 1, h, g->d_xb, m, 1, nullptr, gr + L.w1, m);
  hipLaunchKernelGGL(k_colsum, dim3((h + 255) / 256), dim3(256), 0, s, B, h, (const float *)g->d_dz1, gr + L.b1);
}

// columns of Y [S][q] made orthonormal (modified Gram-Schmidt, twice).  A column that enters the second
// pass with unit norm keeps most of it unless it lies in the span of the columns before it; one left
// with less than 1e-6 has no direction of its own (G of rank below q, e.g. snapshots that repeat bit for
// bit, whose products are exact multiples of one vector, so that their residuals normalise to that
// vector again) and is set to zero: Q^T G Q then has a zero row and column for it instead of counting an
// eigenvalue twice.
void orthonormalise(int S, int q, std::vector<double> &Y) {
  for (int pass = 0; pass < 2; pass++)
    for (int j = 0; j < q; j++) {
      for (int k = 0; k < j; k++) {
        double d = 0.0;
        for (int a = 0; a < S; a++) d += Y[(size_t)a * q + k] * Y[(size_t)a * q + j];
        for (int a = 0; a < S; a++) Y[(size_t)a * q + j] -= d * Y[(size_t)a * q + k];
      }
      double nrm = 0.0;
      for (int a = 0; a < S; a++) nrm += Y[(size_t)a * q + j] * Y[(size_t)a * q + j];
      nrm = std::sqrt(nrm);
      const bool keep = pass == 0 ? nrm > 0 : nrm > 1e-6;
      for (int a = 0; a < S; a++) Y[(size_t)a * q + j] = keep ? Y[(size_t)a * q + j] / nrm : 0.0;
    }
}

}  // namespace

cgp_status guess_initial(cgp_mesh *m, int mode, const double *b, double *x) {
  cgp_guess *g = m->guess;
  if (g) {
    cgp_status ps = pod_finish(g);  // an online rebuild started after the last solve
    if (ps) return ps;
  }
  if (g && g->win > 0 && mode == CGP_X0_POD_GALERKIN && !g->pod_ready) return CGP_OK;  // window still filling
  if (!g || !g->pod_ready || (mode != CGP_X0_POD_GALERKIN && !g->trained)) {
    set_error("learned initial guess requested but no trained model is attached");
    return CGP_E_STATE;
  }
  if ((mode == CGP_X0_LEARNED && g->incremental) || (mode == CGP_X0_LEARNED_CORR && !g->incremental)) {
    set_error(mode == CGP_X0_LEARNED ? "CGP_X0_LEARNED needs a model trained with incremental = 0"
                                     : "CGP_X0_LEARNED_CORR needs a model trained with incremental = 1");
    return CGP_E_STATE;
  }
  hipStream_t s = m->stream;
  const int n = g->n, nm = g->nm, G = kProjectGrid;
  double *a = g->d_scal, *c = g->d_scal + 64;
  const double *mu_a = g->d_stats, *sd_a = g->d_stats + nm, *mu_c = g->d_stats + 2 * nm, *sd_c = g->d_stats + 3 * nm;
  auto project = [&](const double *w, const double *v, double *out) {
    hipLaunchKernelGGL(k_project, dim3(G), dim3(256), 0, s, n, nm, (const double *)g->d_phi, w, v, g->d_part);
    hipLaunchKernelGGL(k_project_finish, dim3(nm), dim3(256), 0, s, G, (const double *)g->d_part, out);
  };
  // features: Phi^T b (absolute model) or Phi^T (b - K x) (incremental model and POD-Galerkin)
  const bool from_residual = (mode != CGP_X0_LEARNED);
  if (from_residual) {
    double *r = m->d_wc[7];
    hipLaunchKernelGGL(k_residual, dim3((n + 255) / 256), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c,
                       (const double *)m->d_Kbc, b, (const double *)x, r);
    project(nullptr, r, a);
  } else {
    project(nullptr, b, a);
  }
  if (mode == CGP_X0_POD_GALERKIN) {
    hipLaunchKernelGGL(k_small_matvec, dim3(1), dim3(64), 0, s, nm, (const double *)g->d_kinv, (const double *)a, c);
  } else {
    hipLaunchKernelGGL(k_feat_in, dim3(1), dim3(64), 0, s, nm, (const double *)a, mu_a, sd_a, g->d_xb);
    forward(g, s, 1);
    hipLaunchKernelGGL(k_feat_out, dim3(1), dim3(64), 0, s, nm, (const float *)g->d_y, mu_c, sd_c, c);
  }
  hipLaunchKernelGGL(k_expand, dim3(kExpandGrid), dim3(256), 0, s, n, nm, (const double *)g->d_phi, (const double *)c,
                     from_residual ? (const double *)x : (const double *)nullptr, x);
  CGP_HIP(hipGetLastError());
  return CGP_OK;
}

cgp_status guess_record(cgp_mesh *m, const double *x) {
  cgp_guess *g = m->guess;
  if (!g || g->win <= 0) return CGP_OK;
  cgp_status st = pod_finish(g);  // a rebuild still reading the window ends before a slot is replaced
  if (st) return st;
  CGP_HIP(hipMemcpyAsync(g->d_ring + (size_t)g->head * g->n, x, sizeof(double) * g->n, hipMemcpyDeviceToDevice,
                         m->stream));
  g->head = (g->head + 1) % g->win;
  g->filled = std::min(g->filled + 1, g->win);
  g->recorded++;
  if (g->filled >= g->nm && g->recorded % g->refresh == 0) {
    // the basis of the newest window (slot order does not matter to the POD), built on the guess's
    // own stream: the Gram matrix now, the rest as the solvers poll and at the next guess
    CGP_HIP(hipEventRecord(g->ev_in, m->stream));
    CGP_HIP(hipStreamWaitEvent(g->side, g->ev_in, 0));
    st = pod_stage_gram(g, g->side, g->d_ring, g->filled);
    if (st) return st;
    g->stage = 1;
  }
  return CGP_OK;
}

}  // namespace cgp

using namespace cgp;

extern "C" {

cgp_status cgp_guess_set_online(cgp_guess *g, int32_t window, int32_t refresh) {
  if (!g || window < 0 || (window > 0 && (window < g->nm || window > 1024 || refresh < 1))) {
    set_error("cgp_guess_set_online: window must be 0 (off) or in n_modes..1024, refresh >= 1");
    return CGP_E_ARG;
  }
  cgp_status ps = pod_finish(g);
  if (ps) return ps;
  if (window > 0) {
    ps = pod_events(g);
    if (ps) return ps;
    if (!g->side && hipStreamCreateWithFlags(&g->side, hipStreamNonBlocking) != hipSuccess) {
      set_error("cgp_guess_set_online: stream creation failed");
      return CGP_E_DEVICE;
    }
  }
  if (window > g->ring_cap) {
    double *r = nullptr;
    cgp_status st = galloc(g, &r, (size_t)window * g->n);
    if (st) return st;
    g->d_ring = r;
    g->ring_cap = window;
  }
  g->win = window;
  g->refresh = std::max(1, refresh);
  g->head = g->filled = 0;
  g->recorded = 0;
  if (window > 0) g->pod_ready = false;  // the basis comes from the window from now on
  return CGP_OK;
}

cgp_status cgp_guess_create(cgp_mesh *m, const cgp_guess_desc *d, cgp_guess **out) {
  if (!m || !d || !out || m->host_only) {
    set_error("cgp_guess_create: null argument or host-only mesh");
    return CGP_E_ARG;
  }
  if (d->n_modes < 1 || d->n_modes > 64 || d->hidden < 16 || d->hidden > 1024) {
    set_error("cgp_guess_create: n_modes must be in 1..64 and hidden in 16..1024");
    return CGP_E_ARG;
  }
  cgp_guess *g = new cgp_guess();
  g->mesh = m;
  g->nm = d->n_modes;
  g->nh = d->hidden;
  g->n = m->pc.n;
  g->seed = d->seed;
  const Layout L = layout(g);
  g->nparams = L.total;
  const int B = kMaxBatch, nm = g->nm, nh = g->nh;
  auto fail = [&](cgp_status st) {
    std::string msg = cgp_last_error();
    cgp_guess_destroy(g);
    set_error(msg);
    return st;
  };
  cgp_status st;
  if ((st = galloc(g, &g->d_phi, (size_t)g->n * nm)) || (st = galloc(g, &g->d_kinv, (size_t)nm * nm)) ||
      (st = galloc(g, &g->d_w, L.total)) || (st = galloc(g, &g->d_g, L.total)) || (st = galloc(g, &g->d_m, L.total)) ||
      (st = galloc(g, &g->d_v, L.total)) || (st = galloc(g, &g->d_wb, L.total)) ||
      (st = galloc(g, &g->d_stats, 4 * (size_t)nm)) || (st = galloc(g, &g->d_xb, (size_t)B * nm)) ||
      (st = galloc(g, &g->d_h1b, (size_t)B * nh)) || (st = galloc(g, &g->d_h2b, (size_t)B * nh)) ||
      (st = galloc(g, &g->d_dyb, (size_t)B * nm)) || (st = galloc(g, &g->d_dz2b, (size_t)B * nh)) ||
      (st = galloc(g, &g->d_dz1b, (size_t)B * nh)) || (st = galloc(g, &g->d_z1, (size_t)B * nh)) ||
      (st = galloc(g, &g->d_z2, (size_t)B * nh)) || (st = galloc(g, &g->d_y, (size_t)B * nm)) ||
      (st = galloc(g, &g->d_t, (size_t)B * nm)) || (st = galloc(g, &g->d_dy, (size_t)B * nm)) ||
      (st = galloc(g, &g->d_dh2, (size_t)B * nh)) || (st = galloc(g, &g->d_dz2, (size_t)B * nh)) ||
      (st = galloc(g, &g->d_dh1, (size_t)B * nh)) || (st = galloc(g, &g->d_dz1, (size_t)B * nh)) ||
      (st = galloc(g, &g->d_part, (size_t)64 * kProjectGrid)) || (st = galloc(g, &g->d_scal, 256)) ||
      (st = galloc(g, &g->d_idx, 65536)))
    return fail(st);
  // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) initialisation from a SplitMix64 stream
  std::vector<float> w(L.total);
  uint64_t state = d->seed;
  auto fill = [&](long off, long count, int fan_in) {
    const double bound = 1.0 / std::sqrt((double)fan_in);
    for (long i = 0; i < count; i++) w[off + i] = (float)((2.0 * uniform01(state) - 1.0) * bound);
  };
  fill(L.w1, (long)nh * nm, nm);
  fill(L.b1, nh, nm);
  fill(L.w2, (long)nh * nh, nh);
  fill(L.b2, nh, nh);
  fill(L.w3, (long)nm * nh, nh);
  fill(L.b3, nm, nh);
  if ((st = cgp_guess_set_params(g, w.data(), w.size()))) return fail(st);
  *out = g;
  return CGP_OK;
}

void cgp_guess_destroy(cgp_guess *g) {
  if (!g) return;
  if (g->mesh && g->mesh->guess == g) g->mesh->guess = nullptr;
  (void)hipDeviceSynchronize();
  for (void *p : g->allocations) (void)hipFree(p);
  if (g->h_pin) (void)hipHostFree(g->h_pin);
  for (hipEvent_t e : {g->ev_in, g->ev_gram, g->ev_basis, g->ev_done})
    if (e) (void)hipEventDestroy(e);
  if (g->side) (void)hipStreamDestroy(g->side);
  delete g;
}

cgp_status cgp_guess_set_params(cgp_guess *g, const float *host, size_t count) {
  if (!g || !host || (long)count != g->nparams) {
    set_error("cgp_guess_set_params: bad argument or size");
    return CGP_E_ARG;
  }
  hipStream_t s = g->mesh->stream;
  CGP_HIP(hipMemcpyAsync(g->d_w, host, count * sizeof(float), hipMemcpyHostToDevice, s));
  CGP_HIP(hipMemsetAsync(g->d_m, 0, count * sizeof(float), s));
  CGP_HIP(hipMemsetAsync(g->d_v, 0, count * sizeof(float), s));
  hipLaunchKernelGGL(k_to_bf16, dim3((count + 255) / 256), dim3(256), 0, s, (int)count, (const float *)g->d_w, g->d_wb);
  CGP_HIP(hipStreamSynchronize(s));
  g->adam_t = 0;
  return CGP_OK;
}

cgp_status cgp_guess_get_params(const cgp_guess *g, float *host, size_t count) {
  if (!g || !host || (long)count != g->nparams) {
    set_error("cgp_guess_get_params: bad argument or size");
    return CGP_E_ARG;
  }
  CGP_HIP(hipStreamSynchronize(g->mesh->stream));
  CGP_HIP(hipMemcpy(host, g->d_w, count * sizeof(float), hipMemcpyDeviceToHost));
  return CGP_OK;
}

cgp_status cgp_guess_export_basis(const cgp_guess *g, double *host, size_t count) {
  if (!g || !host || count != (size_t)g->n * g->nm || !g->pod_ready) {
    set_error("cgp_guess_export_basis: bad argument, size, or no basis yet");
    return CGP_E_ARG;
  }
  CGP_HIP(hipStreamSynchronize(g->mesh->stream));
  CGP_HIP(hipMemcpy(host, g->d_phi, count * sizeof(double), hipMemcpyDeviceToHost));
  return CGP_OK;
}

cgp_status cgp_guess_export_norm(const cgp_guess *g, double *host, size_t count) {
  if (!g || !host || count != 4 * (size_t)g->nm) {
    set_error("cgp_guess_export_norm: bad argument or size");
    return CGP_E_ARG;
  }
  if (!g->trained) {
    set_error("cgp_guess_export_norm: the model has not been trained");
    return CGP_E_STATE;
  }
  const int nm = g->nm;
  std::copy(g->mu_a.begin(), g->mu_a.end(), host);
  std::copy(g->sd_a.begin(), g->sd_a.end(), host + nm);
  std::copy(g->mu_c.begin(), g->mu_c.end(), host + 2 * nm);
  std::copy(g->sd_c.begin(), g->sd_c.end(), host + 3 * nm);
  return CGP_OK;
}

}  // extern "C"

namespace cgp {
namespace {

// ---- the POD build in three stages on a stream `st` (the mesh's stream for an explicit build, the
// guess's own stream for an online rebuild).  Pinned staging: [Gram S*S | Vs S*nm | Phi^T K Phi nm*nm |
// inverse nm*nm].

// stage 1: Gram matrix G = S M S^T (FP64, device) copied to the host; event ev_gram
cgp_status pod_stage_gram(cgp_guess *g, hipStream_t st, const double *snaps, int S) {
  const int n = g->n, nm = g->nm;
  double *hp = nullptr;
  GTRY(pinned(g, (size_t)S * S + (size_t)S * nm + 2 * (size_t)nm * nm, &hp));
  double *dG = nullptr;
  GTRY(scratch(g, 0, (size_t)S * S, &dG));
  GTRY(gemm64(g, st, S, S, n, snaps, n, 1, g->mesh->d_mc, snaps, 1, n, dG));
  CGP_HIP(hipMemcpyAsync(hp, dG, sizeof(double) * S * S, hipMemcpyDeviceToHost, st));
  CGP_HIP(hipEventRecord(g->ev_gram, st));
  g->pend_snaps = snaps;
  g->pend_S = S;
  return CGP_OK;
}

// stage 2 (host, once the Gram matrix is there): top nm eigenpairs, Vs = V Lambda^-1/2 to the device,
// Phi = S^T Vs, K Phi and Phi^T K Phi, the latter to the host; event ev_basis
cgp_status pod_stage_basis(cgp_guess *g, hipStream_t st) {
  cgp_mesh *m = g->mesh;
  const int n = g->n, nm = g->nm, S = g->pend_S;
  const double *snaps = g->pend_snaps;
  CGP_HIP(hipEventSynchronize(g->ev_gram));
  double *hG = g->h_pin, *hV = hG + (size_t)S * S, *hK = hV + (size_t)S * nm;
  std::vector<double> G(hG, hG + (size_t)S * S);
  // randomised subspace iteration for the nm largest eigenpairs (Halko, Martinsson & Tropp 2011);
  // when the oversampled subspace is the whole snapshot space, G itself is decomposed
  const int q = std::min(S, nm + 16);
  std::vector<double> Y((size_t)S * q), Z((size_t)S * q);
  std::vector<double> Bm((size_t)q * q, 0.0), U;
  if (q == S) {
    for (int a = 0; a < S; a++) Y[(size_t)a * q + a] = 1.0;
    Bm = G;
  } else {
    uint64_t state = g->seed ^ 0xA5A5A5A5ull;
    for (auto &v : Y) v = 2.0 * uniform01(state) - 1.0;
    auto mult = [&](const std::vector<double> &X, std::vector<double> &out) {  // out = G X
      std::fill(out.begin(), out.end(), 0.0);
      for (int a = 0; a < S; a++)
        for (int b = 0; b < S; b++) {
          const double gab = G[(size_t)a * S + b];
          const double *xb = &X[(size_t)b * q];
          double *oa = &out[(size_t)a * q];
          for (int j = 0; j < q; j++) oa[j] += gab * xb[j];
        }
    };
    orthonormalise(S, q, Y);
    for (int it = 0; it < 6; it++) {
      mult(Y, Z);
      Y.swap(Z);
      orthonormalise(S, q, Y);
    }
    mult(Y, Z);  // Z = G Q
    for (int i = 0; i < q; i++)
      for (int j = 0; j < q; j++) {
        double d = 0.0;
        for (int a = 0; a < S; a++) d += Y[(size_t)a * q + i] * Z[(size_t)a * q + j];
        Bm[(size_t)i * q + j] = d;
      }
  }
  for (int i = 0; i < q; i++)  // symmetrise
    for (int j = i + 1; j < q; j++) Bm[(size_t)i * q + j] = Bm[(size_t)j * q + i] = 0.5 * (Bm[(size_t)i * q + j] + Bm[(size_t)j * q + i]);
  if (!sym_eigen(q, Bm, U)) {
    set_error("cgp_guess_build_pod: the eigen-decomposition of the snapshot Gram matrix did not converge");
    return CGP_E_NOCONV;
  }
  std::vector<int> order(q);
  for (int i = 0; i < q; i++) order[i] = i;
  // by magnitude: the Gram matrix is semi-definite, and an eigenvalue computed below zero is one at the
  // rounding level whose sign the decomposition does not resolve
  std::sort(order.begin(), order.end(),
            [&](int a, int b) { return std::fabs(Bm[(size_t)a * q + a]) > std::fabs(Bm[(size_t)b * q + b]); });
  // modes with an eigenvalue below 1e-20 of the largest in magnitude are left out: their basis columns
  // are zero and the guesses ignore them.  Small eigenvalues stay, also those at the rounding level of
  // the largest: their modes carry the slowly converging components the Krylov solver left in the
  // snapshots, which is what a Galerkin initial guess removes best, and each is scaled by 1/sqrt|lambda|
  // (the Galerkin guess does not depend on the scaling of a basis column).
  std::vector<double> Vs((size_t)S * nm, 0.0);
  g->energy.assign(nm, 0.0);
  const double lam0 = Bm[(size_t)order[0] * q + order[0]];
  if (!(lam0 > 0.0) || !std::isfinite(lam0)) {
    set_error("cgp_guess_build_pod: the snapshots are zero or not finite");
    return CGP_E_ARG;
  }
  int rank = 0;
  for (int k = 0; k < nm; k++) {
    const int c = order[k];
    const double lam = std::fabs(Bm[(size_t)c * q + c]);
    if (!(lam > 1e-20 * lam0)) break;
    rank = k + 1;
    g->energy[k] = lam;
    const double inv = 1.0 / std::sqrt(lam);
    for (int a = 0; a < S; a++) {
      double v = 0.0;
      for (int j = 0; j < q; j++) v += Y[(size_t)a * q + j] * U[(size_t)j * q + c];
      Vs[(size_t)a * nm + k] = v * inv;
    }
  }
  g->rank = rank;
  // Phi = S^T Vs  ([n][nm])
  double *dV = nullptr;
  GTRY(scratch(g, 1, Vs.size(), &dV));
  std::copy(Vs.begin(), Vs.end(), hV);
  CGP_HIP(hipMemcpyAsync(dV, hV, sizeof(double) * Vs.size(), hipMemcpyHostToDevice, st));
  GTRY(gemm64(g, st, n, nm, S, snaps, 1, n, nullptr, dV, nm, 1, g->d_phi));
  // Phi^T K Phi (POD-Galerkin guess) to the host
  double *dKP = nullptr, *dPKP = nullptr;
  GTRY(scratch(g, 2, (size_t)n * nm, &dKP));
  GTRY(scratch(g, 3, (size_t)nm * nm, &dPKP));
  {
    const int rpw = nm <= 16 ? 4 : (nm <= 32 ? 2 : 1);
    const dim3 grid((unsigned)std::min<long>(65535, ((long)n + 4 * rpw - 1) / (4 * rpw)));
    if (rpw == 4)
      hipLaunchKernelGGL((k_spmm_modes<16>), grid, dim3(256), 0, st, n, nm, m->d_rp_c, m->d_col_c,
                         (const double *)m->d_Kbc, (const double *)g->d_phi, dKP);
    else if (rpw == 2)
      hipLaunchKernelGGL((k_spmm_modes<32>), grid, dim3(256), 0, st, n, nm, m->d_rp_c, m->d_col_c,
                         (const double *)m->d_Kbc, (const double *)g->d_phi, dKP);
    else
      hipLaunchKernelGGL((k_spmm_modes<64>), grid, dim3(256), 0, st, n, nm, m->d_rp_c, m->d_col_c,
                         (const double *)m->d_Kbc, (const double *)g->d_phi, dKP);
  }
  GTRY(gemm64(g, st, nm, nm, n, g->d_phi, 1, nm, nullptr, dKP, nm, 1, dPKP));
  CGP_HIP(hipMemcpyAsync(hK, dPKP, sizeof(double) * nm * nm, hipMemcpyDeviceToHost, st));
  CGP_HIP(hipEventRecord(g->ev_basis, st));
  return CGP_OK;
}

// stage 3 (host, once Phi^T K Phi is there): its inverse to the device; the mesh's stream waits for st
cgp_status pod_stage_inverse(cgp_guess *g, hipStream_t st) {
  const int nm = g->nm, S = g->pend_S, rank = g->rank;
  CGP_HIP(hipEventSynchronize(g->ev_basis));
  double *hK = g->h_pin + (size_t)S * S + (size_t)S * nm, *hI = hK + (size_t)nm * nm;
  std::vector<double> Kc(hK, hK + (size_t)nm * nm);
  // inverse of the leading rank x rank block by Gauss-Jordan with partial pivoting (SPD and tiny);
  // rows and columns of the unused modes stay zero.  A pivot at the rounding level of the largest
  // diagonal entry means that some modes are linearly dependent (snapshots that span fewer directions
  // than modes were kept): then the inverse is taken over an independent subset instead.
  double dmax = 0.0;
  for (int i = 0; i < rank; i++) dmax = std::max(dmax, std::fabs(Kc[(size_t)i * nm + i]));
  std::vector<double> inv((size_t)nm * nm, 0.0);
  for (int i = 0; i < rank; i++) inv[(size_t)i * nm + i] = 1.0;
  for (int col = 0; col < rank; col++) {
    int piv = col;
    for (int r = col + 1; r < rank; r++)
      if (std::fabs(Kc[(size_t)r * nm + col]) > std::fabs(Kc[(size_t)piv * nm + col])) piv = r;
    if (!(std::fabs(Kc[(size_t)piv * nm + col]) > 1e-13 * dmax)) {
      if (!independent_inverse(nm, rank, hK, inv)) {
        set_error("cgp_guess_build_pod: Phi^T K Phi has no positive diagonal entry");
        return CGP_E_ARG;
      }
      break;
    }
    for (int k = 0; k < rank; k++) {
      std::swap(Kc[(size_t)col * nm + k], Kc[(size_t)piv * nm + k]);
      std::swap(inv[(size_t)col * nm + k], inv[(size_t)piv * nm + k]);
    }
    const double d = Kc[(size_t)col * nm + col];
    for (int k = 0; k < rank; k++) {
      Kc[(size_t)col * nm + k] /= d;
      inv[(size_t)col * nm + k] /= d;
    }
    for (int r = 0; r < rank; r++) {
      if (r == col) continue;
      const double f = Kc[(size_t)r * nm + col];
      if (f == 0.0) continue;
      for (int k = 0; k < rank; k++) {
        Kc[(size_t)r * nm + k] -= f * Kc[(size_t)col * nm + k];
        inv[(size_t)r * nm + k] -= f * inv[(size_t)col * nm + k];
      }
    }
  }
  // the staging stays untouched until the next build's first synchronisation, after this copy
  std::copy(inv.begin(), inv.end(), hI);
  CGP_HIP(hipMemcpyAsync(g->d_kinv, hI, sizeof(double) * inv.size(), hipMemcpyHostToDevice, st));
  if (st != g->mesh->stream) {
    CGP_HIP(hipEventRecord(g->ev_done, st));
    CGP_HIP(hipStreamWaitEvent(g->mesh->stream, g->ev_done, 0));
  }
  g->pod_ready = true;
  g->trained = false;
  return CGP_OK;
}

cgp_status pod_events(cgp_guess *g) {
  if (g->ev_gram) return CGP_OK;
  for (hipEvent_t *e : {&g->ev_in, &g->ev_gram, &g->ev_basis, &g->ev_done})
    CGP_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  return CGP_OK;
}

// finish an online rebuild in progress (blocking); an error from a stage run inside a solver's poll is
// reported here
cgp_status pod_finish(cgp_guess *g) {
  if (g->stage_err) {
    const cgp_status e = g->stage_err;
    g->stage_err = CGP_OK;
    g->stage = 0;
    set_error(g->stage_msg);
    return e;
  }
  if (g->stage == 1) {
    cgp_status st = pod_stage_basis(g, g->side);
    if (st) {
      g->stage = 0;
      return st;
    }
    g->stage = 2;
  }
  if (g->stage == 2) {
    g->stage = 0;
    return pod_stage_inverse(g, g->side);
  }
  return CGP_OK;
}

}  // namespace

void guess_progress(cgp_mesh *m) {
  cgp_guess *g = m->guess;
  if (!g || (g->stage != 1 && g->stage != 2) || g->stage_err) return;
  const bool clean = hipPeekAtLastError() == hipSuccess;
  // the stage's input not there yet: a later poll or the next guess ("not ready" is no error of the
  // caller's launches)
  if (hipEventQuery(g->stage == 1 ? g->ev_gram : g->ev_basis) != hipSuccess) {
    if (clean) (void)hipGetLastError();
    return;
  }
  // stage 1 -> 2: eigen-decomposition and basis; stage 2 -> done: the inverse of Phi^T K Phi (the
  // mesh's stream then waits for its upload, so every later guess sees the new basis whole)
  const cgp_status st = g->stage == 1 ? pod_stage_basis(g, g->side) : pod_stage_inverse(g, g->side);
  if (st) {
    g->stage_err = st;
    g->stage_msg = cgp_last_error();
    return;
  }
  g->stage = g->stage == 1 ? 2 : 0;
}

}  // namespace cgp

extern "C" {

cgp_status cgp_guess_build_pod(cgp_guess *g, const double *snaps, int32_t S, double *energy) {
  if (!g || !snaps || S < g->nm) {
    set_error("cgp_guess_build_pod: need at least n_modes snapshots");
    return CGP_E_ARG;
  }
  GTRY(pod_events(g));
  GTRY(pod_finish(g));
  hipStream_t s = g->mesh->stream;
  GTRY(pod_stage_gram(g, s, snaps, S));
  GTRY(pod_stage_basis(g, s));
  if (energy) std::copy(g->energy.begin(), g->energy.end(), energy);
  return pod_stage_inverse(g, s);
}

cgp_status cgp_guess_train(cgp_guess *g, const double *rhs, const double *p, int32_t S, const cgp_train_opts *o,
                           cgp_train_stats *stats) {
  if (g) GTRY(pod_finish(g));
  if (!g || !rhs || !p || !o || S < 2 || S > 65536 || !g->pod_ready || o->batch < 1 || o->batch > kMaxBatch ||
      o->epochs < 1 || !(o->lr > 0)) {
    set_error("cgp_guess_train: bad argument (basis built? 2 <= S <= 65536, batch in 1..256, epochs >= 1, lr > 0)");
    return CGP_E_ARG;
  }
  cgp_mesh *m = g->mesh;
  hipStream_t s = m->stream;
  const int n = g->n, nm = g->nm;
  const bool incr = o->p_prev != nullptr;
  hipEvent_t e0, e1;
  CGP_HIP(hipEventCreate(&e0));
  CGP_HIP(hipEventCreate(&e1));
  CGP_HIP(hipEventRecord(e0, s));
  // modal coefficients Phi^T M p of every pressure ([S][nm], FP64) and, for the incremental model,
  // of every previous pressure; features Phi^T b, or Phi^T (b - K p_prev) for the incremental model
  double *dA = nullptr, *dC = nullptr, *dCp = nullptr, *dR = nullptr;
  const int NS = S;
  CGP_HIP(hipMallocAsync((void **)&dA, sizeof(double) * (size_t)S * nm, s));
  CGP_HIP(hipMallocAsync((void **)&dC, sizeof(double) * (size_t)S * nm, s));
  GTRY(gemm64(g, s, S, nm, n, p, n, 1, m->d_mc, g->d_phi, nm, 1, dC));
  std::vector<double> A((size_t)S * nm), Cc((size_t)S * nm), Cprev;
  if (incr) {
    CGP_HIP(hipMallocAsync((void **)&dCp, sizeof(double) * (size_t)S * nm, s));
    GTRY(gemm64(g, s, S, nm, n, o->p_prev, n, 1, m->d_mc, g->d_phi, nm, 1, dCp));
    CGP_HIP(hipMallocAsync((void **)&dR, sizeof(double) * (size_t)S * n, s));
    hipLaunchKernelGGL(k_pair_residual, dim3((n + 255) / 256, S), dim3(256), 0, s, n, m->d_rp_c, m->d_col_c,
                       (const double *)m->d_Kbc, rhs, o->p_prev, dR);
    GTRY(gemm64(g, s, S, nm, n, dR, n, 1, nullptr, g->d_phi, nm, 1, dA));
    CGP_HIP(hipFreeAsync(dR, s));
    Cprev.resize((size_t)S * nm);
    CGP_HIP(hipMemcpyAsync(Cprev.data(), dCp, sizeof(double) * Cprev.size(), hipMemcpyDeviceToHost, s));
    CGP_HIP(hipFreeAsync(dCp, s));
  } else {
    GTRY(gemm64(g, s, S, nm, n, rhs, n, 1, nullptr, g->d_phi, nm, 1, dA));
  }
  CGP_HIP(hipMemcpyAsync(A.data(), dA, sizeof(double) * A.size(), hipMemcpyDeviceToHost, s));
  CGP_HIP(hipMemcpyAsync(Cc.data(), dC, sizeof(double) * Cc.size(), hipMemcpyDeviceToHost, s));
  CGP_HIP(hipFreeAsync(dA, s));
  CGP_HIP(hipFreeAsync(dC, s));
  CGP_HIP(hipStreamSynchronize(s));
  if (incr)
    for (size_t e = 0; e < Cc.size(); e++) Cc[e] -= Cprev[e];
  // features: z-scores per mode.  Targets: mean per mode, one common scale for all modes, so that the
  // loss weighs each mode by its share of the pressure's M-norm (Phi is M-orthonormal)
  g->mu_a.assign(nm, 0.0);
  g->sd_a.assign(nm, 0.0);
  g->mu_c.assign(nm, 0.0);
  g->sd_c.assign(nm, 0.0);
  double vc_all = 0.0;
  for (int k = 0; k < nm; k++) {
    double sa = 0, sc = 0;
    for (int r = 0; r < NS; r++) {
      sa += A[(size_t)r * nm + k];
      sc += Cc[(size_t)r * nm + k];
    }
    g->mu_a[k] = sa / NS;
    g->mu_c[k] = sc / NS;
    double va = 0, vc = 0;
    for (int r = 0; r < NS; r++) {
      va += (A[(size_t)r * nm + k] - g->mu_a[k]) * (A[(size_t)r * nm + k] - g->mu_a[k]);
      vc += (Cc[(size_t)r * nm + k] - g->mu_c[k]) * (Cc[(size_t)r * nm + k] - g->mu_c[k]);
    }
    g->sd_a[k] = va > 0 ? std::sqrt(va / NS) : 1.0;
    vc_all += vc / NS;
  }
  const double sd_common = vc_all > 0 ? std::sqrt(vc_all / nm) : 1.0;
  for (int k = 0; k < nm; k++) g->sd_c[k] = sd_common;
  std::vector<float> X((size_t)NS * nm), T((size_t)NS * nm);
  for (int r = 0; r < NS; r++)
    for (int k = 0; k < nm; k++) {
      X[(size_t)r * nm + k] = (float)((A[(size_t)r * nm + k] - g->mu_a[k]) / g->sd_a[k]);
      T[(size_t)r * nm + k] = (float)((Cc[(size_t)r * nm + k] - g->mu_c[k]) / g->sd_c[k]);
    }
  std::vector<double> stats4(4 * (size_t)nm);
  std::copy(g->mu_a.begin(), g->mu_a.end(), stats4.begin());
  std::copy(g->sd_a.begin(), g->sd_a.end(), stats4.begin() + nm);
  std::copy(g->mu_c.begin(), g->mu_c.end(), stats4.begin() + 2 * nm);
  std::copy(g->sd_c.begin(), g->sd_c.end(), stats4.begin() + 3 * nm);
  CGP_HIP(hipMemcpyAsync(g->d_stats, stats4.data(), sizeof(double) * stats4.size(), hipMemcpyHostToDevice, s));
  float *dX = nullptr, *dT = nullptr;
  CGP_HIP(hipMallocAsync((void **)&dX, sizeof(float) * X.size(), s));
  CGP_HIP(hipMallocAsync((void **)&dT, sizeof(float) * T.size(), s));
  CGP_HIP(hipMemcpyAsync(dX, X.data(), sizeof(float) * X.size(), hipMemcpyHostToDevice, s));
  CGP_HIP(hipMemcpyAsync(dT, T.data(), sizeof(float) * T.size(), hipMemcpyHostToDevice, s));
  // mini-batch Adam
  const int B = o->batch;
  const int nb = (NS + B - 1) / B;
  std::vector<int> idx(NS);
  for (int i = 0; i < NS; i++) idx[i] = i;
  uint64_t state = o->seed;
  const float b1 = (float)(o->beta1 > 0 ? o->beta1 : 0.9), b2 = (float)(o->beta2 > 0 ? o->beta2 : 0.999);
  const float eps = (float)(o->eps > 0 ? o->eps : 1e-8);
  double loss_first = 0, loss_last = 0;
  std::vector<double> epoch_loss(nb);
  int steps = 0;
  double *h_loss = nullptr;
  CGP_HIP(hipHostMalloc((void **)&h_loss, sizeof(double) * nb, hipHostMallocDefault));
  for (int ep = 0; ep < o->epochs; ep++) {
    for (int i = NS - 1; i > 0; i--) std::swap(idx[i], idx[(int)(splitmix(state) % (uint64_t)(i + 1))]);
    CGP_HIP(hipMemcpyAsync(g->d_idx, idx.data(), sizeof(int) * NS, hipMemcpyHostToDevice, s));
    for (int bi = 0; bi < nb; bi++) {
      const int rows = std::min(B, NS - bi * B);
      hipLaunchKernelGGL(k_gather_batch, dim3((rows * nm + 255) / 256), dim3(256), 0, s, rows, nm,
                         (const int *)g->d_idx + bi * B, (const float *)dX, (const float *)dT, g->d_xb, g->d_t);
      forward(g, s, rows);
      backward(g, s, rows);
      hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, 16, (const double *)g->d_part, g->d_scal + 192 + 0);
      CGP_HIP(hipMemcpyAsync(h_loss + bi, g->d_scal + 192, sizeof(double), hipMemcpyDeviceToHost, s));
      g->adam_t++;
      const float c1 = 1.0f - std::pow(b1, (float)g->adam_t), c2 = 1.0f - std::pow(b2, (float)g->adam_t);
      hipLaunchKernelGGL(k_adam, dim3((g->nparams + 255) / 256), dim3(256), 0, s, (int)g->nparams, g->d_w, g->d_wb,
                         (const float *)g->d_g, g->d_m, g->d_v, (float)o->lr, b1, b2, eps, c1, c2);
      CGP_HIP(hipStreamSynchronize(s));  // h_loss slot reuse
      epoch_loss[bi] = h_loss[bi] / double(rows * nm);
      steps++;
    }
    double mean = 0;
    for (int bi = 0; bi < nb; bi++) mean += epoch_loss[bi];
    mean /= nb;
    if (ep == 0) loss_first = mean;
    loss_last = mean;
  }
  CGP_HIP(hipHostFree(h_loss));
  CGP_HIP(hipFreeAsync(dX, s));
  CGP_HIP(hipFreeAsync(dT, s));
  CGP_HIP(hipEventRecord(e1, s));
  CGP_HIP(hipEventSynchronize(e1));
  float ms = 0;
  (void)hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  CGP_HIP(hipGetLastError());
  g->trained = true;
  g->incremental = incr;
  if (stats) {
    stats->loss_first = loss_first;
    stats->loss_last = loss_last;
    stats->steps = steps;
    stats->ms = ms;
  }
  return CGP_OK;
}

cgp_status cgp_guess_mlp_grad(cgp_guess *g, const float *x, const float *t, int32_t B, double *loss, float *y,
                              float *grad) {
  if (!g || !x || !t || B < 1 || B > kMaxBatch) {
    set_error("cgp_guess_mlp_grad: bad argument (batch in 1..256)");
    return CGP_E_ARG;
  }
  hipStream_t s = g->mesh->stream;
  const int nm = g->nm;
  std::vector<int> idx(B);
  for (int i = 0; i < B; i++) idx[i] = i;
  float *dX = nullptr, *dT = nullptr;
  CGP_HIP(hipMallocAsync((void **)&dX, sizeof(float) * B * nm, s));
  CGP_HIP(hipMallocAsync((void **)&dT, sizeof(float) * B * nm, s));
  CGP_HIP(hipMemcpyAsync(dX, x, sizeof(float) * B * nm, hipMemcpyHostToDevice, s));
  CGP_HIP(hipMemcpyAsync(dT, t, sizeof(float) * B * nm, hipMemcpyHostToDevice, s));
  CGP_HIP(hipMemcpyAsync(g->d_idx, idx.data(), sizeof(int) * B, hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_gather_batch, dim3((B * nm + 255) / 256), dim3(256), 0, s, B, nm, (const int *)g->d_idx,
                     (const float *)dX, (const float *)dT, g->d_xb, g->d_t);
  forward(g, s, B);
  backward(g, s, B);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, 16, (const double *)g->d_part, g->d_scal + 192);
  double sse = 0;
  CGP_HIP(hipMemcpyAsync(&sse, g->d_scal + 192, sizeof(double), hipMemcpyDeviceToHost, s));
  if (y) CGP_HIP(hipMemcpyAsync(y, g->d_y, sizeof(float) * B * nm, hipMemcpyDeviceToHost, s));
  if (grad) CGP_HIP(hipMemcpyAsync(grad, g->d_g, sizeof(float) * g->nparams, hipMemcpyDeviceToHost, s));
  CGP_HIP(hipFreeAsync(dX, s));
  CGP_HIP(hipFreeAsync(dT, s));
  CGP_HIP(hipStreamSynchronize(s));
  if (loss) *loss = sse / double(B * nm);
  return CGP_OK;
}

cgp_status cgp_guess_attach(cgp_mesh *m, cgp_guess *g) {
  if (!m || (g && g->mesh != m)) {
    set_error("cgp_guess_attach: the guess belongs to another mesh");
    return CGP_E_ARG;
  }
  m->guess = g;
  return CGP_OK;
}

cgp_status cgp_guess_predict(cgp_guess *g, int32_t mode, const double *b, double *x) {
  if (!g || !b || !x || mode < CGP_X0_LEARNED || mode > CGP_X0_POD_GALERKIN) {
    set_error("cgp_guess_predict: bad argument");
    return CGP_E_ARG;
  }
  cgp_guess *keep = g->mesh->guess;
  g->mesh->guess = g;
  cgp_status st = guess_initial(g->mesh, mode, b, x);
  g->mesh->guess = keep;
  return st;
}

cgp_status cgp_last_poisson_rhs(const cgp_mesh *m, double *dst) {
  if (!m || !dst || m->host_only) {
    set_error("cgp_last_poisson_rhs: bad argument");
    return CGP_E_ARG;
  }
  CGP_HIP(hipMemcpyAsync(dst, m->d_wc[0], sizeof(double) * m->pc.n, hipMemcpyDeviceToDevice, m->stream));
  return CGP_OK;
}

}  // extern "C"
