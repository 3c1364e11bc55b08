// Internal declarations of libcgp (host topology, device buffers, kernel launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cgp.h"

namespace cgp {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
#define CGP_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess) {                                                            \
      ::cgp::set_error(std::string(#call) + ": " + hipGetErrorString(e_));             \
      return (e_ == hipErrorOutOfMemory) ? CGP_E_OOM : CGP_E_DEVICE;                   \
    }                                                                                  \
  } while (0)

// ------------------------------------------------------------------ host topology
struct HostLevel {
  int n = 0, t = 0, nb = 0, ne = 0;
  std::vector<double> xy;     // [n][2]
  std::vector<int> tri;       // [t][3]
  std::vector<int> bedge;     // [nb][2]
  std::vector<int> bkind;     // [nb]
  std::vector<int> edge;      // [ne][2] sorted (min,max)
  std::vector<int> parent;    // [n - n_prev][2]
};

struct HostCSR {
  int n = 0, nnz = 0;
  std::vector<int> rp, col;
};

struct HostColouring {
  int ncol = 0;
  std::vector<int> colour;    // [t]
  std::vector<int> perm;      // elements sorted by (colour, id)
  std::vector<int> cptr;      // [ncol+1] ranges in perm
};

namespace topo {
cgp_status validate(int n, const double *xy, int t, const int *tri, int nb, const int *bedge, const int *bkind);
void edges(const HostLevel &L, std::vector<int> &edge);
void refine(const HostLevel &c, HostLevel &f);
void csr(int n, const std::vector<int> &tri, HostCSR &A);
void slots(const std::vector<int> &tri, const HostCSR &A, std::vector<int> &slot);
void colour(int n, const std::vector<int> &tri, HostColouring &C);
uint64_t priority(uint64_t t);
}  // namespace topo

// ------------------------------------------------------------------ device state
template <typename T>
struct DBuf {
  T *p = nullptr;
  size_t n = 0;
};

// scalars of a Krylov solve kept in device memory.  Scalars that a later
// kernel of the same loop reads are kept per iteration parity ([it & 1]).
struct KrylovState {
  double tol;
  int maxit, ncomp;
  double bnorm[2], rnorm[2];
  double rz[2][2];                  // PCG r.z
  double rho[2][2], alpha[2][2], omega[2][2];  // BiCGStab
  int done[2];                      // component converged (or zero right-hand side)
  int zero_b[2];
  int iters;                        // completed iterations
  int status;                       // 0, or CGP_E_NONFINITE / CGP_E_NOCONV / CGP_E_DEVICE
};

// A captured run of kCg1GraphChunk fused PCG iterations: gx[0] starts at iteration 0, gx[1] at
// iteration kCg1GraphChunk (replayed at every later even iteration); key = the launches' arguments.
constexpr int kCg1GraphChunk = 8;
struct Cg1Graph {
  static constexpr int kKey = 14;
  uintptr_t key[kKey] = {};
  hipGraphExec_t gx[2] = {nullptr, nullptr};
};

// ILU(0)-GMRES(m) of the coarse Poisson solve: level schedule (pattern only), factors, Krylov basis
struct GmresState {
  bool ready = false;              // levels and buffers set up
  bool factored = false;           // d_lu holds ILU(0) of the current Kbar (cleared by cgp_assemble)
  int cap = 0;                     // restart length the basis holds
  std::vector<int> lptr, uptr;     // level pointers of the forward / backward substitution
  int *d_diag = nullptr, *d_lrows = nullptr, *d_urows = nullptr;
  double *d_lu = nullptr, *d_V = nullptr, *d_work = nullptr, *d_part = nullptr, *d_h = nullptr;
};

struct ReduceScratch {
  double *partials = nullptr;   // 4 regions of [8][red_grid] block partials
};

}  // namespace cgp

struct cgp_guess;

struct cgp_mesh {
  hipStream_t stream = nullptr;
  bool host_only = false;
  int levels = 0;
  std::vector<cgp::HostLevel> lev;
  cgp::HostCSR pf, pc;
  std::vector<int> slot_f, slot_c;             // original element order
  cgp::HostColouring col_f, col_c;
  std::vector<int> vdir, pdir;                 // masks
  int n_pdir = 0;
  std::vector<std::vector<int>> rt_ptr, rt_idx; // per level k>=1: coarse node -> midpoints (Galerkin restriction)
  bool assembled = false;
  cgp_params params{};
  cgp_guess *guess = nullptr;                  // learned initial guess attached to the Poisson solve

  // device topology
  double *d_xy_f = nullptr, *d_xy_c = nullptr;
  int *d_tri_f = nullptr, *d_slot_f = nullptr;      // permuted by colour
  int *d_inc_ptr_f = nullptr, *d_incv_f = nullptr;  // fine node -> vertex triples {v0, v1, v2, 0} of its elements
  int *d_tri_c = nullptr, *d_slot_c = nullptr;
  int *d_rp_f = nullptr, *d_col_f = nullptr, *d_rp_c = nullptr, *d_col_c = nullptr;
  unsigned char *d_vdir = nullptr, *d_pdir = nullptr;
  std::vector<int *> d_parent;                      // per level k>=1
  std::vector<int *> d_rt_ptr, d_rt_idx;            // per level k>=1
  // device operators
  double *d_S = nullptr, *d_M = nullptr, *d_D = nullptr, *d_Mbc = nullptr, *d_dinvM = nullptr, *d_ml = nullptr;
  double *d_A = nullptr, *d_dinvA = nullptr;
  float *d_A32 = nullptr, *d_dinvA32 = nullptr;  // FP32 momentum matrix and Jacobi inverse (first FP32-refined solve)
  float2 *d_wf32 = nullptr;                      // 7 fine FP32 2-vectors of the inner BiCGStab (same)
  double *d_K = nullptr, *d_Kbc = nullptr, *d_Dc = nullptr, *d_mc = nullptr, *d_dinvK = nullptr;
  float *d_Kbc32 = nullptr, *d_dinvK32 = nullptr;
  double mc_sum = 0.0;
  // work vectors: fine [n_f][2], coarse [n_c]
  std::vector<double *> d_wf;     // 8 fine 2-vectors
  std::vector<double *> d_wc;     // 8 coarse vectors
  std::vector<float *> d_wc32;    // 6 coarse float vectors
  std::vector<double *> d_wlev;   // per level scratch [n_k] (prolong/restrict chains)
  double *d_ut = nullptr;         // u-tilde [n_f][2] for cgp_step
  double *d_ut_prev = nullptr;    // the step before's u-tilde (extrapolated momentum guess)
  double *d_ut_prev2 = nullptr;   // and the one before that
  int ut_hist = 0;                // consecutive cgp_step momentum solves kept in d_ut / d_ut_prev / d_ut_prev2
  double *d_uhist = nullptr;      // [n_f][8] double2 ring of momentum solutions (projected guess; on first use)
  double *d_mdelta = nullptr;     // [n_f][2] last consistent-minus-lumped correction (mass x0 EXTRAP; first use)
  bool mdelta_ok = false;         // d_mdelta holds the previous cgp_step's difference
  double *d_proj = nullptr;       // projected guess: Gram block partials, coefficients [2][8], entry sums
  int uh_count = 0, uh_head = 0;  // filled ring slots (consecutive cgp_step solves) and the next slot to write
  double *d_rec = nullptr;        // 2 x [n_c] records {r, w, s, D^-1} of the fused Poisson PCG (double4 or float4)
  double *d_bc = nullptr;         // coarse rhs
  double *d_pfn = nullptr;        // incremental pressure modes: prolonged P^n [n_f], allocated on first use
  double *d_phi = nullptr;        //   the last pressure increment [n_c] (its solve's initial guess)
  double *d_phif = nullptr;       //   the prolonged increment [n_f]
  int n_surf = 0;                 // fine boundary edges of the marked surface (cgp_surface_set)
  int *d_surf = nullptr;          // their {a, b, third vertex, 0} (int4)
  int n_surf_cap = 0;             // rows d_surf holds
  cgp::KrylovState *d_state = nullptr;   // 5 solver states
  cgp::KrylovState *h_state = nullptr;   // pinned mirror
  cgp::ReduceScratch red;
  cgp::GmresState gm;
  int cu_count = 0;
  int device = -1;                // HIP device the mesh's buffers live on
  int red_grid = 0;               // blocks of every reducing kernel (one partial per block)
  int coop_blocks = 0;            // blocks of the persistent PCG (0: not set up)
  int coop_max = 0;               // co-resident blocks reported by the runtime
  int *d_row_begin = nullptr;     // row range per persistent block
  void *d_bar = nullptr;          // grid barrier
  double *d_ppartials = nullptr;  // persistent-kernel partials
  bool coop_ok = true;            // cooperative launch available (checked once)
  std::vector<void *> allocations;
  double *d_scalar = nullptr;     // device scalar for sums (means)
  double *h_scalar = nullptr;     // pinned [4]
  cgp_tuning tune{{4, 512, 4}, {2, 1024, 1}, 0, 0, 0, 0};  // Krylov launch shapes (fine, coarse), persistent kernel
  // captured chunks of the fused Poisson PCG (per argument set) and the stream they are captured on
  std::vector<cgp::Cg1Graph> cg1_graphs;
  hipStream_t cap_stream = nullptr;
  // Krylov iterations queued before the first poll of a solve (the last solve's count), per solve
  // kind; the FP32 inner solves keep one per refinement step, whose lengths differ
  int mom_chunk = 4, mom32_chunk = 4, p_chunk = 32, p32_chunk[4] = {16, 16, 16, 16}, mass_chunk = 8;
  int cheb_steps = 16;  // Chebyshev steps of the first cycle of a mass solve (the last solve's count)
  // HIP-event timing of every launch of the Poisson SpMV kernel (cgp_step_opts.timing == 2)
  hipEvent_t step_ev[7] = {};      // per-phase events of cgp_step (timing >= 1)
  bool kt_on = false;
  std::vector<hipEvent_t> kt_ev;   // event pairs
  std::vector<int> kt_iter;        // Krylov iteration of each pair
  int kt_used = 0;                 // pairs recorded since the last harvest
  double kt_ms = 0.0;
  long kt_count = 0;
  long kt_iters = 0;               // Krylov iterations covered by the timed launches
};
