// Learned initial guess for the coarse Poisson solve (POD basis + BF16 MFMA MLP).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "internal.h"

struct cgp_guess {
  cgp_mesh *mesh = nullptr;
  int nm = 64, nh = 256, n = 0;       // modes, hidden width, coarse nodes
  uint64_t seed = 0;
  bool pod_ready = false, trained = false, incremental = false;
  std::vector<void *> allocations;
  // basis
  double *d_phi = nullptr;            // [n][nm], M-orthonormal
  double *d_kinv = nullptr;           // [nm][nm] inverse of Phi^T K Phi (POD-Galerkin guess)
  std::vector<double> energy;         // POD eigenvalues (largest first; 0 for unused modes)
  int rank = 0;                       // modes in use (the rest of Phi is zero)
  // online basis: the pressures of the last `win` solves, the basis rebuilt every `refresh` solves
  double *d_ring = nullptr;           // [ring_cap][n]
  int ring_cap = 0, win = 0, refresh = 1, head = 0, filled = 0;
  long recorded = 0;
  // an online rebuild runs in stages on its own stream, overlapping the next step's momentum solve:
  // 0 idle, 1 Gram matrix queued, 2 basis queued (the host finishes each stage when its event is done)
  int stage = 0;
  cgp_status stage_err = CGP_OK;
  std::string stage_msg;
  hipStream_t side = nullptr;
  hipEvent_t ev_in = nullptr, ev_gram = nullptr, ev_basis = nullptr, ev_done = nullptr;
  const double *pend_snaps = nullptr;  // snapshots of the rebuild in progress
  int pend_S = 0;
  // network: parameters [W1 nh*nm | b1 nh | W2 nh*nh | b2 nh | W3 nm*nh | b3 nm]
  long nparams = 0;
  float *d_w = nullptr, *d_g = nullptr, *d_m = nullptr, *d_v = nullptr;
  unsigned short *d_wb = nullptr;     // BF16 copy of the parameters
  long adam_t = 0;
  // normalisation of features (Phi^T b) and targets (Phi^T M p), host and device
  std::vector<double> mu_a, sd_a, mu_c, sd_c;
  double *d_stats = nullptr;          // [4][nm]: mu_a, sd_a, mu_c, sd_c
  // batch workspace (max batch kMaxBatch)
  unsigned short *d_xb = nullptr, *d_h1b = nullptr, *d_h2b = nullptr, *d_dyb = nullptr, *d_dz2b = nullptr,
                 *d_dz1b = nullptr;
  float *d_z1 = nullptr, *d_z2 = nullptr, *d_y = nullptr, *d_t = nullptr, *d_dy = nullptr, *d_dh2 = nullptr,
        *d_dz2 = nullptr, *d_dh1 = nullptr, *d_dz1 = nullptr;
  double *d_part = nullptr, *d_scal = nullptr;  // partials, small scalars/vectors
  double *scr[5] = {};                           // grown scratch (basis construction, split-K partials)
  size_t scr_cap[5] = {};
  double *h_pin = nullptr;                       // pinned staging
  size_t pin_cap = 0;
  int *d_idx = nullptr;
};

namespace cgp {
constexpr int kMaxBatch = 256;
// x0 for the Poisson solve from the right-hand side b (after boundary conditions):
// mode CGP_X0_LEARNED: x0 = Phi c (absolute model); CGP_X0_LEARNED_CORR: x0 = x + Phi dc with dc from
// the incremental model applied to Phi^T (b - K x);
// CGP_X0_POD_GALERKIN: x0 = x + Phi (Phi^T K Phi)^-1 Phi^T (b - K x).  x holds the previous pressure.
cgp_status guess_initial(cgp_mesh *m, int mode, const double *b, double *x);
// After a converged Poisson solve: keep x in the attached guess's window and start the refresh of its
// basis when due (completed by guess_progress or at the next guess_initial).
cgp_status guess_record(cgp_mesh *m, const double *x);
// Called by the solvers before they wait on the mesh's stream: moves a pending online rebuild on
// (host eigen-decomposition) when its Gram matrix is ready, without blocking.
void guess_progress(cgp_mesh *m);
}  // namespace cgp
