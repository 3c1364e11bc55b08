// Allocation-free coarse Poisson solve (cgp_poisson_solve_noalloc).
//
// The same FP64 Jacobi-PCG as cgp_poisson_solve with the fused one-kernel-per-iteration launch, for
// callers that cannot allocate device memory.  Everything that solve writes besides x (the copy of
// the right-hand side with its boundary conditions, the search direction, the two node-record slots
// {r, w, s, D^-1}, the per-block partial sums and the solver state) lives in one file-scope device
// array per GPU instead of the mesh's buffers.  Its device address is taken once per device, when
// the first device mesh is created there with that device current; the kernels receive that address,
// never the array's host-side name.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"
#include "kernels.h"

namespace cgp {
namespace noalloc {
constexpr long kRows = 1L << 18;  // largest coarse system the array serves
constexpr size_t up256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kOffB = 0;                                               // b with BCs [n]
constexpr size_t kOffP = kOffB + up256(kRows * sizeof(double));           // p [n]
constexpr size_t kOffRec = kOffP + up256(kRows * sizeof(double));         // 2 x [n] double4 records
constexpr size_t kOffPart = kOffRec + up256(2 * kRows * 4 * sizeof(double));
constexpr size_t kOffState = kOffPart + up256(size_t(4) * 8 * kMaxRedGrid * sizeof(double));
constexpr size_t kBytes = kOffState + up256(4 * sizeof(KrylovState));
constexpr int kMaxDevices = 64;
}  // namespace noalloc
}  // namespace cgp

// One copy per GPU, kept until the process ends (about 21 MB).
static __device__ __align__(256) unsigned char scratch[cgp::noalloc::kBytes];

namespace cgp {
namespace {
std::mutex g_mu;
void *g_scratch[noalloc::kMaxDevices] = {};  // device address of `scratch` on each device
}  // namespace

// With `device` current: look up the array's address on it (once per device).
cgp_status noalloc_setup(int device) {
  if (device < 0 || device >= noalloc::kMaxDevices) {
    set_error("noalloc_setup: device index out of range");
    return CGP_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return CGP_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    return CGP_E_DEVICE;
  }
  g_scratch[device] = p;
  return CGP_OK;
}

}  // namespace cgp

using namespace cgp;

extern "C" cgp_status cgp_poisson_solve_noalloc(cgp_mesh *m, const double *b, double *x, const cgp_solver_opts *o,
                                               cgp_stats *stats) {
  if (!m || !b || !x || !o) {
    set_error("cgp_poisson_solve_noalloc: null argument");
    return CGP_E_ARG;
  }
  if (m->host_only || !m->assembled) {
    set_error("cgp_poisson_solve_noalloc: needs an assembled device mesh");
    return CGP_E_STATE;
  }
  if (!(o->tol > 0.0) || o->max_iter < 1 || o->precision != CGP_PREC_FP64 ||
      (o->x0_mode != CGP_X0_ZERO && o->x0_mode != CGP_X0_PREV) ||
      (o->launch != CGP_LAUNCH_AUTO && o->launch != CGP_LAUNCH_FUSED) || o->method != CGP_METHOD_DEFAULT) {
    set_error("cgp_poisson_solve_noalloc: FP64, x0 zero or previous, fused launch only");
    return CGP_E_ARG;
  }
  if (m->pc.n > noalloc::kRows) {
    set_error("cgp_poisson_solve_noalloc: the coarse system has " + std::to_string(m->pc.n) +
              " rows, more than the " + std::to_string(noalloc::kRows) + " its device array serves");
    return CGP_E_ARG;
  }
  void *base = (m->device >= 0 && m->device < noalloc::kMaxDevices) ? g_scratch[m->device] : nullptr;
  if (!base) {
    set_error("cgp_poisson_solve_noalloc: no device array on this mesh's device");
    return CGP_E_STATE;
  }
  unsigned char *s = static_cast<unsigned char *>(base);
  // the solve's own buffers point into the array for this call; the mesh's are put back on every
  // return.  The attached guess is set aside: the call records no solution and starts no rebuild.
  // Graph capture is off for the call: instantiating a graph may allocate.
  struct Swap {
    cgp_mesh *m;
    double *wc0, *wc7, *rec, *part;
    KrylovState *state;
    cgp_guess *guess;
    int32_t graph;
    ~Swap() {
      m->d_wc[0] = wc0;
      m->d_wc[7] = wc7;
      m->d_rec = rec;
      m->red.partials = part;
      m->d_state = state;
      m->guess = guess;
      m->tune.pcg_graph = graph;
    }
  } keep{m, m->d_wc[0], m->d_wc[7], m->d_rec, m->red.partials, m->d_state, m->guess, m->tune.pcg_graph};
  m->tune.pcg_graph = 0;
  m->d_wc[0] = reinterpret_cast<double *>(s + noalloc::kOffB);
  m->d_wc[7] = reinterpret_cast<double *>(s + noalloc::kOffP);
  m->d_rec = reinterpret_cast<double *>(s + noalloc::kOffRec);
  m->red.partials = reinterpret_cast<double *>(s + noalloc::kOffPart);
  m->d_state = reinterpret_cast<KrylovState *>(s + noalloc::kOffState);
  m->guess = nullptr;
  cgp_solver_opts fused = *o;
  fused.launch = CGP_LAUNCH_FUSED;
  return drv_poisson(m, b, x, &fused, stats);
}
