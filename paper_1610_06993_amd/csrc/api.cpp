// C ABI of libcgp: argument checking, host topology build and upload, and the
// sequencing of the five IFE-CGP steps (Section 2.2, Eqs. 19-23).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <unordered_map>

#include "internal.h"
#include "kernels.h"

namespace cgp {
static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace cgp

using namespace cgp;

namespace {

template <typename T>
cgp_status dalloc(cgp_mesh *m, T **p, size_t count) {
  void *q = nullptr;
  hipError_t e = hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T));
  if (e != hipSuccess) {
    set_error(std::string("hipMalloc: ") + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? CGP_E_OOM : CGP_E_DEVICE;
  }
  m->allocations.push_back(q);
  *p = static_cast<T *>(q);
  return CGP_OK;
}

template <typename T>
cgp_status upload(cgp_mesh *m, T **p, const T *src, size_t count) {
  cgp_status s = dalloc(m, p, count);
  if (s) return s;
  if (count) CGP_HIP(hipMemcpyAsync(*p, src, count * sizeof(T), hipMemcpyHostToDevice, m->stream));
  return CGP_OK;
}

#define TRY(x)                  \
  do {                          \
    cgp_status s_ = (x);        \
    if (s_ != CGP_OK) return s_; \
  } while (0)

cgp_status build_device(cgp_mesh *m) {
  int dev = 0;
  CGP_HIP(hipGetDevice(&dev));
  CGP_HIP(hipDeviceGetAttribute(&m->cu_count, hipDeviceAttributeMultiprocessorCount, dev));
  m->device = dev;
  TRY(noalloc_setup(dev));
  const HostLevel &F = m->lev[m->levels], &C = m->lev[0];
  // element arrays permuted by colour (contiguous range per colour)
  auto permute = [](const std::vector<int> &a, int w, const std::vector<int> &perm) {
    std::vector<int> out(a.size());
    for (size_t i = 0; i < perm.size(); i++)
      std::memcpy(&out[i * w], &a[size_t(perm[i]) * w], sizeof(int) * w);
    return out;
  };
  std::vector<int> trif = permute(F.tri, 3, m->col_f.perm), slotf = permute(m->slot_f, 9, m->col_f.perm);
  std::vector<int> tric = permute(C.tri, 3, m->col_c.perm), slotc = permute(m->slot_c, 9, m->col_c.perm);
  std::vector<unsigned char> vd(m->vdir.begin(), m->vdir.end()), pd(m->pdir.begin(), m->pdir.end());
  TRY(upload(m, &m->d_xy_f, F.xy.data(), F.xy.size()));
  TRY(upload(m, &m->d_xy_c, C.xy.data(), C.xy.size()));
  TRY(upload(m, &m->d_tri_f, trif.data(), trif.size()));
  TRY(upload(m, &m->d_slot_f, slotf.data(), slotf.size()));
  {  // fine node i -> the vertex triples {v0, v1, v2, 0} of its elements, in element order, row after row
    const int nf = F.n, tf = F.t;
    std::vector<int> ptr(nf + 1, 0);
    for (int v : F.tri) ptr[v + 1]++;
    for (int i = 0; i < nf; i++) ptr[i + 1] += ptr[i];
    std::vector<int> pos(ptr.begin(), ptr.end() - 1), incv(4 * (size_t)ptr[nf]);
    for (int e = 0; e < tf; e++)
      for (int a = 0; a < 3; a++) {
        const size_t q = (size_t)pos[F.tri[3 * e + a]]++;
        for (int b = 0; b < 3; b++) incv[4 * q + b] = F.tri[3 * e + b];
        incv[4 * q + 3] = 0;
      }
    TRY(upload(m, &m->d_inc_ptr_f, ptr.data(), ptr.size()));
    TRY(upload(m, &m->d_incv_f, incv.data(), incv.size()));
  }
  TRY(upload(m, &m->d_tri_c, tric.data(), tric.size()));
  TRY(upload(m, &m->d_slot_c, slotc.data(), slotc.size()));
  TRY(upload(m, &m->d_rp_f, m->pf.rp.data(), m->pf.rp.size()));
  TRY(upload(m, &m->d_col_f, m->pf.col.data(), m->pf.col.size()));
  TRY(upload(m, &m->d_rp_c, m->pc.rp.data(), m->pc.rp.size()));
  TRY(upload(m, &m->d_col_c, m->pc.col.data(), m->pc.col.size()));
  TRY(upload(m, &m->d_vdir, vd.data(), vd.size()));
  TRY(upload(m, &m->d_pdir, pd.data(), pd.size()));
  m->d_parent.assign(m->levels + 1, nullptr);
  m->d_rt_ptr.assign(m->levels + 1, nullptr);
  m->d_rt_idx.assign(m->levels + 1, nullptr);
  for (int k = 1; k <= m->levels; k++) {
    TRY(upload(m, &m->d_parent[k], m->lev[k].parent.data(), m->lev[k].parent.size()));
    TRY(upload(m, &m->d_rt_ptr[k], m->rt_ptr[k].data(), m->rt_ptr[k].size()));
    TRY(upload(m, &m->d_rt_idx[k], m->rt_idx[k].data(), m->rt_idx[k].size()));
  }
  const size_t nf = m->pf.nnz, nc = m->pc.nnz, Nf = m->pf.n, Nc = m->pc.n;
  TRY(dalloc(m, &m->d_S, nf));
  TRY(dalloc(m, &m->d_M, nf));
  TRY(dalloc(m, &m->d_D, 2 * nf));
  TRY(dalloc(m, &m->d_Mbc, nf));
  TRY(dalloc(m, &m->d_dinvM, Nf));
  TRY(dalloc(m, &m->d_ml, Nf));
  TRY(dalloc(m, &m->d_A, nf));
  TRY(dalloc(m, &m->d_dinvA, Nf));
  TRY(dalloc(m, &m->d_K, nc));
  TRY(dalloc(m, &m->d_Kbc, nc));
  TRY(dalloc(m, &m->d_Dc, 2 * nc));
  TRY(dalloc(m, &m->d_mc, Nc));
  TRY(dalloc(m, &m->d_dinvK, Nc));
  TRY(dalloc(m, &m->d_Kbc32, nc));
  TRY(dalloc(m, &m->d_dinvK32, Nc));
  m->d_wf.assign(8, nullptr);
  for (auto &p : m->d_wf) TRY(dalloc(m, &p, 2 * Nf));
  m->d_wc.assign(8, nullptr);
  for (auto &p : m->d_wc) TRY(dalloc(m, &p, Nc));
  m->d_wc32.assign(8, nullptr);
  for (auto &p : m->d_wc32) TRY(dalloc(m, &p, Nc));
  m->d_wlev.assign(m->levels + 1, nullptr);
  for (int k = 0; k <= m->levels; k++) TRY(dalloc(m, &m->d_wlev[k], size_t(m->lev[k].n)));
  TRY(dalloc(m, &m->d_ut, 2 * Nf));
  TRY(dalloc(m, &m->d_ut_prev, 2 * Nf));
  TRY(dalloc(m, &m->d_ut_prev2, 2 * Nf));
  TRY(dalloc(m, &m->d_rec, 8 * Nc));
  TRY(dalloc(m, &m->d_bc, Nc));
  TRY(dalloc(m, &m->d_state, 5));
  m->red_grid = std::max(8, m->cu_count);
  TRY(dalloc(m, &m->red.partials, size_t(4) * 8 * kMaxRedGrid));
  TRY(dalloc(m, &m->d_scalar, 4));
  CGP_HIP(hipMemsetAsync(m->d_state, 0, 5 * sizeof(KrylovState), m->stream));
  CGP_HIP(hipHostMalloc((void **)&m->h_state, 5 * sizeof(KrylovState), hipHostMallocDefault));
  CGP_HIP(hipHostMalloc((void **)&m->h_scalar, 4 * sizeof(double), hipHostMallocDefault));
  CGP_HIP(hipStreamSynchronize(m->stream));
  return CGP_OK;
}

// poisson: the coarse Poisson solve; allow_extrap: the momentum solve of cgp_step (history-based
// guesses); allow_fp32: the momentum solve (FP32 inner BiCGStab inside FP64 refinement); mass: the
// velocity correction's mass solve (may use the Chebyshev iteration)
bool valid_opts(const cgp_solver_opts *o, bool poisson, bool allow_extrap = false, bool allow_fp32 = false,
                bool mass = false) {
  if (!o) return false;
  if (!(o->tol > 0.0) || o->max_iter < 1) return false;
  if (o->precision != CGP_PREC_FP64 && !((poisson || allow_fp32) && o->precision == CGP_PREC_FP32_IR)) return false;
  if (o->x0_mode < CGP_X0_ZERO || o->x0_mode > (poisson ? CGP_X0_POD_GALERKIN : CGP_X0_PREV)) {
    if (!(allow_extrap && !poisson && (o->x0_mode == CGP_X0_EXTRAP || o->x0_mode == CGP_X0_PROJECT))) return false;
  }
  if (o->launch < CGP_LAUNCH_AUTO || o->launch > CGP_LAUNCH_FUSED) return false;
  if (o->method != CGP_METHOD_DEFAULT &&
      !(poisson && o->method == CGP_METHOD_ILU_GMRES && o->precision == CGP_PREC_FP64) &&
      !(mass && o->method == CGP_METHOD_CHEBYSHEV))
    return false;
  if (o->restart < 0 || o->restart > 200) return false;
  return true;
}

cgp_status ready(const cgp_mesh *m) {
  if (!m) {
    set_error("null mesh");
    return CGP_E_ARG;
  }
  if (m->host_only) {
    set_error("mesh was created host-only");
    return CGP_E_STATE;
  }
  if (!m->assembled) {
    set_error("cgp_assemble has not been called");
    return CGP_E_STATE;
  }
  return CGP_OK;
}

}  // namespace

extern "C" {

int32_t cgp_abi_version(void) { return CGP_ABI_VERSION; }
const char *cgp_last_error(void) { return g_err.c_str(); }

cgp_status cgp_mesh_create(const cgp_mesh_desc *d, void *hip_stream, cgp_mesh **out) {
  if (!d || !out) {
    set_error("cgp_mesh_create: null argument");
    return CGP_E_ARG;
  }
  *out = nullptr;
  if (d->levels < 0 || d->levels > 6) {
    set_error("cgp_mesh_create: levels must be in [0, 6]");
    return CGP_E_ARG;
  }
  cgp_status vs = topo::validate(d->n_nodes, d->xy, d->n_tris, d->tri, d->n_bedges, d->bedge, d->bedge_kind);
  if (vs) return vs;
  cgp_mesh *m = new (std::nothrow) cgp_mesh();
  if (!m) return CGP_E_OOM;
  m->stream = static_cast<hipStream_t>(hip_stream);
  m->host_only = (d->flags & CGP_MESH_HOST_ONLY) != 0;
  m->levels = d->levels;
  m->lev.resize(d->levels + 1);
  HostLevel &L0 = m->lev[0];
  L0.n = d->n_nodes;
  L0.t = d->n_tris;
  L0.nb = d->n_bedges;
  L0.xy.assign(d->xy, d->xy + 2 * size_t(d->n_nodes));
  L0.tri.assign(d->tri, d->tri + 3 * size_t(d->n_tris));
  L0.bedge.assign(d->bedge, d->bedge + 2 * size_t(d->n_bedges));
  L0.bkind.assign(d->bedge_kind, d->bedge_kind + size_t(d->n_bedges));
  topo::edges(L0, L0.edge);
  L0.ne = int(L0.edge.size() / 2);
  for (int k = 0; k < d->levels; k++) topo::refine(m->lev[k], m->lev[k + 1]);
  const HostLevel &F = m->lev[d->levels];
  topo::csr(F.n, F.tri, m->pf);
  topo::csr(L0.n, L0.tri, m->pc);
  topo::slots(F.tri, m->pf, m->slot_f);
  topo::slots(L0.tri, m->pc, m->slot_c);
  topo::colour(F.n, F.tri, m->col_f);
  topo::colour(L0.n, L0.tri, m->col_c);
  m->vdir.assign(F.n, 0);
  for (int k = 0; k < F.nb; k++)
    if (F.bkind[k] == CGP_EDGE_VEL_DIRICHLET) m->vdir[F.bedge[2 * k]] = m->vdir[F.bedge[2 * k + 1]] = 1;
  m->pdir.assign(L0.n, 0);
  for (int k = 0; k < L0.nb; k++)
    if (L0.bkind[k] == CGP_EDGE_OUTFLOW) m->pdir[L0.bedge[2 * k]] = m->pdir[L0.bedge[2 * k + 1]] = 1;
  m->n_pdir = 0;
  for (int v : m->pdir) m->n_pdir += v;
  // transpose of the parent table per level (coarse node -> its midpoints, ascending)
  m->rt_ptr.assign(d->levels + 1, {});
  m->rt_idx.assign(d->levels + 1, {});
  for (int k = 1; k <= d->levels; k++) {
    const int np = m->lev[k - 1].n, nk = m->lev[k].n;
    std::vector<int> &ptr = m->rt_ptr[k], &idx = m->rt_idx[k];
    ptr.assign(np + 1, 0);
    for (int q = 0; q < nk - np; q++) {
      ptr[m->lev[k].parent[2 * q] + 1]++;
      ptr[m->lev[k].parent[2 * q + 1] + 1]++;
    }
    for (int i = 0; i < np; i++) ptr[i + 1] += ptr[i];
    idx.assign(ptr[np], 0);
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int q = 0; q < nk - np; q++) {
      idx[fill[m->lev[k].parent[2 * q]]++] = np + q;
      idx[fill[m->lev[k].parent[2 * q + 1]]++] = np + q;
    }
  }
  if (!m->host_only) {
    cgp_status s = build_device(m);
    if (s) {
      std::string keep = g_err;
      cgp_mesh_destroy(m);
      g_err = keep;
      return s;
    }
  }
  *out = m;
  return CGP_OK;
}

cgp_status cgp_mesh_query(const cgp_mesh *m, cgp_mesh_info *o) {
  if (!m || !o) {
    set_error("cgp_mesh_query: null argument");
    return CGP_E_ARG;
  }
  const HostLevel &F = m->lev[m->levels], &C = m->lev[0];
  o->n_f = F.n; o->t_f = F.t; o->n_c = C.n; o->t_c = C.t;
  o->nnz_f = m->pf.nnz; o->nnz_c = m->pc.nnz;
  o->ncol_f = m->col_f.ncol; o->ncol_c = m->col_c.ncol;
  o->nb_f = F.nb; o->nb_c = C.nb;
  o->levels = m->levels; o->n_pdir = m->n_pdir;
  return CGP_OK;
}

cgp_status cgp_mesh_export(const cgp_mesh *m, int32_t what, int32_t level, void *dst, size_t bytes) {
  if (!m || !dst) {
    set_error("cgp_mesh_export: null argument");
    return CGP_E_ARG;
  }
  if (level < 0 || level > m->levels) {
    set_error("cgp_mesh_export: bad level");
    return CGP_E_ARG;
  }
  const HostLevel &L = m->lev[level];
  const void *src = nullptr;
  size_t need = 0;
  std::vector<int> tmp;
  const double *dsrc = nullptr;
  const bool device_value = what >= CGP_X_S_F;
  if (device_value && (m->host_only || !m->assembled)) {
    set_error("cgp_mesh_export: operators not assembled");
    return CGP_E_STATE;
  }
  switch (what) {
    case CGP_X_XY: src = L.xy.data(); need = L.xy.size() * 8; break;
    case CGP_X_TRI: src = L.tri.data(); need = L.tri.size() * 4; break;
    case CGP_X_BEDGE: src = L.bedge.data(); need = L.bedge.size() * 4; break;
    case CGP_X_BKIND: src = L.bkind.data(); need = L.bkind.size() * 4; break;
    case CGP_X_PARENT:
      if (level == 0) { set_error("cgp_mesh_export: level 0 has no parents"); return CGP_E_ARG; }
      src = L.parent.data(); need = L.parent.size() * 4; break;
    case CGP_X_EDGES: src = L.edge.data(); need = L.edge.size() * 4; break;
    case CGP_X_ROWPTR_F: src = m->pf.rp.data(); need = m->pf.rp.size() * 4; break;
    case CGP_X_COL_F: src = m->pf.col.data(); need = m->pf.col.size() * 4; break;
    case CGP_X_SLOT_F: src = m->slot_f.data(); need = m->slot_f.size() * 4; break;
    case CGP_X_COLOUR_F: src = m->col_f.colour.data(); need = m->col_f.colour.size() * 4; break;
    case CGP_X_ROWPTR_C: src = m->pc.rp.data(); need = m->pc.rp.size() * 4; break;
    case CGP_X_COL_C: src = m->pc.col.data(); need = m->pc.col.size() * 4; break;
    case CGP_X_SLOT_C: src = m->slot_c.data(); need = m->slot_c.size() * 4; break;
    case CGP_X_COLOUR_C: src = m->col_c.colour.data(); need = m->col_c.colour.size() * 4; break;
    case CGP_X_VDIR: src = m->vdir.data(); need = m->vdir.size() * 4; break;
    case CGP_X_PDIR: src = m->pdir.data(); need = m->pdir.size() * 4; break;
    case CGP_X_SIZES:
      tmp = {L.n, L.t, L.nb, L.ne};
      src = tmp.data(); need = 16; break;
    case CGP_X_S_F: dsrc = m->d_S; need = m->pf.nnz * 8; break;
    case CGP_X_M_F: dsrc = m->d_M; need = m->pf.nnz * 8; break;
    case CGP_X_DX_F: case CGP_X_DY_F: case CGP_X_DX_C: case CGP_X_DY_C: {
      const bool fine = (what == CGP_X_DX_F || what == CGP_X_DY_F);
      const size_t nnz = fine ? m->pf.nnz : m->pc.nnz;
      if (bytes != nnz * 8) { set_error("cgp_mesh_export: size mismatch"); return CGP_E_ARG; }
      std::vector<double> pair(2 * nnz);
      CGP_HIP(hipStreamSynchronize(m->stream));
      CGP_HIP(hipMemcpy(pair.data(), fine ? m->d_D : m->d_Dc, 16 * nnz, hipMemcpyDeviceToHost));
      const int off = (what == CGP_X_DX_F || what == CGP_X_DX_C) ? 0 : 1;
      double *o = static_cast<double *>(dst);
      for (size_t k = 0; k < nnz; k++) o[k] = pair[2 * k + off];
      return CGP_OK;
    }
    case CGP_X_K_C: dsrc = m->d_K; need = m->pc.nnz * 8; break;
    case CGP_X_KBC_C: dsrc = m->d_Kbc; need = m->pc.nnz * 8; break;
    case CGP_X_MC: dsrc = m->d_mc; need = size_t(m->pc.n) * 8; break;
    case CGP_X_A_F: dsrc = m->d_A; need = m->pf.nnz * 8; break;
    case CGP_X_ML_F: dsrc = m->d_ml; need = size_t(m->pf.n) * 8; break;
    case CGP_X_ILU_C:
      if (!m->gm.factored) {
        set_error("cgp_mesh_export: no ILU(0) factors yet (run a CGP_METHOD_ILU_GMRES solve first)");
        return CGP_E_STATE;
      }
      dsrc = m->gm.d_lu;
      need = m->pc.nnz * 8;
      break;
    default: set_error("cgp_mesh_export: unknown selector"); return CGP_E_ARG;
  }
  if (bytes != need) {
    set_error("cgp_mesh_export: size mismatch (expected " + std::to_string(need) + " bytes)");
    return CGP_E_ARG;
  }
  if (what == CGP_X_VDIR || what == CGP_X_PDIR) {
    const std::vector<int> &v = (what == CGP_X_VDIR) ? m->vdir : m->pdir;
    std::memcpy(dst, v.data(), need);
    return CGP_OK;
  }
  if (device_value) {
    CGP_HIP(hipStreamSynchronize(m->stream));
    CGP_HIP(hipMemcpy(dst, dsrc, need, hipMemcpyDeviceToHost));
    return CGP_OK;
  }
  if (need) std::memcpy(dst, src, need);
  return CGP_OK;
}

void cgp_mesh_destroy(cgp_mesh *m) {
  if (!m) return;
  if (!m->host_only) {
    (void)hipStreamSynchronize(m->stream);
    for (void *p : m->allocations) (void)hipFree(p);
    for (hipEvent_t e : m->kt_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : m->step_ev)
      if (e) (void)hipEventDestroy(e);
    for (cgp::Cg1Graph &g : m->cg1_graphs)
      for (hipGraphExec_t x : g.gx)
        if (x) (void)hipGraphExecDestroy(x);
    if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
    if (m->h_state) (void)hipHostFree(m->h_state);
    if (m->h_scalar) (void)hipHostFree(m->h_scalar);
  }
  delete m;
}

cgp_status cgp_assemble(cgp_mesh *m, const cgp_params *p) {
  if (!m || !p) {
    set_error("cgp_assemble: null argument");
    return CGP_E_ARG;
  }
  if (!(p->rho > 0.0) || !(p->mu >= 0.0) || !(p->dt > 0.0) || !std::isfinite(p->rho) || !std::isfinite(p->mu) ||
      !std::isfinite(p->dt) || (p->restrict_mode != CGP_RESTRICT_INJECT && p->restrict_mode != CGP_RESTRICT_GALERKIN) ||
      (p->mass_mode != CGP_MASS_CONSISTENT && p->mass_mode != CGP_MASS_LUMPED) ||
      p->pressure_mode < CGP_PRESSURE_NONINCREMENTAL || p->pressure_mode > CGP_PRESSURE_ROTATIONAL) {
    set_error("cgp_assemble: invalid parameters");
    return CGP_E_ARG;
  }
  if (m->host_only) {
    set_error("cgp_assemble: mesh was created host-only");
    return CGP_E_STATE;
  }
  m->params = *p;
  m->assembled = false;
  m->gm.factored = false;  // the ILU(0) factors belong to the previous operators
  cgp_status s = drv_assemble(m);
  if (s == CGP_OK) m->assembled = true;
  return s;
}

cgp_status cgp_momentum(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *f, const double *u,
                        double *ut, cgp_stats *st) {
  TRY(ready(m));
  if (!valid_opts(o, false, false, true) || !g || !u || !ut) {
    set_error("cgp_momentum: invalid argument");
    return CGP_E_ARG;
  }
  return drv_momentum(m, o, g, f, u, ut, st);
}

cgp_status cgp_restrict(cgp_mesh *m, const double *ut, double *bc) {
  TRY(ready(m));
  if (!ut || !bc) {
    set_error("cgp_restrict: null argument");
    return CGP_E_ARG;
  }
  return drv_restrict(m, ut, bc);
}

cgp_status cgp_poisson_solve(cgp_mesh *m, const double *b, double *x, const cgp_solver_opts *o, cgp_stats *st) {
  TRY(ready(m));
  if (!valid_opts(o, true) || !b || !x) {
    set_error("cgp_poisson_solve: invalid argument");
    return CGP_E_ARG;
  }
  return drv_poisson(m, b, x, o, st);
}

cgp_status cgp_prolong(cgp_mesh *m, const double *pc, double *pf) {
  TRY(ready(m));
  if (!pc || !pf) {
    set_error("cgp_prolong: null argument");
    return CGP_E_ARG;
  }
  return drv_prolong(m, pc, pf);
}

cgp_status cgp_correct(cgp_mesh *m, const cgp_solver_opts *o, const double *g, const double *ut, const double *pf,
                       double *u, cgp_stats *st) {
  TRY(ready(m));
  if (!valid_opts(o, false, false, false, true) || !g || !ut || !pf || !u) {
    set_error("cgp_correct: invalid argument");
    return CGP_E_ARG;
  }
  return drv_correct(m, o, g, ut, pf, u, st);
}

// buffers of the incremental pressure modes, allocated at their first step (the increment starts at 0)
static cgp_status incremental_buffers(cgp_mesh *m) {
  if (m->d_phi) return CGP_OK;
  void *p = nullptr;
  for (double **dst : {&m->d_pfn, &m->d_phif, &m->d_phi}) {
    const size_t n = (dst == &m->d_phi) ? size_t(m->pc.n) : size_t(m->pf.n);
    if (hipMalloc(&p, n * sizeof(double)) != hipSuccess) {
      set_error("cgp_step: out of device memory for the incremental pressure buffers");
      return CGP_E_OOM;
    }
    m->allocations.push_back(p);
    *dst = static_cast<double *>(p);
    CGP_HIP(hipMemsetAsync(p, 0, n * sizeof(double), m->stream));
  }
  return CGP_OK;
}

cgp_status cgp_step(cgp_mesh *m, const cgp_step_opts *o, const double *g, const double *f, double *u, double *pf,
                    double *pc, cgp_stats *st) {
  TRY(ready(m));
  const bool mass_ok = o && (valid_opts(&o->mass, false, false, false, true) ||
                             (valid_opts(&o->mass, false, true, false, true) && o->mass.x0_mode == CGP_X0_EXTRAP));
  if (!o || !valid_opts(&o->momentum, false, true, true) || !valid_opts(&o->poisson, true) || !mass_ok ||
      !g || !u || !pf || !pc) {
    set_error("cgp_step: invalid argument");
    return CGP_E_ARG;
  }
  cgp_stats local{};
  cgp_stats *S = st ? st : &local;
  *S = cgp_stats{};
  hipEvent_t *ev = m->step_ev;  // created at the first timed step, kept until the mesh is destroyed
  const bool timing = o->timing != 0;
  if (timing) {
    if (!ev[0])
      for (int k = 0; k < 7; k++) CGP_HIP(hipEventCreate(&ev[k]));
    CGP_HIP(hipEventRecord(ev[0], m->stream));
  }
  cgp_status worst = CGP_OK;
  auto note = [&](cgp_status s) {
    if (s == CGP_E_NOCONV && worst == CGP_OK) worst = s;
    return s == CGP_OK || s == CGP_E_NOCONV;
  };
  cgp_status s = CGP_OK;
  std::string msg;
  m->kt_on = (o->timing == 2);
  m->kt_ms = 0.0;
  m->kt_count = 0;
  m->kt_iters = 0;
  m->kt_used = 0;
  if (m->params.pressure_mode != CGP_PRESSURE_NONINCREMENTAL) {
    s = incremental_buffers(m);
    if (s) goto out;
    // P_f^n for the momentum right-hand side
    s = drv_prolong(m, pc, m->d_pfn);
    if (s) goto out;
  }
  // step 1 (Eq. 19): momentum on the fine mesh
  s = drv_momentum(m, &o->momentum, g, f, u, m->d_ut, S, m->params.pressure_mode ? m->d_pfn : nullptr);
  if (!note(s)) goto out;
  if (s) msg = g_err;
  if (timing) CGP_HIP(hipEventRecord(ev[2], m->stream));
  // step 2 (Eqs. 20-21): restriction and coarse divergence
  s = drv_restrict(m, m->d_ut, m->d_bc);
  if (!note(s)) goto out;
  if (timing) CGP_HIP(hipEventRecord(ev[3], m->stream));
  if (m->params.pressure_mode == CGP_PRESSURE_NONINCREMENTAL) {
    // step 3 (Eq. 21): coarse pressure Poisson
    s = drv_poisson(m, m->d_bc, pc, &o->poisson, S);
    if (!note(s)) goto out;
    if (s) msg = g_err;
    if (timing) CGP_HIP(hipEventRecord(ev[4], m->stream));
    // step 4 (Eq. 22): prolongation
    s = drv_prolong(m, pc, pf);
    if (!note(s)) goto out;
    if (timing) CGP_HIP(hipEventRecord(ev[5], m->stream));
    // step 5 (Eq. 23): velocity correction
    s = drv_correct(m, &o->mass, g, m->d_ut, pf, u, S);
    if (!note(s)) goto out;
    if (s) msg = g_err;
  } else {
    // step 3: Eq. (21) for the pressure increment (d_bc is left as restricted: the rotational term reads it)
    s = drv_poisson(m, m->d_bc, m->d_phi, &o->poisson, S);
    if (!note(s)) goto out;
    if (s) msg = g_err;
    if (timing) CGP_HIP(hipEventRecord(ev[4], m->stream));
    // step 4: the prolonged increment
    s = drv_prolong(m, m->d_phi, m->d_phif);
    if (!note(s)) goto out;
    if (timing) CGP_HIP(hipEventRecord(ev[5], m->stream));
    // step 5: Eq. (23) with the increment, then the new pressure and its prolongation
    s = drv_correct(m, &o->mass, g, m->d_ut, m->d_phif, u, S);
    if (!note(s)) goto out;
    if (s) msg = g_err;
    launch_pressure_update(m, pc, m->d_phi, m->d_bc);
    CGP_HIP(hipGetLastError());
    s = drv_prolong(m, pc, pf);
    if (s) goto out;
  }
  if (timing) {
    CGP_HIP(hipEventRecord(ev[6], m->stream));
    CGP_HIP(hipEventSynchronize(ev[6]));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, ev[0], ev[2]); S->ms_momentum = ms;
    (void)hipEventElapsedTime(&ms, ev[2], ev[3]); S->ms_restrict = ms;
    (void)hipEventElapsedTime(&ms, ev[3], ev[4]); S->ms_poisson = ms;
    (void)hipEventElapsedTime(&ms, ev[4], ev[5]); S->ms_prolong = ms;
    (void)hipEventElapsedTime(&ms, ev[5], ev[6]); S->ms_correct = ms;
  }
  S->ms_dominant = m->kt_ms;
  S->n_dominant = int32_t(m->kt_count);
  S->dominant_iters = int32_t(m->kt_iters);
  s = worst;
  if (s) g_err = msg;
out:
  m->kt_on = false;
  if (st) CGP_HIP(hipStreamSynchronize(m->stream));
  return s;
}

cgp_status cgp_surface_set(cgp_mesh *m, int32_t count, const int32_t *ids) {
  if (!m || count < 0 || (count > 0 && !ids)) {
    set_error("cgp_surface_set: invalid argument");
    return CGP_E_ARG;
  }
  if (m->host_only) {
    set_error("cgp_surface_set: mesh was created host-only");
    return CGP_E_STATE;
  }
  const HostLevel &C = m->lev[0], &F = m->lev[m->levels];
  std::vector<char> mark(C.nb, 0);
  for (int i = 0; i < count; i++) {
    if (ids[i] < 0 || ids[i] >= C.nb) {
      set_error("cgp_surface_set: boundary edge index " + std::to_string(ids[i]) + " out of range");
      return CGP_E_ARG;
    }
    mark[ids[i]] = 1;
  }
  // fine boundary edge j descends from coarse edge j >> l (each subdivision splits edge k into 2k, 2k+1)
  std::unordered_map<long long, int> slot;  // marked fine edge (min, max) -> row
  std::vector<int> rows;
  for (int j = 0; j < F.nb; j++) {
    if (!mark[j >> m->levels]) continue;
    const int a = F.bedge[2 * j], b = F.bedge[2 * j + 1];
    slot[(long long)std::min(a, b) << 32 | std::max(a, b)] = int(rows.size() / 4);
    rows.insert(rows.end(), {a, b, -1, 0});
  }
  for (int t = 0; t < F.t; t++)
    for (int k = 0; k < 3; k++) {
      const int a = F.tri[3 * t + k], b = F.tri[3 * t + (k + 1) % 3];
      auto it = slot.find((long long)std::min(a, b) << 32 | std::max(a, b));
      if (it != slot.end()) rows[4 * it->second + 2] = F.tri[3 * t + (k + 2) % 3];
    }
  const int ne = int(rows.size() / 4);
  for (int i = 0; i < ne; i++)
    if (rows[4 * i + 2] < 0) {
      set_error("cgp_surface_set: a marked boundary edge lies on no triangle");
      return CGP_E_MESH;
    }
  if (ne > m->n_surf_cap) {
    void *p = nullptr;
    if (hipMalloc(&p, rows.size() * sizeof(int)) != hipSuccess) {
      set_error("cgp_surface_set: out of device memory");
      return CGP_E_OOM;
    }
    m->allocations.push_back(p);
    m->d_surf = static_cast<int *>(p);
    m->n_surf_cap = ne;
  }
  if (ne) CGP_HIP(hipMemcpy(m->d_surf, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice));
  m->n_surf = ne;
  return CGP_OK;
}

cgp_status cgp_surface_traction(cgp_mesh *m, const double *u, const double *pf, double *rows, int32_t *n_rows) {
  TRY(ready(m));
  if (!u || !pf || !n_rows) {
    set_error("cgp_surface_traction: null argument");
    return CGP_E_ARG;
  }
  *n_rows = m->n_surf;
  if (rows && m->n_surf) {
    launch_surface(m, u, pf, rows);
    CGP_HIP(hipGetLastError());
  }
  return CGP_OK;
}

cgp_status cgp_surface_force(cgp_mesh *m, const double *u, const double *pf, double *out) {
  TRY(ready(m));
  if (!u || !pf || !out) {
    set_error("cgp_surface_force: null argument");
    return CGP_E_ARG;
  }
  if (m->n_surf == 0) {
    for (int k = 0; k < 4; k++) out[k] = 0.0;
    return CGP_OK;
  }
  launch_surface(m, u, pf, nullptr);
  CGP_HIP(hipGetLastError());
  CGP_HIP(hipMemcpyAsync(m->h_scalar, m->d_scalar, 4 * sizeof(double), hipMemcpyDeviceToHost, m->stream));
  CGP_HIP(hipStreamSynchronize(m->stream));
  for (int k = 0; k < 4; k++) out[k] = m->h_scalar[k];
  return CGP_OK;
}

cgp_status cgp_mesh_get_tuning(const cgp_mesh *m, cgp_tuning *out) {
  if (!m || !out) {
    set_error("cgp_mesh_get_tuning: null argument");
    return CGP_E_ARG;
  }
  *out = m->tune;
  return CGP_OK;
}

cgp_status cgp_mesh_set_tuning(cgp_mesh *m, const cgp_tuning *t) {
  if (!m || !t) {
    set_error("cgp_mesh_set_tuning: null argument");
    return CGP_E_ARG;
  }
  for (const cgp_tuning_knobs *k : {&t->fine, &t->coarse}) {
    const bool lanes_ok = k->lanes == 2 || k->lanes == 4 || k->lanes == 8 || k->lanes == 16;
    const bool block_ok = k->block == 64 || k->block == 128 || k->block == 256 || k->block == 512 || k->block == 1024;
    if (!lanes_ok || !block_ok || k->passes < 1 || k->passes > 64) {
      set_error("cgp_mesh_set_tuning: lanes must be 2/4/8/16, block 64..1024 (power of two), passes 1..64");
      return CGP_E_ARG;
    }
  }
  if ((t->pcg_barrier != 0 && t->pcg_barrier != 1) || t->pcg_grid < 0 || t->pcg_spin_log2 < 0 ||
      t->pcg_spin_log2 > 30 || (t->pcg_graph != 0 && t->pcg_graph != 1)) {
    set_error("cgp_mesh_set_tuning: pcg_barrier must be 0 or 1, pcg_grid >= 0, pcg_spin_log2 in 0..30 and "
              "pcg_graph 0 or 1");
    return CGP_E_ARG;
  }
  // one block per compute unit at most: the persistent kernel needs every block resident at once
  const int max_grid = m->cu_count > 0 ? m->cu_count : 256;
  if (t->pcg_grid > max_grid) {
    set_error("cgp_mesh_set_tuning: pcg_grid " + std::to_string(t->pcg_grid) + " exceeds one block per compute unit (" +
              std::to_string(max_grid) + ")");
    return CGP_E_ARG;
  }
  m->tune = *t;
  return CGP_OK;
}

cgp_status cgp_spmv(cgp_mesh *m, int32_t op, const void *x, void *y) {
  TRY(ready(m));
  if (!x || !y) {
    set_error("cgp_spmv: null argument");
    return CGP_E_ARG;
  }
  return drv_spmv(m, op, x, y);
}

}  // extern "C"
