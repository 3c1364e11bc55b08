"""ctypes binding of libcgp (argument marshalling only; see include/cgp.h)."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from pathlib import Path

import numpy as np

_PKG = Path(__file__).resolve().parent
library_path = _PKG / "libcgp.so"

STATUS = {0: "CGP_OK", 1: "CGP_E_ARG", 2: "CGP_E_MESH", 3: "CGP_E_NOCONV", 4: "CGP_E_NONFINITE",
          5: "CGP_E_DEVICE", 6: "CGP_E_OOM", 7: "CGP_E_STATE"}
OK, E_ARG, E_MESH, E_NOCONV, E_NONFINITE, E_DEVICE, E_OOM, E_STATE = range(8)
VEL_DIRICHLET, OUTFLOW = 1, 2
RESTRICT_INJECT, RESTRICT_GALERKIN = 0, 1
MASS_CONSISTENT, MASS_LUMPED = 0, 1
PRESSURE_NONINCREMENTAL, PRESSURE_INCREMENTAL, PRESSURE_ROTATIONAL = 0, 1, 2
PREC_FP64, PREC_FP32_IR = 0, 1
X0_ZERO, X0_PREV, X0_LEARNED, X0_LEARNED_CORR, X0_POD_GALERKIN, X0_EXTRAP, X0_PROJECT = 0, 1, 2, 3, 4, 5, 6
LAUNCH_AUTO, LAUNCH_LOOP, LAUNCH_PERSISTENT, LAUNCH_FUSED = 0, 1, 2, 3
METHOD_DEFAULT, METHOD_ILU_GMRES, METHOD_CHEBYSHEV = 0, 1, 2
OP_KBC_C, OP_M_F, OP_A_F, OP_KBC_C32 = 0, 1, 2, 3

EXPORT = {"xy": 0, "tri": 1, "bedge": 2, "bkind": 3, "parent": 4, "edges": 5, "rowptr_f": 6, "col_f": 7,
          "slot_f": 8, "colour_f": 9, "rowptr_c": 10, "col_c": 11, "slot_c": 12, "colour_c": 13, "vdir": 14,
          "pdir": 15, "sizes": 16, "S_f": 20, "M_f": 21, "Dx_f": 22, "Dy_f": 23, "K_c": 24, "K_c_bc": 25,
          "Dx_c": 26, "Dy_c": 27, "m_c": 28, "A_f": 29, "ml_f": 30, "ilu_c": 31}


class CGPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Desc(C.Structure):
    _fields_ = [("n_nodes", C.c_int32), ("xy", C.c_void_p), ("n_tris", C.c_int32), ("tri", C.c_void_p),
                ("n_bedges", C.c_int32), ("bedge", C.c_void_p), ("bedge_kind", C.c_void_p), ("levels", C.c_int32),
                ("flags", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("dt", C.c_double), ("restrict_mode", C.c_int32),
                ("mass_mode", C.c_int32), ("pressure_mode", C.c_int32)]


class _SolverOpts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int32), ("inner_tol", C.c_double),
                ("x0_mode", C.c_int32), ("launch", C.c_int32), ("method", C.c_int32), ("restart", C.c_int32)]


class _StepOpts(C.Structure):
    _fields_ = [("momentum", _SolverOpts), ("poisson", _SolverOpts), ("mass", _SolverOpts), ("timing", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("mom_iters", C.c_int32), ("p_iters", C.c_int32), ("p_outer", C.c_int32), ("mass_iters", C.c_int32),
                ("mom_relres", C.c_double), ("p_relres", C.c_double), ("mass_relres", C.c_double),
                ("ms_assemble", C.c_float), ("ms_momentum", C.c_float), ("ms_restrict", C.c_float),
                ("ms_poisson", C.c_float), ("ms_prolong", C.c_float), ("ms_correct", C.c_float),
                ("ms_dominant", C.c_double), ("n_dominant", C.c_int32), ("dominant_iters", C.c_int32)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _Knobs(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("block", C.c_int32), ("passes", C.c_int32)]


class _Tuning(C.Structure):
    _fields_ = [("fine", _Knobs), ("coarse", _Knobs), ("pcg_barrier", C.c_int32), ("pcg_grid", C.c_int32),
                ("pcg_spin_log2", C.c_int32), ("pcg_graph", C.c_int32)]


class _GuessDesc(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("hidden", C.c_int32), ("seed", C.c_uint64)]


class _TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double), ("seed", C.c_uint64), ("p_prev", C.c_void_p)]


class _TrainStats(C.Structure):
    _fields_ = [("loss_first", C.c_double), ("loss_last", C.c_double), ("steps", C.c_int32), ("ms", C.c_float)]


class _BatchTuning(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("block", C.c_int32), ("passes", C.c_int32), ("use_graph", C.c_int32),
                ("chunk", C.c_int32), ("ahead", C.c_int32)]


class _Info(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("n_f", "t_f", "n_c", "t_c", "nnz_f", "nnz_c", "ncol_f", "ncol_c", "nb_f",
                                          "nb_c", "levels", "n_pdir")]


@dataclass
class SolverOpts:
    tol: float = 1e-10
    max_iter: int = 20000
    precision: int = PREC_FP64
    inner_tol: float = 1e-4
    x0_mode: int = X0_PREV
    launch: int = LAUNCH_AUTO
    method: int = METHOD_DEFAULT
    restart: int = 0

    def c(self):
        return _SolverOpts(self.precision, self.tol, self.max_iter, self.inner_tol, self.x0_mode, self.launch,
                           self.method, self.restart)


@dataclass
class StepOpts:
    momentum: SolverOpts = field(default_factory=lambda: SolverOpts(tol=1e-10, max_iter=2000))
    poisson: SolverOpts = field(default_factory=lambda: SolverOpts(tol=1e-10))
    mass: SolverOpts = field(default_factory=lambda: SolverOpts(tol=1e-12, max_iter=2000))
    timing: int = 0

    def c(self):
        return _StepOpts(self.momentum.c(), self.poisson.c(), self.mass.c(), int(self.timing))


_lib = None


def lib():
    """Load libcgp.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not library_path.exists():
        raise ImportError(f"{library_path} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    L = C.CDLL(str(library_path))
    vp = C.c_void_p
    L.cgp_abi_version.restype = C.c_int32
    L.cgp_last_error.restype = C.c_char_p
    L.cgp_mesh_create.argtypes = [C.POINTER(_Desc), vp, C.POINTER(vp)]
    L.cgp_mesh_query.argtypes = [vp, C.POINTER(_Info)]
    L.cgp_mesh_export.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_size_t]
    L.cgp_mesh_destroy.argtypes = [vp]
    L.cgp_mesh_destroy.restype = None
    L.cgp_assemble.argtypes = [vp, C.POINTER(_Params)]
    L.cgp_step.argtypes = [vp, C.POINTER(_StepOpts), vp, vp, vp, vp, vp, C.POINTER(_Stats)]
    L.cgp_momentum.argtypes = [vp, C.POINTER(_SolverOpts), vp, vp, vp, vp, C.POINTER(_Stats)]
    L.cgp_restrict.argtypes = [vp, vp, vp]
    L.cgp_poisson_solve.argtypes = [vp, vp, vp, C.POINTER(_SolverOpts), C.POINTER(_Stats)]
    L.cgp_poisson_solve_noalloc.argtypes = [vp, vp, vp, C.POINTER(_SolverOpts), C.POINTER(_Stats)]
    L.cgp_prolong.argtypes = [vp, vp, vp]
    L.cgp_correct.argtypes = [vp, C.POINTER(_SolverOpts), vp, vp, vp, vp, C.POINTER(_Stats)]
    L.cgp_spmv.argtypes = [vp, C.c_int32, vp, vp]
    L.cgp_surface_set.argtypes = [vp, C.c_int32, vp]
    L.cgp_surface_traction.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_int32)]
    L.cgp_surface_force.argtypes = [vp, vp, vp, vp]
    L.cgp_mesh_get_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    L.cgp_mesh_set_tuning.argtypes = [vp, C.POINTER(_Tuning)]
    L.cgp_guess_create.argtypes = [vp, C.POINTER(_GuessDesc), C.POINTER(vp)]
    L.cgp_guess_destroy.argtypes = [vp]
    L.cgp_guess_destroy.restype = None
    L.cgp_guess_build_pod.argtypes = [vp, vp, C.c_int32, vp]
    L.cgp_guess_train.argtypes = [vp, vp, vp, C.c_int32, C.POINTER(_TrainOpts), C.POINTER(_TrainStats)]
    L.cgp_guess_attach.argtypes = [vp, vp]
    L.cgp_guess_predict.argtypes = [vp, C.c_int32, vp, vp]
    L.cgp_guess_get_params.argtypes = [vp, vp, C.c_size_t]
    L.cgp_guess_set_params.argtypes = [vp, vp, C.c_size_t]
    L.cgp_guess_mlp_grad.argtypes = [vp, vp, vp, C.c_int32, C.POINTER(C.c_double), vp, vp]
    L.cgp_guess_export_basis.argtypes = [vp, vp, C.c_size_t]
    L.cgp_guess_export_norm.argtypes = [vp, vp, C.c_size_t]
    L.cgp_guess_set_online.argtypes = [vp, C.c_int32, C.c_int32]
    L.cgp_last_poisson_rhs.argtypes = [vp, vp]
    pp = C.POINTER(vp)
    L.cgp_batch_create.argtypes = [pp, C.c_int32, C.POINTER(vp)]
    L.cgp_batch_destroy.argtypes = [vp]
    L.cgp_batch_destroy.restype = None
    L.cgp_batch_poisson_solve.argtypes = [vp, pp, pp, C.POINTER(_SolverOpts), C.POINTER(_Stats)]
    L.cgp_batch_step.argtypes = [vp, C.POINTER(_StepOpts), pp, pp, pp, pp, pp, C.POINTER(_Stats)]
    L.cgp_batch_get_tuning.argtypes = [vp, C.POINTER(_BatchTuning)]
    L.cgp_batch_set_tuning.argtypes = [vp, C.POINTER(_BatchTuning)]
    L.cgp_batch_autotune.argtypes = [vp, C.c_char_p, C.POINTER(_BatchTuning)]
    for name in ("cgp_guess_create", "cgp_guess_build_pod", "cgp_guess_train", "cgp_guess_attach", "cgp_guess_predict",
                 "cgp_guess_get_params", "cgp_guess_set_params", "cgp_guess_mlp_grad", "cgp_guess_export_basis",
                 "cgp_guess_export_norm", "cgp_guess_set_online", "cgp_last_poisson_rhs", "cgp_mesh_get_tuning",
                 "cgp_mesh_set_tuning",
                 "cgp_mesh_create", "cgp_mesh_query", "cgp_mesh_export", "cgp_assemble", "cgp_step", "cgp_momentum",
                 "cgp_restrict", "cgp_poisson_solve", "cgp_poisson_solve_noalloc", "cgp_prolong", "cgp_correct",
                 "cgp_spmv", "cgp_surface_set", "cgp_surface_traction", "cgp_surface_force", "cgp_batch_create",
                 "cgp_batch_poisson_solve", "cgp_batch_step", "cgp_batch_get_tuning", "cgp_batch_set_tuning",
                 "cgp_batch_autotune"):
        getattr(L, name).restype = C.c_int32
    _lib = L
    return L


def abi_version() -> int:
    return int(lib().cgp_abi_version())


def _check(status: int, allow=(OK,)):
    if status not in allow:
        raise CGPError(status, lib().cgp_last_error().decode(errors="replace"))
    return status


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """A coarse mesh with ``levels`` 1:4 subdivisions, its operators and solver state on the GPU."""

    def __init__(self, coarse, levels: int, host_only: bool = False):
        L = lib()
        self._keep = [np.ascontiguousarray(coarse.xy, np.float64), np.ascontiguousarray(coarse.tri, np.int32),
                      np.ascontiguousarray(coarse.bedge, np.int32), np.ascontiguousarray(coarse.bkind, np.int32)]
        xy, tri, be, bk = self._keep
        d = _Desc(xy.shape[0], xy.ctypes.data, tri.shape[0], tri.ctypes.data, be.shape[0], be.ctypes.data,
                  bk.ctypes.data, levels, 1 if host_only else 0)
        h = C.c_void_p()
        stream = C.c_void_p(None) if host_only else _stream()
        _check(L.cgp_mesh_create(C.byref(d), stream, C.byref(h)))
        self._h = h
        self.levels = levels
        info = _Info()
        _check(L.cgp_mesh_query(self._h, C.byref(info)))
        self.info = {k: int(getattr(info, k)) for k, _ in _Info._fields_}
        self.host_only = host_only

    def close(self):
        if getattr(self, "_h", None):
            lib().cgp_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- export
    def sizes(self, level: int):
        out = np.zeros(4, np.int32)
        _check(lib().cgp_mesh_export(self._h, EXPORT["sizes"], level, out.ctypes.data, out.nbytes))
        return dict(n=int(out[0]), t=int(out[1]), nb=int(out[2]), ne=int(out[3]))

    def export(self, what: str, level: int | None = None) -> np.ndarray:
        lv = self.levels if level is None else level
        s = self.sizes(lv)
        inf = self.info
        shapes = {
            "xy": ((s["n"], 2), np.float64), "tri": ((s["t"], 3), np.int32), "bedge": ((s["nb"], 2), np.int32),
            "bkind": ((s["nb"],), np.int32),
            "parent": ((s["n"] - (self.sizes(lv - 1)["n"] if lv > 0 else 0), 2), np.int32),
            "edges": ((s["ne"], 2), np.int32), "rowptr_f": ((inf["n_f"] + 1,), np.int32),
            "col_f": ((inf["nnz_f"],), np.int32), "slot_f": ((inf["t_f"], 9), np.int32),
            "colour_f": ((inf["t_f"],), np.int32), "rowptr_c": ((inf["n_c"] + 1,), np.int32),
            "col_c": ((inf["nnz_c"],), np.int32), "slot_c": ((inf["t_c"], 9), np.int32),
            "colour_c": ((inf["t_c"],), np.int32), "vdir": ((inf["n_f"],), np.int32),
            "pdir": ((inf["n_c"],), np.int32),
        }
        nnzf, nnzc = inf["nnz_f"], inf["nnz_c"]
        for k in ("S_f", "M_f", "Dx_f", "Dy_f", "A_f"):
            shapes[k] = ((nnzf,), np.float64)
        for k in ("K_c", "K_c_bc", "Dx_c", "Dy_c", "ilu_c"):
            shapes[k] = ((nnzc,), np.float64)
        shapes["m_c"] = ((inf["n_c"],), np.float64)
        shapes["ml_f"] = ((inf["n_f"],), np.float64)
        shape, dt = shapes[what]
        out = np.zeros(shape, dt)
        _check(lib().cgp_mesh_export(self._h, EXPORT[what], lv, out.ctypes.data, out.nbytes))
        return out

    # ---------------------------------------------------------------- compute
    def assemble(self, rho: float, mu: float, dt: float, restrict_mode: int = RESTRICT_INJECT,
                 mass_mode: int = MASS_CONSISTENT, pressure_mode: int = PRESSURE_NONINCREMENTAL):
        p = _Params(rho, mu, dt, restrict_mode, mass_mode, pressure_mode)
        _check(lib().cgp_assemble(self._h, C.byref(p)))
        self.params = dict(rho=rho, mu=mu, dt=dt, restrict_mode=restrict_mode, mass_mode=mass_mode,
                           pressure_mode=pressure_mode)

    def step(self, g, u, p_fine, p_coarse, f=None, opts: StepOpts | None = None, allow_noconv=False):
        """One IFE-CGP step in place on device tensors; returns the stats dict."""
        o = (opts or StepOpts()).c()
        st = _Stats()
        s = lib().cgp_step(self._h, C.byref(o), _ptr(g), _ptr(f), _ptr(u), _ptr(p_fine), _ptr(p_coarse),
                           C.byref(st))
        _check(s, (OK, E_NOCONV) if allow_noconv else (OK,))
        d = st.asdict()
        d["status"] = s
        return d

    def momentum(self, g, u, u_tilde, f=None, opts: SolverOpts | None = None):
        o = (opts or SolverOpts()).c()
        st = _Stats()
        _check(lib().cgp_momentum(self._h, C.byref(o), _ptr(g), _ptr(f), _ptr(u), _ptr(u_tilde), C.byref(st)))
        return st.asdict()

    def restrict(self, u_tilde, b_coarse):
        _check(lib().cgp_restrict(self._h, _ptr(u_tilde), _ptr(b_coarse)))

    def poisson_solve(self, b, x, opts: SolverOpts | None = None, allow_noconv=False):
        o = (opts or SolverOpts()).c()
        st = _Stats()
        s = lib().cgp_poisson_solve(self._h, _ptr(b), _ptr(x), C.byref(o), C.byref(st))
        _check(s, (OK, E_NOCONV) if allow_noconv else (OK,))
        d = st.asdict()
        d["status"] = s
        return d

    def poisson_solve_noalloc(self, b, x, opts: SolverOpts | None = None, allow_noconv=False):
        """cgp_poisson_solve with its working memory in the library's fixed device array (no allocation)."""
        o = (opts or SolverOpts()).c()
        st = _Stats()
        s = lib().cgp_poisson_solve_noalloc(self._h, _ptr(b), _ptr(x), C.byref(o), C.byref(st))
        _check(s, (OK, E_NOCONV) if allow_noconv else (OK,))
        d = st.asdict()
        d["status"] = s
        return d

    def prolong(self, p_coarse, p_fine):
        _check(lib().cgp_prolong(self._h, _ptr(p_coarse), _ptr(p_fine)))

    def correct(self, g, u_tilde, p_fine, u, opts: SolverOpts | None = None):
        o = (opts or SolverOpts(tol=1e-12)).c()
        st = _Stats()
        _check(lib().cgp_correct(self._h, C.byref(o), _ptr(g), _ptr(u_tilde), _ptr(p_fine), _ptr(u), C.byref(st)))
        return st.asdict()

    def get_tuning(self):
        t = _Tuning()
        _check(lib().cgp_mesh_get_tuning(self._h, C.byref(t)))
        d = {lvl: (getattr(t, lvl).lanes, getattr(t, lvl).block, getattr(t, lvl).passes) for lvl in ("fine", "coarse")}
        d["pcg_barrier"] = t.pcg_barrier
        d["pcg_grid"] = t.pcg_grid
        d["pcg_spin_log2"] = t.pcg_spin_log2
        d["pcg_graph"] = t.pcg_graph
        return d

    def set_tuning(self, fine=None, coarse=None, pcg_barrier=None, pcg_grid=None, pcg_spin_log2=None,
                   pcg_graph=None):
        cur = self.get_tuning()
        f = fine or cur["fine"]
        c = coarse or cur["coarse"]
        b = cur["pcg_barrier"] if pcg_barrier is None else pcg_barrier
        g = cur["pcg_grid"] if pcg_grid is None else pcg_grid
        sp = cur["pcg_spin_log2"] if pcg_spin_log2 is None else pcg_spin_log2
        gr = cur["pcg_graph"] if pcg_graph is None else pcg_graph
        t = _Tuning(_Knobs(*f), _Knobs(*c), b, g, sp, gr)
        _check(lib().cgp_mesh_set_tuning(self._h, C.byref(t)))

    def last_poisson_rhs(self, dst):
        _check(lib().cgp_last_poisson_rhs(self._h, _ptr(dst)))

    def surface_set(self, coarse_bedge_ids):
        """Mark the measured surface by coarse boundary-edge indices (drag/lift body or a wall)."""
        ids = np.ascontiguousarray(coarse_bedge_ids, np.int32)
        _check(lib().cgp_surface_set(self._h, ids.size, ids.ctypes.data if ids.size else None))

    def surface_traction(self, u, p_fine):
        """Device tensor [n_edges][8]: midpoint x, y, length, pressure force x, y, viscous force x, y, 0."""
        import torch
        n = C.c_int32()
        _check(lib().cgp_surface_traction(self._h, _ptr(u), _ptr(p_fine), None, C.byref(n)))
        rows = torch.zeros((n.value, 8), dtype=torch.float64, device=u.device)
        if n.value:
            _check(lib().cgp_surface_traction(self._h, _ptr(u), _ptr(p_fine), _ptr(rows), C.byref(n)))
        return rows

    def surface_force(self, u, p_fine):
        """Force of the fluid on the surface: [pressure x, pressure y, viscous x, viscous y] (host)."""
        out = np.zeros(4)
        _check(lib().cgp_surface_force(self._h, _ptr(u), _ptr(p_fine), out.ctypes.data))
        return out

    def spmv(self, op: int, x, y):
        _check(lib().cgp_spmv(self._h, op, _ptr(x), _ptr(y)))


class Guess:
    """Learned initial guess for the Poisson solve: POD basis + BF16 MFMA MLP (include/cgp.h)."""

    def __init__(self, mesh: Mesh, n_modes: int = 64, hidden: int = 256, seed: int = 4):
        self.mesh = mesh
        self.n_modes, self.hidden = n_modes, hidden
        h = C.c_void_p()
        _check(lib().cgp_guess_create(mesh._h, C.byref(_GuessDesc(n_modes, hidden, seed)), C.byref(h)))
        self._h = h
        m, hd = n_modes, hidden
        self.nparams = hd * m + hd + hd * hd + hd + m * hd + m

    def close(self):
        if getattr(self, "_h", None):
            lib().cgp_guess_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_pod(self, snaps):
        energy = np.zeros(self.n_modes)
        _check(lib().cgp_guess_build_pod(self._h, _ptr(snaps), snaps.shape[0], energy.ctypes.data))
        return energy

    def train(self, rhs, p, epochs=200, batch=256, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=4,
              p_prev=None):
        """Absolute model (p_prev None) or incremental model (p_prev: previous pressure of each sample)."""
        st = _TrainStats()
        o = _TrainOpts(epochs, batch, lr, beta1, beta2, eps, seed, _ptr(p_prev) if p_prev is not None else None)
        _check(lib().cgp_guess_train(self._h, _ptr(rhs), _ptr(p), rhs.shape[0], C.byref(o), C.byref(st)))
        return {k: getattr(st, k) for k, _ in _TrainStats._fields_}

    def set_online(self, window: int, refresh: int = 1):
        """Rebuild the basis every `refresh` Poisson solves from the last `window` solutions (0: off)."""
        _check(lib().cgp_guess_set_online(self._h, window, refresh))

    def attach(self):
        _check(lib().cgp_guess_attach(self.mesh._h, self._h))

    def detach(self):
        _check(lib().cgp_guess_attach(self.mesh._h, None))

    def predict(self, mode: int, b, x):
        _check(lib().cgp_guess_predict(self._h, mode, _ptr(b), _ptr(x)))

    def get_params(self):
        out = np.zeros(self.nparams, np.float32)
        _check(lib().cgp_guess_get_params(self._h, out.ctypes.data, out.size))
        return out

    def set_params(self, w):
        w = np.ascontiguousarray(w, np.float32)
        _check(lib().cgp_guess_set_params(self._h, w.ctypes.data, w.size))

    def mlp_grad(self, x, t):
        x = np.ascontiguousarray(x, np.float32)
        t = np.ascontiguousarray(t, np.float32)
        B = x.shape[0]
        loss = C.c_double()
        y = np.zeros((B, self.n_modes), np.float32)
        g = np.zeros(self.nparams, np.float32)
        _check(lib().cgp_guess_mlp_grad(self._h, x.ctypes.data, t.ctypes.data, B, C.byref(loss), y.ctypes.data,
                                        g.ctypes.data))
        return loss.value, y, g

    def norm(self):
        out = np.zeros((4, self.n_modes))
        _check(lib().cgp_guess_export_norm(self._h, out.ctypes.data, out.size))
        return out

    def basis(self):
        out = np.zeros((self.mesh.info["n_c"], self.n_modes))
        _check(lib().cgp_guess_export_basis(self._h, out.ctypes.data, out.size))
        return out


def _ptrs(ts):
    arr = (C.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        arr[i] = _ptr(t).value
    return arr


class Batch:
    """Independent meshes solved together: one batched Poisson PCG per step (include/cgp.h)."""

    def __init__(self, meshes):
        self.meshes = list(meshes)
        hs = (C.c_void_p * len(self.meshes))(*[m._h.value for m in self.meshes])
        h = C.c_void_p()
        _check(lib().cgp_batch_create(hs, len(self.meshes), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().cgp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def poisson_solve(self, rhs, xs, opts: SolverOpts | None = None, allow_noconv=False):
        o = (opts or SolverOpts()).c()
        st = (_Stats * len(self.meshes))()
        s = lib().cgp_batch_poisson_solve(self._h, _ptrs(rhs), _ptrs(xs), C.byref(o), st)
        _check(s, (OK, E_NOCONV) if allow_noconv else (OK,))
        return [x.asdict() for x in st]

    def step(self, g, u, p_fine, p_coarse, f=None, opts: StepOpts | None = None, allow_noconv=False):
        o = (opts or StepOpts()).c()
        st = (_Stats * len(self.meshes))()
        s = lib().cgp_batch_step(self._h, C.byref(o), _ptrs(g), _ptrs(f) if f is not None else None, _ptrs(u),
                                 _ptrs(p_fine), _ptrs(p_coarse), st)
        _check(s, (OK, E_NOCONV) if allow_noconv else (OK,))
        return [x.asdict() for x in st]

    def get_tuning(self):
        t = _BatchTuning()
        _check(lib().cgp_batch_get_tuning(self._h, C.byref(t)))
        return {k: getattr(t, k) for k, _ in _BatchTuning._fields_}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = _BatchTuning(*[cur[k] for k, _ in _BatchTuning._fields_])
        _check(lib().cgp_batch_set_tuning(self._h, C.byref(t)))

    def autotune(self, cache_path=None):
        t = _BatchTuning()
        _check(lib().cgp_batch_autotune(self._h, str(cache_path).encode() if cache_path else None, C.byref(t)))
        return {k: getattr(t, k) for k, _ in _BatchTuning._fields_}
