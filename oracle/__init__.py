"""ctypes binding of the plain FP64 CPU oracle (``oracle/*.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the benchmark's CPU-baseline leg.  The GPU product path never imports
it.  ``build()`` compiles the C sources with gcc into ``oracle/liboracle.so``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

_DIR = Path(__file__).resolve().parent
# CGP_ORACLE_OPENMP=1 selects the OpenMP build (multi-core CPU-baseline timing only; parity uses the
# single-thread build)
_OPENMP = os.environ.get("CGP_ORACLE_OPENMP", "") == "1"
_LIB_PATH = _DIR / ("liboracle_omp.so" if _OPENMP else "liboracle.so")
_SOURCES = ["mesh.c", "fem.c", "krylov.c", "cgp.c", "learn.c", "pod.c", "norms.c", "forces.c", "gmres.c"]
_lib = None

ERRORS = {0: "ok", 1: "bad argument", 2: "invalid mesh", 3: "no convergence", 4: "non-finite value"}


def build(openmp: bool = False) -> Path:
    """Compile the oracle with gcc (plain C99, -O2, no fast-math); openmp=True builds liboracle_omp.so."""
    srcs = [str(_DIR / s) for s in _SOURCES if (_DIR / s).exists()]
    out = _DIR / ("liboracle_omp.so" if openmp else "liboracle.so")
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-fPIC", "-shared", "-Wall",
           "-Wno-unused-function", "-Wno-unknown-pragmas"] + (["-fopenmp"] if openmp else []) + \
          ["-o", str(out) + ".tmp"] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(str(out) + ".tmp", out)
    return out


def lib():
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            build(openmp=_OPENMP)
        _lib = C.CDLL(str(_LIB_PATH))
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


class Stats(C.Structure):
    _fields_ = [("mom_iters", C.c_int * 2), ("p_iters", C.c_int), ("mass_iters", C.c_int * 2),
                ("mom_relres", C.c_double * 2), ("p_relres", C.c_double), ("mass_relres", C.c_double * 2)]

    def asdict(self):
        return {"mom_iters": list(self.mom_iters), "p_iters": self.p_iters, "mass_iters": list(self.mass_iters),
                "mom_relres": list(self.mom_relres), "p_relres": self.p_relres,
                "mass_relres": list(self.mass_relres)}


def _declare(L):
    L.orc_check_mesh.restype = C.c_int
    L.orc_check_mesh.argtypes = [C.c_int, _dp, C.c_int, _ip, C.c_int, _ip, _ip]
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.c_int, _dp, C.c_int, _ip, C.c_int, _ip, _ip, C.c_int, _ip]
    L.orc_free.argtypes = [C.c_void_p]
    L.orc_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
    L.orc_export.restype = C.c_int
    L.orc_export.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
    L.orc_priority.restype = C.c_uint64
    L.orc_priority.argtypes = [C.c_uint64]
    L.orc_element.argtypes = [_dp, _dp, C.c_double, _dp, _dp, _dp, _dp, _dp]
    L.orc_assemble.restype = C.c_int
    L.orc_assemble.argtypes = [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int]
    L.orc_export_values.restype = C.c_int
    L.orc_export_values.argtypes = [C.c_void_p, C.c_int, _dp]
    L.orc_step.restype = C.c_int
    L.orc_step.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int,
                           C.c_int, C.POINTER(Stats)]
    L.orc_projection_step.restype = C.c_int
    L.orc_projection_step.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                      C.c_int, C.POINTER(Stats)]
    L.orc_momentum.restype = C.c_int
    L.orc_momentum.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_double, C.c_int, C.POINTER(Stats)]
    L.orc_convection.restype = None
    L.orc_convection.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_restrict.restype = C.c_int
    L.orc_restrict.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
    L.orc_prolong.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_poisson_solve.restype = C.c_int
    L.orc_poisson_solve.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, _ip, _dp]
    L.orc_dense_solve.restype = C.c_int
    L.orc_dense_solve.argtypes = [C.c_int, _dp, _dp, _dp]
    for name in ("orc_pcg", "orc_bicgstab"):
        f = getattr(L, name)
        f.restype = C.c_int
        f.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_double, C.c_int, _ip, _dp]
    L.orc_spmv.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_set_pressure_mode.restype = C.c_int
    L.orc_set_pressure_mode.argtypes = [C.c_void_p, C.c_int]
    L.orc_pressure_update.restype = C.c_int
    L.orc_pressure_update.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_correct.restype = C.c_int
    L.orc_correct.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_double, C.c_int, C.POINTER(Stats)]
    L.orc_jacobi_eigen.restype = None
    L.orc_jacobi_eigen.argtypes = [C.c_int, _dp, _dp]
    L.orc_pod.restype = C.c_int
    L.orc_pod.argtypes = [C.c_int, C.c_int, _dp, _dp, C.c_int, _dp, _dp]
    L.orc_ilu0.restype = C.c_int
    L.orc_ilu0.argtypes = [C.c_void_p, _dp, _dp]
    L.orc_ilu0_apply.restype = None
    L.orc_ilu0_apply.argtypes = [C.c_void_p, _dp, _dp, _dp]
    L.orc_gmres.restype = C.c_int
    L.orc_gmres.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_int, C.c_double, C.c_int, C.c_int, _ip, _dp]
    L.orc_surface_traction.restype = C.c_int
    L.orc_surface_traction.argtypes = [C.c_void_p, _ip, _dp, _dp, _dp, C.c_int]
    L.orc_surface_force.restype = C.c_int
    L.orc_surface_force.argtypes = [C.c_void_p, _ip, _dp, _dp, _dp]
    L.orc_quad_npts.restype = C.c_int
    L.orc_quad_points.restype = C.c_int
    L.orc_quad_points.argtypes = [C.c_void_p, C.c_int, _dp]
    L.orc_error_norms.restype = C.c_int
    L.orc_error_norms.argtypes = [C.c_void_p, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp]
    if hasattr(L, "orc_mlp_forward_backward"):
        _declare_learn(L)


class _CSR(C.Structure):
    _fields_ = [("n", C.c_int), ("nnz", C.c_int), ("rp", _ip), ("col", _ip)]


def _csr(rp, col):
    rp = np.ascontiguousarray(rp, np.int32)
    col = np.ascontiguousarray(col, np.int32)
    s = _CSR(len(rp) - 1, len(col), _i(rp), _i(col))
    return s, (rp, col)


def priority(t: int) -> int:
    return int(lib().orc_priority(C.c_uint64(t)))


def element(xy3, u3=None, rho=1.0):
    """P1 element matrices (M, K, Dx, Dy, N) of one triangle."""
    xy3 = np.ascontiguousarray(xy3, np.float64).reshape(6)
    out = [np.zeros(9) for _ in range(5)]
    u = np.ascontiguousarray(u3, np.float64).reshape(6) if u3 is not None else None
    lib().orc_element(_d(xy3), _d(u) if u is not None else None, rho, *[_d(o) for o in out])
    return [o.reshape(3, 3) for o in out]


def check_mesh(mesh) -> int:
    return lib().orc_check_mesh(mesh.n_nodes, _d(mesh.xy), mesh.n_tris, _i(mesh.tri), len(mesh.bedge),
                                _i(mesh.bedge), _i(mesh.bkind))


def pcg(rp, col, val, b, x0=None, tol=1e-12, maxit=100000, method="cg"):
    s, keep = _csr(rp, col)
    val = np.ascontiguousarray(val, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    it, rr = C.c_int(), C.c_double()
    f = lib().orc_pcg if method == "cg" else lib().orc_bicgstab
    st = f(C.byref(s), _d(val), _d(b), _d(x), tol, maxit, C.byref(it), C.byref(rr))
    return x, st, it.value, rr.value


def ilu0(rp, col, val):
    """ILU(0) factors of a CSR matrix on its own pattern (unit L below the diagonal, U on and above)."""
    s, keep = _csr(rp, col)
    val = np.ascontiguousarray(val, np.float64)
    lu = np.zeros_like(val)
    if lib().orc_ilu0(C.byref(s), _d(val), _d(lu)):
        raise RuntimeError("zero pivot in ILU(0)")
    return lu


def ilu0_apply(rp, col, lu, r):
    s, keep = _csr(rp, col)
    z = np.zeros(len(rp) - 1)
    lib().orc_ilu0_apply(C.byref(s), _d(np.ascontiguousarray(lu, np.float64)), _d(np.ascontiguousarray(r, np.float64)),
                         _d(z))
    return z


def gmres(rp, col, val, b, x0=None, m=30, tol=1e-12, maxit=100000, ilu=True, orth="mgs"):
    """ILU(0)-preconditioned (or plain) GMRES(m): solution, status, iterations, relative residual.
    orth: "mgs" (modified Gram-Schmidt) or "cgs2" (classical Gram-Schmidt applied twice)."""
    s, keep = _csr(rp, col)
    val = np.ascontiguousarray(val, np.float64)
    b = np.ascontiguousarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    lu = ilu0(rp, col, val) if ilu else None
    it, rr = C.c_int(), C.c_double()
    st = lib().orc_gmres(C.byref(s), _d(val), _d(lu) if lu is not None else None, _d(b), _d(x), m, tol, maxit,
                         {"mgs": 0, "cgs2": 1}[orth], C.byref(it), C.byref(rr))
    return x, st, it.value, rr.value


def spmv(rp, col, val, x):
    s, keep = _csr(rp, col)
    x = np.ascontiguousarray(x, np.float64)
    y = np.zeros(len(rp) - 1)
    lib().orc_spmv(C.byref(s), _d(np.ascontiguousarray(val, np.float64)), _d(x), _d(y))
    return y


def dense_solve(A, b):
    A = np.array(A, np.float64, order="C")
    b = np.array(b, np.float64)
    x = np.zeros_like(b)
    st = lib().orc_dense_solve(len(b), _d(A), _d(b), _d(x))
    if st:
        raise RuntimeError("singular matrix")
    return x


class Problem:
    """A coarse mesh refined ``levels`` times, with the CGP operators of the oracle."""

    INFO = ("n_f", "t_f", "n_c", "t_c", "nnz_f", "nnz_c", "ncol_f", "ncol_c", "nb_f", "nb_c", "levels", "n_pdir")

    def __init__(self, mesh, levels: int):
        st = C.c_int()
        self._h = lib().orc_create(mesh.n_nodes, _d(mesh.xy), mesh.n_tris, _i(mesh.tri), len(mesh.bedge),
                                   _i(mesh.bedge), _i(mesh.bkind), levels, C.byref(st))
        if not self._h:
            raise ValueError(f"oracle rejected the mesh: {ERRORS.get(st.value, st.value)}")
        out = (C.c_int64 * 12)()
        lib().orc_info(self._h, out)
        self.info = dict(zip(self.INFO, [int(v) for v in out]))
        self.levels = levels

    def __del__(self):
        if getattr(self, "_h", None):
            lib().orc_free(self._h)
            self._h = None

    def level_sizes(self, level):
        o = np.zeros(4, np.int32)
        lib().orc_export(self._h, 16, level, o.ctypes.data_as(C.c_void_p))
        return dict(n=int(o[0]), t=int(o[1]), nb=int(o[2]), ne=int(o[3]))

    def export(self, what: str, level: int | None = None):
        lv = self.levels if level is None else level
        s = self.level_sizes(lv)
        inf = self.info
        table = {
            "xy": (0, (s["n"], 2), np.float64), "tri": (1, (s["t"], 3), np.int32),
            "bedge": (2, (s["nb"], 2), np.int32), "bkind": (3, (s["nb"],), np.int32),
            "parent": (4, (s["n"] - (self.level_sizes(lv - 1)["n"] if lv > 0 else 0), 2), np.int32),
            "edges": (5, (s["ne"], 2), np.int32),
            "rowptr_f": (6, (inf["n_f"] + 1,), np.int32), "col_f": (7, (inf["nnz_f"],), np.int32),
            "slot_f": (8, (inf["t_f"], 9), np.int32), "colour_f": (9, (inf["t_f"],), np.int32),
            "rowptr_c": (10, (inf["n_c"] + 1,), np.int32), "col_c": (11, (inf["nnz_c"],), np.int32),
            "slot_c": (12, (inf["t_c"], 9), np.int32), "colour_c": (13, (inf["t_c"],), np.int32),
            "vdir": (14, (inf["n_f"],), np.int32), "pdir": (15, (inf["n_c"],), np.int32),
        }
        code, shape, dt = table[what]
        out = np.zeros(shape, dt)
        st = lib().orc_export(self._h, code, lv, out.ctypes.data_as(C.c_void_p))
        if st:
            raise ValueError(f"export {what} failed")
        return out

    def assemble(self, rho, mu, dt, restrict_mode=0, mass_mode=0, pressure_mode=0):
        """pressure_mode: 0 non-incremental (the paper's scheme), 1 standard incremental, 2 rotational."""
        st = lib().orc_assemble(self._h, rho, mu, dt, restrict_mode, mass_mode)
        if st or lib().orc_set_pressure_mode(self._h, pressure_mode):
            raise ValueError("assemble failed")
        self.params = dict(rho=rho, mu=mu, dt=dt, restrict_mode=restrict_mode, mass_mode=mass_mode,
                           pressure_mode=pressure_mode)

    def values(self, what: str):
        names = ["M_f", "K_f", "Dx_f", "Dy_f", "ml_f", "K_c", "K_c_bc", "Dx_c", "Dy_c", "m_c"]
        code = names.index(what)
        n = {4: self.info["n_f"], 9: self.info["n_c"]}.get(code)
        if n is None:
            n = self.info["nnz_f"] if code < 4 else self.info["nnz_c"]
        out = np.zeros(n)
        if lib().orc_export_values(self._h, code, _d(out)):
            raise ValueError("not assembled")
        return out

    def convection(self, u):
        """Values of the convection matrix N(u) of Eq. (16) on the fine CSR pattern (rho included)."""
        u = np.ascontiguousarray(u, np.float64)
        out = np.zeros(self.info["nnz_f"])
        lib().orc_convection(self._h, _d(u), _d(out))
        return out

    def momentum(self, g, u, f=None, tol=1e-12, maxit=100000):
        g = np.ascontiguousarray(g, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        ut = np.zeros_like(u)
        st = Stats()
        fa = np.ascontiguousarray(f, np.float64) if f is not None else None
        code = lib().orc_momentum(self._h, _d(g), _d(fa) if fa is not None else None, _d(u), _d(ut), tol, maxit,
                                  C.byref(st))
        return ut, code, st.asdict()

    def restrict(self, ut, mode=0):
        ut = np.ascontiguousarray(ut, np.float64)
        b = np.zeros(self.info["n_c"])
        if lib().orc_restrict(self._h, mode, _d(ut), _d(b)):
            raise ValueError("bad restriction mode")
        return b

    def prolong(self, pc):
        pc = np.ascontiguousarray(pc, np.float64)
        pf = np.zeros(self.info["n_f"])
        lib().orc_prolong(self._h, _d(pc), _d(pf))
        return pf

    def poisson_solve(self, b, x0=None, tol=1e-12, maxit=100000):
        b = np.ascontiguousarray(b, np.float64)
        x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
        it, rr = C.c_int(), C.c_double()
        code = lib().orc_poisson_solve(self._h, _d(b), _d(x), tol, maxit, C.byref(it), C.byref(rr))
        return x, code, it.value, rr.value

    def step(self, g, u, pc=None, f=None, tol_mom=1e-12, tol_p=1e-12, tol_mass=1e-12, maxit=100000,
             x0_prev=True):
        g = np.ascontiguousarray(g, np.float64)
        u = np.array(u, np.float64, order="C")
        pf = np.zeros(self.info["n_f"])
        pc = np.zeros(self.info["n_c"]) if pc is None else np.array(pc, np.float64)
        fa = np.ascontiguousarray(f, np.float64) if f is not None else None
        st = Stats()
        code = lib().orc_step(self._h, _d(g), _d(fa) if fa is not None else None, _d(u), _d(pf), _d(pc), tol_mom,
                              tol_p, tol_mass, maxit, int(x0_prev), C.byref(st))
        return u, pf, pc, code, st.asdict()

    def correct(self, g, ut, pf, tol=1e-12, maxit=100000):
        """Step 5 alone (Eq. 23): U^{n+1} from U~ and the fine pressure, with the assembled mass mode."""
        g = np.ascontiguousarray(g, np.float64)
        ut = np.ascontiguousarray(ut, np.float64)
        pf = np.ascontiguousarray(pf, np.float64)
        u = np.zeros_like(ut)
        st = Stats()
        code = lib().orc_correct(self._h, _d(g), _d(ut), _d(pf), _d(u), tol, maxit, C.byref(st))
        return u, code, st.asdict()

    def pressure_update(self, bc, phi, pc):
        """New coarse pressure of the incremental schemes from the restricted right-hand side, the increment
        and the previous pressure."""
        out = np.array(pc, np.float64)
        if lib().orc_pressure_update(self._h, _d(np.ascontiguousarray(bc, np.float64)),
                                     _d(np.ascontiguousarray(phi, np.float64)), _d(out)):
            raise ValueError("not an incremental pressure mode")
        return out

    def surface_traction(self, mark, u, pf):
        """Per fine edge of the marked coarse boundary edges: [x, y, length, Fp_x, Fp_y, Fv_x, Fv_y, 0]."""
        mark = np.ascontiguousarray(mark, np.int32)
        u = np.ascontiguousarray(u, np.float64)
        pf = np.ascontiguousarray(pf, np.float64)
        n = lib().orc_surface_traction(self._h, _i(mark), _d(u), _d(pf), None, 0)
        if n < 0:
            raise ValueError("bad surface")
        out = np.zeros((n, 8))
        lib().orc_surface_traction(self._h, _i(mark), _d(u), _d(pf), _d(out), n)
        return out

    def surface_force(self, mark, u, pf):
        """Force of the fluid on the marked boundary: [pressure x, pressure y, viscous x, viscous y]."""
        out = np.zeros(4)
        if lib().orc_surface_force(self._h, _i(np.ascontiguousarray(mark, np.int32)),
                                   _d(np.ascontiguousarray(u, np.float64)),
                                   _d(np.ascontiguousarray(pf, np.float64)), _d(out)):
            raise ValueError("bad surface")
        return out

    def quad_points(self, level=None):
        """Quadrature points [t][q][2] of the error-norm rule on a level (default: the fine level)."""
        lv = self.levels if level is None else level
        q = int(lib().orc_quad_npts())
        out = np.zeros((self.level_sizes(lv)["t"], q, 2))
        if lib().orc_quad_points(self._h, lv, _d(out)):
            raise ValueError("bad level")
        return out

    def error_norms(self, A, exact, level=None):
        """Eqs. (32)-(33) of the nodal field A ([n] or [n][2]) against the callable exact(xy) -> values."""
        lv = self.levels if level is None else level
        A = np.ascontiguousarray(A, np.float64)
        nc = 1 if A.ndim == 1 else A.shape[1]
        xq = self.quad_points(lv)
        aq = np.ascontiguousarray(exact(xq.reshape(-1, 2)), np.float64)
        an = np.ascontiguousarray(exact(self.export("xy", lv)), np.float64)
        l2, linf = C.c_double(), C.c_double()
        if lib().orc_error_norms(self._h, lv, nc, _d(A), _d(aq), _d(an), C.byref(l2), C.byref(linf)):
            raise ValueError("bad arguments")
        return l2.value, linf.value

    def projection_step(self, g, u, f=None, tol_mom=1e-12, tol_p=1e-12, tol_mass=1e-12, maxit=100000):
        g = np.ascontiguousarray(g, np.float64)
        u = np.array(u, np.float64, order="C")
        pf = np.zeros(self.info["n_f"])
        fa = np.ascontiguousarray(f, np.float64) if f is not None else None
        st = Stats()
        code = lib().orc_projection_step(self._h, _d(g), _d(fa) if fa is not None else None, _d(u), _d(pf),
                                         tol_mom, tol_p, tol_mass, maxit, C.byref(st))
        return u, pf, code, st.asdict()


def _declare_learn(L):
    L.orc_bf16.restype = C.c_double
    L.orc_bf16.argtypes = [C.c_double]
    L.orc_gelu.restype = C.c_double
    L.orc_gelu.argtypes = [C.c_double]
    L.orc_gelu_grad.restype = C.c_double
    L.orc_gelu_grad.argtypes = [C.c_double]
    fp = C.POINTER(C.c_float)
    L.orc_mlp_forward_backward.argtypes = [C.c_int, C.c_int, C.c_int, fp, fp, fp, C.c_int, _dp, _dp, _dp]
    L.orc_adam.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_int, C.c_double, C.c_double, C.c_double, C.c_double]


def jacobi_eigen(A):
    """Eigenvalues (unsorted) and eigenvectors (columns) of a symmetric matrix by the oracle's cyclic Jacobi."""
    A = np.array(A, np.float64, order="C")
    V = np.zeros_like(A)
    lib().orc_jacobi_eigen(A.shape[0], _d(A), _d(V))
    return np.diag(A).copy(), V


def pod(snaps, w, m):
    """POD of the rows of snaps [S][n] in the w-weighted inner product: basis [n][m], energies [m], rank."""
    snaps = np.ascontiguousarray(snaps, np.float64)
    w = np.ascontiguousarray(w, np.float64)
    S, n = snaps.shape
    phi = np.zeros((n, m))
    energy = np.zeros(m)
    rank = lib().orc_pod(S, n, _d(snaps), _d(w), m, _d(phi), _d(energy))
    if rank < 0:
        raise ValueError("bad POD arguments")
    return phi, energy, rank


def bf16(x: float) -> float:
    return lib().orc_bf16(float(x))


def gelu(z: float) -> float:
    return lib().orc_gelu(float(z))


def gelu_grad(z: float) -> float:
    return lib().orc_gelu_grad(float(z))


def mlp_nparams(m: int, h: int) -> int:
    return h * m + h + h * h + h + m * h + m


def mlp(m, h, params, X, T, emulate=True):
    """Loss, outputs [B][m] and parameter gradients of the guess network (FP64, BF16 emulated)."""
    fp = C.POINTER(C.c_float)
    params = np.ascontiguousarray(params, np.float32)
    X = np.ascontiguousarray(X, np.float32)
    T = np.ascontiguousarray(T, np.float32)
    B = X.shape[0]
    loss = C.c_double()
    Y = np.zeros((B, m))
    g = np.zeros(mlp_nparams(m, h))
    lib().orc_mlp_forward_backward(m, h, B, params.ctypes.data_as(fp), X.ctypes.data_as(fp), T.ctypes.data_as(fp),
                                   int(emulate), C.byref(loss), _d(Y), _d(g))
    return loss.value, Y, g


def adam(w, g, m1, m2, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    lib().orc_adam(len(w), _d(w), _d(np.ascontiguousarray(g, np.float64)), _d(m1), _d(m2), t, lr, b1, b2, eps)
