"""Plain FP64 CPU oracle for the Richards-equation Picard / DIC-PCG hot path.

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only callers.  The product library
never imports this package, and this package never imports the product.

The arithmetic lives in ``rf_oracle.c`` (plain C, built with gcc); this module
only builds it and marshals NumPy arrays through ctypes.  Every function
follows a passage of Orgogozo et al. (arXiv:1809.10895):

* ``theta`` / ``capacity`` / ``conductivity`` -- van Genuchten-Mualem
  retention, capacity and conductivity, Sec. 1, Eqs. 2-4 (Gardner's
  conductivity of Appendix A, Eq. A6, with ``model=GARDNER``).
* ``Problem.assemble`` -- the linearised backward-Euler system of one Picard
  iteration: chord-slope capacity, implicit pressure diffusion, explicit
  gravity with arithmetic-mean face conductivity (Sec. 2.2).
* ``Problem.pcg`` / ``dic_apply`` -- DIC-preconditioned conjugate gradients
  (Sec. 2.2).
* ``Problem.step`` -- Picard loop with the global exit test (Sec. 2.2, 2.3).
* ``Problem.run`` -- the EBATS adaptive time stepping (Sec. 2.2).
* ``Problem.mass_balance`` -- storage against cumulative boundary inflow.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rf_oracle.c")
LIB = os.path.join(HERE, "liboracle_rf.so")

VGM, GARDNER = 0, 1
PICARD_CHORD, PICARD_MODIFIED = 0, 1
XMIN, XMAX, YMIN, YMAX, ZMIN, ZMAX = range(6)
NOFLOW, DIRICHLET, FLUX, FREE_DRAINAGE = range(4)
OK, ERR_ARG, ERR_NOT_CONVERGED, ERR_LINEAR, ERR_NONFINITE = 0, -1, -5, -6, -7
MAX_PICARD_LOG = 128


def build(force: bool = True) -> str:
    """Compile rf_oracle.c into liboracle_rf.so (gcc, -O2, FP64, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-fopenmp", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Options(C.Structure):
    _fields_ = [("tol_picard", C.c_double), ("tol_cg", C.c_double),
                ("max_picard", C.c_int), ("max_cg", C.c_int), ("chord_eps", C.c_double),
                ("dt0", C.c_double), ("dt_max", C.c_double), ("dt_min", C.c_double),
                ("ebats", C.c_int), ("inc_after", C.c_int), ("few_iters", C.c_int),
                ("max_iters", C.c_int), ("factor", C.c_double), ("picard_variant", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("converged", C.c_int), ("picard_iters", C.c_int), ("cg_iters_total", C.c_int),
                ("cg_iters", C.c_int * MAX_PICARD_LOG), ("delta", C.c_double * MAX_PICARD_LOG),
                ("dt", C.c_double), ("t", C.c_double)]


class RunStats(C.Structure):
    _fields_ = [("accepted", C.c_int), ("rejected", C.c_int), ("picard_total", C.c_long),
                ("cg_total", C.c_long), ("dt_last", C.c_double), ("t", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        vp = C.c_void_p
        L.orc_theta.restype = C.c_double
        L.orc_theta.argtypes = [C.c_int, C.c_double, dp]
        L.orc_capacity.restype = C.c_double
        L.orc_capacity.argtypes = [C.c_int, C.c_double, dp]
        L.orc_conductivity.restype = C.c_double
        L.orc_conductivity.argtypes = [C.c_int, C.c_double, dp]
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                                 vp, vp]
        L.orc_free.argtypes = [vp]
        L.orc_set_soil.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp]
        L.orc_set_bc.argtypes = [vp, C.c_int, C.c_int, C.c_double]
        L.orc_set_forcing.argtypes = [vp, C.c_int, C.c_int, vp, vp]
        L.orc_set_options.argtypes = [vp, C.POINTER(Options)]
        L.orc_set_state.argtypes = [vp, vp, C.c_double]
        L.orc_get_state.argtypes = [vp, vp, dp]
        L.orc_step.argtypes = [vp, C.c_double, vp, C.POINTER(StepStats)]
        L.orc_run.argtypes = [vp, C.c_double, C.POINTER(RunStats)]
        L.orc_mass_balance.argtypes = [vp, vp]
        L.orc_assemble.argtypes = [vp, vp, C.c_double, vp, vp, vp, vp, vp]
        L.orc_pcg.argtypes = [vp, vp, vp, vp, vp, C.c_double, C.c_int]
        L.orc_matvec.argtypes = [vp, vp, vp, vp, vp]
        L.orc_dic_apply.argtypes = [vp, vp, vp, vp, vp]
        L.orc_eval_cells.argtypes = [vp, vp, vp, vp, vp]
        L.orc_storage.restype = C.c_double
        L.orc_storage.argtypes = [vp, vp]
        L.orc_set_slabs.argtypes = [vp, C.c_int]
        L.orc_picard_iterate.argtypes = [vp, vp, C.c_double, C.c_int, vp]
        L.orc_threads.restype = C.c_int
        L.orc_threads.argtypes = []
        L.orc_time.restype = C.c_double
        L.orc_time.argtypes = [vp]
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [vp]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _params(p):
    return (C.c_double * 6)(*[float(v) for v in p])


def theta(h, p, model=VGM):
    """theta~(h) of Eq. 2 (+ S*h for h >= 0), p = (theta_r, theta_s, alpha, n, Ks, S)."""
    L, pp = lib(), _params(p)
    return np.array([L.orc_theta(model, float(x), pp) for x in np.atleast_1d(h)])


def capacity(h, p, model=VGM):
    """C(h) of Eq. 3."""
    L, pp = lib(), _params(p)
    return np.array([L.orc_capacity(model, float(x), pp) for x in np.atleast_1d(h)])


def conductivity(h, p, model=VGM):
    """K(h) of Eq. 4 (Gardner, Eq. A6, with model=GARDNER)."""
    L, pp = lib(), _params(p)
    return np.array([L.orc_conductivity(model, float(x), pp) for x in np.atleast_1d(h)])


def threads() -> int:
    """OpenMP threads the slab mode uses."""
    return lib().orc_threads()


def step_stats_dict(st: StepStats) -> dict:
    n = min(st.picard_iters, MAX_PICARD_LOG)
    return {"converged": bool(st.converged), "picard_iters": st.picard_iters,
            "cg_iters_total": st.cg_iters_total, "cg_iters": list(st.cg_iters[:n]),
            "delta": list(st.delta[:n]), "dt": st.dt, "t": st.t}


class Problem:
    """One Richards problem on a uniform nx*ny*nz grid (cell k + nz*(i + nx*j))."""

    def __init__(self, nx, ny, nz, dx, dy, dz, ktop=None, grad_elev=None):
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self._ktop = None if ktop is None else np.ascontiguousarray(ktop, dtype=np.int32).ravel()
        self._g = None if grad_elev is None else np.ascontiguousarray(grad_elev, dtype=np.float64)
        self.h = lib().orc_create(nx, ny, nz, dx, dy, dz, _ptr(self._ktop), _ptr(self._g))
        if not self.h:
            raise ValueError("invalid grid")
        self.ktop = (np.full(nx * ny, nz, np.int32) if ktop is None
                     else np.clip(self._ktop, 0, nz))

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_free(self.h)
            self.h = None

    def active_mask(self):
        nx, ny, nz = self.shape
        k = np.arange(nz)[None, :]
        return (k < self.ktop[:, None]).ravel()

    def set_soil(self, params, layer_of_cell=None, lnks=None, model=VGM):
        params = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
        self._layer = None if layer_of_cell is None else np.ascontiguousarray(layer_of_cell, np.uint8)
        self._lnks = None if lnks is None else np.ascontiguousarray(lnks, np.float64)
        s = lib().orc_set_soil(self.h, model, params.shape[0], _ptr(params), _ptr(self._layer),
                               _ptr(self._lnks))
        if s:
            raise ValueError("set_soil failed %d" % s)

    def set_slabs(self, nslab):
        """Slab mode: nslab sub-domains of whole y-rows with block-Jacobi DIC
        (the 'simple' decomposition of Sec. 2.3) and OpenMP threads; 1 = the
        serial method."""
        if lib().orc_set_slabs(self.h, int(nslab)):
            raise ValueError("set_slabs")

    def set_bc(self, face, kind, value=0.0):
        if lib().orc_set_bc(self.h, face, kind, float(value)):
            raise ValueError("set_bc")

    def set_forcing(self, face, t_start, flux):
        t0 = np.ascontiguousarray(t_start, np.float64)
        q = np.ascontiguousarray(flux, np.float64)
        if lib().orc_set_forcing(self.h, face, len(t0), _ptr(t0), _ptr(q)):
            raise ValueError("set_forcing")

    def set_options(self, **kw):
        o = Options(tol_picard=1e-6, tol_cg=1e-8, max_picard=50, max_cg=10000, chord_eps=1e-9,
                    dt0=1.0, dt_max=3600.0, dt_min=1e-6, ebats=1, inc_after=10, few_iters=3,
                    max_iters=8, factor=1.3, picard_variant=0)
        for k, v in kw.items():
            if k not in dict(Options._fields_):
                raise KeyError("unknown oracle option %r" % k)
            setattr(o, k, v)
        lib().orc_set_options(self.h, C.byref(o))

    def set_state(self, h, t=0.0):
        h = np.ascontiguousarray(h, np.float64).ravel()
        assert h.size == self.N
        return lib().orc_set_state(self.h, _ptr(h), float(t))

    def get_state(self):
        h = np.empty(self.N)
        t = C.c_double()
        lib().orc_get_state(self.h, _ptr(h), C.byref(t))
        return h, t.value

    @property
    def t(self):
        return lib().orc_time(self.h)

    @property
    def dt(self):
        return lib().orc_dt(self.h)

    def step(self, dt, guess=None):
        st = StepStats()
        g = None if guess is None else np.ascontiguousarray(guess, np.float64).ravel()
        s = lib().orc_step(self.h, float(dt), _ptr(g), C.byref(st))
        return s, step_stats_dict(st)

    def picard_iterate(self, hn, dt, m):
        """The Picard iterate h^m of a step of size dt from the state hn (at
        the problem's current time): the iterates the step takes, state
        unchanged."""
        hn = np.ascontiguousarray(hn, np.float64).ravel()
        out = np.empty(self.N)
        lib().orc_picard_iterate(self.h, _ptr(hn), float(dt), int(m), _ptr(out))
        return out

    def run(self, t_end):
        rs = RunStats()
        s = lib().orc_run(self.h, float(t_end), C.byref(rs))
        return s, {"accepted": rs.accepted, "rejected": rs.rejected,
                   "picard_total": rs.picard_total, "cg_total": rs.cg_total,
                   "dt_last": rs.dt_last, "t": rs.t}

    def mass_balance(self):
        out = np.zeros(9)
        lib().orc_mass_balance(self.h, _ptr(out))
        return {"storage": out[0], "storage0": out[1], "inflow": out[2:8].copy(),
                "error": out[8]}

    def storage(self, h):
        h = np.ascontiguousarray(h, np.float64)
        return lib().orc_storage(self.h, _ptr(h))

    def eval_cells(self, h):
        h = np.ascontiguousarray(h, np.float64).ravel()
        th, cap, k = np.empty(self.N), np.empty(self.N), np.empty(self.N)
        lib().orc_eval_cells(self.h, _ptr(h), _ptr(th), _ptr(cap), _ptr(k))
        return th, cap, k

    def assemble(self, hm, dt):
        hm = np.ascontiguousarray(hm, np.float64).ravel()
        N = self.N
        diag, off, b, K, Cc = (np.empty(N), np.empty(6 * N), np.empty(N), np.empty(N),
                               np.empty(N))
        s = lib().orc_assemble(self.h, _ptr(hm), float(dt), _ptr(diag), _ptr(off), _ptr(b),
                               _ptr(K), _ptr(Cc))
        if s:
            raise ValueError("assemble")
        return {"diag": diag, "off": off.reshape(6, N), "b": b, "K": K, "C": Cc}

    def matvec(self, sysd, x):
        y = np.empty(self.N)
        x = np.ascontiguousarray(x, np.float64)
        off = np.ascontiguousarray(sysd["off"]).ravel()
        lib().orc_matvec(self.h, _ptr(sysd["diag"]), _ptr(off), _ptr(x), _ptr(y))
        return y

    def dic_apply(self, sysd, r):
        z = np.empty(self.N)
        r = np.ascontiguousarray(r, np.float64)
        off = np.ascontiguousarray(sysd["off"]).ravel()
        s = lib().orc_dic_apply(self.h, _ptr(sysd["diag"]), _ptr(off), _ptr(r), _ptr(z))
        if s:
            raise ValueError("DIC breakdown")
        return z

    def pcg(self, sysd, x0, tol, max_it=100000):
        x = np.array(x0, np.float64, copy=True)
        off = np.ascontiguousarray(sysd["off"]).ravel()
        its = lib().orc_pcg(self.h, _ptr(sysd["diag"]), _ptr(off), _ptr(sysd["b"]), _ptr(x),
                            float(tol), int(max_it))
        return x, its

    def dense_matrix(self, sysd):
        """The assembled operator as a dense matrix (tiny grids only)."""
        N = self.N
        A = np.zeros((N, N))
        for c in range(N):
            e = np.zeros(N)
            e[c] = 1.0
            A[:, c] = self.matvec(sysd, e)
        return A
