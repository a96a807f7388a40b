"""ctypes binding of the C ABI declared in include/rf.h.

Argument marshalling only: every step of the Picard / PCG loop runs in the
HIP kernels of librf_mi355x.so.  PyTorch provides device memory (the
workspace and the state tensors) and the HIP stream.  Importing this module
does not need a GPU; creating a Solver does, and fails loudly if the library
has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "librf_mi355x.so")

RF_OK, RF_ERR_ARG, RF_ERR_STATE, RF_ERR_HIP, RF_ERR_NOMEM = 0, -1, -2, -3, -4
RF_ERR_NOT_CONVERGED, RF_ERR_LINEAR, RF_ERR_NONFINITE = -5, -6, -7
RF_VGM, RF_GARDNER = 0, 1
RF_XMIN, RF_XMAX, RF_YMIN, RF_YMAX, RF_ZMIN, RF_ZMAX = range(6)
RF_NOFLOW, RF_DIRICHLET, RF_FLUX, RF_FREE_DRAINAGE = range(4)
RF_PRECOND_JACOBI, RF_PRECOND_ZLINE = 0, 1
RF_PREC_FP64, RF_PREC_MIXED = 0, 1
RF_PICARD_CHORD, RF_PICARD_MODIFIED = 0, 1
RF_FIRST_PREVIOUS, RF_FIRST_EXTRAPOLATE = 0, 1
RF_REFACTOR_EVERY, RF_REFACTOR_STEP = 0, 1
RF_WAIT_SPIN, RF_WAIT_BLOCK = 0, 1
RF_STENCIL_COLUMNS, RF_STENCIL_TILES, RF_STENCIL_AUTO = 0, 1, 2
RF_MAX_PICARD_LOG = 128
RF_NKERNELS = 8

STATUS_NAMES = {0: "RF_OK", -1: "RF_ERR_ARG", -2: "RF_ERR_STATE", -3: "RF_ERR_HIP",
                -4: "RF_ERR_NOMEM", -5: "RF_ERR_NOT_CONVERGED", -6: "RF_ERR_LINEAR",
                -7: "RF_ERR_NONFINITE"}

# Every function the header declares (checked against include/rf.h by the tests).
EXPORTS = ["rf_default_options", "rf_create", "rf_destroy", "rf_last_error", "rf_setup_grid",
           "rf_set_soil", "rf_set_bc", "rf_set_forcing", "rf_set_options", "rf_workspace_bytes",
           "rf_bind_workspace", "rf_set_state", "rf_get_state", "rf_step", "rf_run",
           "rf_run_steps", "rf_bind_static_workspace", "rf_mass_balance", "rf_eval_soil", "rf_assemble", "rf_apply_operator",
           "rf_apply_precond", "rf_set_timing", "rf_select_timing", "rf_get_timing",
           # include/rf_ensemble.h
           "rf_ens_create", "rf_ens_destroy", "rf_ens_last_error", "rf_ens_setup", "rf_ens_set_bc",
           "rf_ens_set_options", "rf_ens_set_tile", "rf_ens_set_limits", "rf_ens_get_tile",
           "rf_ens_cells", "rf_ens_workspace_bytes", "rf_ens_bind_workspace", "rf_ens_set_state",
           "rf_ens_get_state", "rf_ens_run", "rf_ens_get_columns", "rf_ens_autotune",
           # include/rf_guess.h
           "rf_guess_create", "rf_guess_destroy", "rf_guess_last_error", "rf_guess_setup",
           "rf_guess_workspace_bytes", "rf_guess_bind_workspace", "rf_guess_param_count",
           "rf_guess_set_params", "rf_guess_get_params", "rf_guess_predict", "rf_guess_gradient",
           "rf_guess_train_step"]
RF_ENS_MAX_LEN = 448


class RfOptions(C.Structure):
    _fields_ = [("tol_picard", C.c_double), ("tol_cg", C.c_double), ("max_picard", C.c_int),
                ("max_cg", C.c_int), ("chord_eps", C.c_double), ("precond", C.c_int),
                ("check_every", C.c_int), ("dt0", C.c_double), ("dt_max", C.c_double),
                ("dt_min", C.c_double), ("ebats", C.c_int), ("inc_after", C.c_int),
                ("few_iters", C.c_int), ("max_iters", C.c_int), ("factor", C.c_double),
                ("cols_per_wave", C.c_int), ("precision", C.c_int), ("cg_rel_tol", C.c_double),
                ("picard_variant", C.c_int), ("first_iterate", C.c_int), ("zline_refactor", C.c_int),
                ("host_wait", C.c_int), ("stencil", C.c_int), ("tile_rows", C.c_int)]


class RfStepStats(C.Structure):
    _fields_ = [("converged", C.c_int), ("picard_iters", C.c_int), ("cg_iters_total", C.c_int),
                ("cg_iters", C.c_int * RF_MAX_PICARD_LOG),
                ("delta", C.c_double * RF_MAX_PICARD_LOG), ("dt", C.c_double), ("t", C.c_double)]


class RfRunStats(C.Structure):
    _fields_ = [("accepted", C.c_int), ("rejected", C.c_int), ("picard_total", C.c_long),
                ("cg_total", C.c_long), ("dt_last", C.c_double), ("t", C.c_double)]


class RfMass(C.Structure):
    _fields_ = [("storage", C.c_double), ("storage0", C.c_double), ("inflow", C.c_double * 6),
                ("error", C.c_double)]


class RfTiming(C.Structure):
    _fields_ = [("name", C.c_char_p * RF_NKERNELS), ("launches", C.c_long * RF_NKERNELS),
                ("ms", C.c_double * RF_NKERNELS), ("idle_launches", C.c_long * RF_NKERNELS),
                ("idle_ms", C.c_double * RF_NKERNELS), ("cells", C.c_long)]


class RfEnsTile(C.Structure):
    _fields_ = [("waves_per_block", C.c_int), ("blocks_per_cu", C.c_int)]


class RfEnsColumn(C.Structure):
    _fields_ = [("status", C.c_int), ("accepted", C.c_int), ("rejected", C.c_int),
                ("easy", C.c_int), ("picard_total", C.c_long), ("t", C.c_double),
                ("dt_next", C.c_double), ("storage0", C.c_double), ("storage", C.c_double),
                ("inflow_top", C.c_double), ("inflow_bottom", C.c_double)]


class RfEnsSummary(C.Structure):
    _fields_ = [("accepted", C.c_long), ("rejected", C.c_long), ("picard_total", C.c_long),
                ("cell_steps", C.c_long), ("failed", C.c_int), ("t_min", C.c_double),
                ("max_balance_error", C.c_double), ("kernel_ms", C.c_double)]


class RfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def load_library(path: str = LIB):
    """Loads librf_mi355x.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("HIP library %s is missing: build it with __graft_entry__.build()" % path)
    L = C.CDLL(path)
    vp, dp, ip = C.c_void_p, C.c_double, C.c_int
    L.rf_default_options.argtypes = [C.POINTER(RfOptions)]
    L.rf_default_options.restype = None
    L.rf_create.argtypes = [C.POINTER(vp), ip, vp]
    L.rf_destroy.argtypes = [vp]
    L.rf_destroy.restype = None
    L.rf_last_error.argtypes = [vp]
    L.rf_last_error.restype = C.c_char_p
    L.rf_setup_grid.argtypes = [vp, ip, ip, ip, dp, dp, dp, vp, vp]
    L.rf_set_soil.argtypes = [vp, ip, ip, vp, vp, vp]
    L.rf_set_bc.argtypes = [vp, ip, ip, dp]
    L.rf_set_forcing.argtypes = [vp, ip, ip, vp, vp]
    L.rf_set_options.argtypes = [vp, C.POINTER(RfOptions)]
    L.rf_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.rf_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    L.rf_set_state.argtypes = [vp, vp, dp]
    L.rf_get_state.argtypes = [vp, vp, C.POINTER(C.c_double)]
    L.rf_step.argtypes = [vp, dp, vp, C.POINTER(RfStepStats)]
    L.rf_run.argtypes = [vp, dp, C.POINTER(RfRunStats)]
    L.rf_run_steps.argtypes = [vp, dp, C.c_long, C.POINTER(RfRunStats)]
    L.rf_bind_static_workspace.argtypes = [vp]
    L.rf_mass_balance.argtypes = [vp, C.POINTER(RfMass)]
    L.rf_eval_soil.argtypes = [vp, vp, vp, vp, vp]
    L.rf_assemble.argtypes = [vp, vp, dp, vp, vp]
    L.rf_apply_operator.argtypes = [vp, vp, vp]
    L.rf_apply_precond.argtypes = [vp, vp, vp]
    L.rf_set_timing.argtypes = [vp, ip]
    L.rf_select_timing.argtypes = [vp, ip, ip]
    L.rf_get_timing.argtypes = [vp, C.POINTER(RfTiming)]
    L.rf_ens_create.argtypes = [C.POINTER(vp), ip, vp]
    L.rf_ens_destroy.argtypes = [vp]
    L.rf_ens_last_error.argtypes = [vp]
    L.rf_ens_last_error.restype = C.c_char_p
    L.rf_ens_setup.argtypes = [vp, ip, vp, dp, ip, vp]
    L.rf_ens_set_bc.argtypes = [vp, ip, ip, dp]
    L.rf_ens_set_options.argtypes = [vp, C.POINTER(RfOptions)]
    L.rf_ens_set_tile.argtypes = [vp, C.POINTER(RfEnsTile)]
    L.rf_ens_set_limits.argtypes = [vp, C.c_long, dp]
    L.rf_ens_get_tile.argtypes = [vp, C.POINTER(RfEnsTile)]
    L.rf_ens_cells.argtypes = [vp, C.POINTER(C.c_long)]
    L.rf_ens_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.rf_ens_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    L.rf_ens_set_state.argtypes = [vp, vp, dp]
    L.rf_ens_get_state.argtypes = [vp, vp]
    L.rf_ens_run.argtypes = [vp, dp, C.POINTER(RfEnsSummary)]
    L.rf_ens_get_columns.argtypes = [vp, C.POINTER(RfEnsColumn)]
    L.rf_ens_autotune.argtypes = [vp, dp, C.POINTER(RfEnsTile)]
    L.rf_guess_create.argtypes = [C.POINTER(vp), ip, vp]
    L.rf_guess_destroy.argtypes = [vp]
    L.rf_guess_last_error.argtypes = [vp]
    L.rf_guess_last_error.restype = C.c_char_p
    L.rf_guess_setup.argtypes = [vp, ip, ip, ip, C.c_uint]
    L.rf_guess_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.rf_guess_bind_workspace.argtypes = [vp, vp, C.c_size_t]
    L.rf_guess_param_count.argtypes = []
    L.rf_guess_param_count.restype = C.c_size_t
    L.rf_guess_set_params.argtypes = [vp, vp]
    L.rf_guess_get_params.argtypes = [vp, vp]
    L.rf_guess_predict.argtypes = [vp, vp, vp, vp, dp, vp]
    L.rf_guess_gradient.argtypes = [vp, vp, vp, vp, dp, vp, C.POINTER(C.c_double), vp]
    L.rf_guess_train_step.argtypes = [vp, vp, vp, vp, dp, vp, dp, C.POINTER(C.c_double)]
    for name in EXPORTS:
        if name not in ("rf_default_options", "rf_destroy", "rf_last_error", "rf_ens_last_error",
                        "rf_guess_last_error", "rf_guess_param_count"):
            getattr(L, name).restype = C.c_int      # rf_status
    _lib = L
    return L


def default_options() -> dict:
    o = RfOptions()
    load_library().rf_default_options(C.byref(o))
    return {name: getattr(o, name) for name, _ in RfOptions._fields_}


def step_stats_dict(st: RfStepStats) -> dict:
    n = min(st.picard_iters, RF_MAX_PICARD_LOG)
    return {"converged": bool(st.converged), "picard_iters": st.picard_iters,
            "cg_iters_total": st.cg_iters_total, "cg_iters": list(st.cg_iters[:n]),
            "delta": list(st.delta[:n]), "dt": st.dt, "t": st.t}


def _ptr(t):
    """Device pointer of a CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return C.c_void_p(t.data_ptr())


def _host(a, dtype):
    import numpy as np
    if a is None:
        return None, None
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr, arr.ctypes.data_as(C.c_void_p)


class Solver:
    """One problem on one GPU: grid, soil, boundary conditions, state."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.L = load_library()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        s = self.L.rf_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if s != RF_OK:
            raise RfError(s, "rf_create failed")
        self.h = h
        self.ws = None
        self.shape = None

    def close(self):
        if getattr(self, "h", None):
            self.L.rf_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, s):
        if s != RF_OK:
            raise RfError(s, self.L.rf_last_error(self.h).decode())
        return s

    def last_error(self) -> str:
        return self.L.rf_last_error(self.h).decode()

    # --- set-up -------------------------------------------------------------
    def setup_grid(self, nx, ny, nz, dx, dy, dz, ktop=None, grad_elev=None):
        import numpy as np
        kt, ktp = _host(ktop, np.int32)
        g, gp = _host(grad_elev, np.float64)
        self._check(self.L.rf_setup_grid(self.h, nx, ny, nz, dx, dy, dz, ktp, gp))
        self.shape = (nx, ny, nz)
        self.N = nx * ny * nz
        self.ws = None

    def set_soil(self, params, layer_of_cell=None, ln_ks_offset=None, model=RF_VGM):
        import numpy as np
        p = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
        lay, layp = _host(layer_of_cell, np.uint8)
        lk, lkp = _host(ln_ks_offset, np.float64)
        self._check(self.L.rf_set_soil(self.h, model, p.shape[0], p.ctypes.data_as(C.c_void_p),
                                       layp, lkp))

    def set_bc(self, face, kind, value=0.0):
        self._check(self.L.rf_set_bc(self.h, face, kind, float(value)))

    def set_forcing(self, face, t_start, flux):
        import numpy as np
        t0, t0p = _host(t_start, np.float64)
        q, qp = _host(flux, np.float64)
        self._check(self.L.rf_set_forcing(self.h, face, len(t0), t0p, qp))

    def set_options(self, **kw):
        o = RfOptions()
        self.L.rf_default_options(C.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self._check(self.L.rf_set_options(self.h, C.byref(o)))

    def workspace_bytes(self) -> int:
        n = C.c_size_t()
        self._check(self.L.rf_workspace_bytes(self.h, C.byref(n)))
        return n.value

    def bind(self):
        nbytes = self.workspace_bytes()
        self.ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        self._check(self.L.rf_bind_workspace(self.h, _ptr(self.ws), nbytes))

    def bind_static(self):
        """rf_bind_static_workspace: the library's own static workspace; returns the status."""
        self.ws = None
        return self.L.rf_bind_static_workspace(self.h)

    # --- state --------------------------------------------------------------
    def set_state(self, h, t=0.0):
        return self.L.rf_set_state(self.h, _ptr(h), float(t))

    def get_state(self, out=None):
        if out is None:
            out = self.torch.empty(self.N, dtype=self.torch.float64, device=self.device)
        t = C.c_double()
        self._check(self.L.rf_get_state(self.h, _ptr(out), C.byref(t)))
        return out, t.value

    def step(self, dt, guess=None):
        st = RfStepStats()
        s = self.L.rf_step(self.h, float(dt), _ptr(guess), C.byref(st))
        return s, step_stats_dict(st)

    def run(self, t_end, max_steps=None):
        """rf_run to t_end, or rf_run_steps when max_steps (accepted steps) is given."""
        rs = RfRunStats()
        if max_steps is None:
            s = self.L.rf_run(self.h, float(t_end), C.byref(rs))
        else:
            s = self.L.rf_run_steps(self.h, float(t_end), int(max_steps), C.byref(rs))
        return s, {"accepted": rs.accepted, "rejected": rs.rejected,
                   "picard_total": rs.picard_total, "cg_total": rs.cg_total,
                   "dt_last": rs.dt_last, "t": rs.t}

    def mass_balance(self):
        m = RfMass()
        self._check(self.L.rf_mass_balance(self.h, C.byref(m)))
        return {"storage": m.storage, "storage0": m.storage0, "inflow": list(m.inflow),
                "error": m.error}

    # --- building blocks ----------------------------------------------------
    def eval_soil(self, h):
        t = self.torch
        th, cap, k = (t.full((self.N,), float("nan"), dtype=t.float64, device=self.device)
                      for _ in range(3))
        self._check(self.L.rf_eval_soil(self.h, _ptr(h), _ptr(th), _ptr(cap), _ptr(k)))
        return th, cap, k

    def assemble(self, hm, dt):
        t = self.torch
        diag, rhs = (t.full((self.N,), float("nan"), dtype=t.float64, device=self.device)
                     for _ in range(2))
        self._check(self.L.rf_assemble(self.h, _ptr(hm), float(dt), _ptr(diag), _ptr(rhs)))
        return diag, rhs

    def apply_operator(self, x):
        y = self.torch.full((self.N,), float("nan"), dtype=self.torch.float64, device=self.device)
        self._check(self.L.rf_apply_operator(self.h, _ptr(x), _ptr(y)))
        return y

    def apply_precond(self, r):
        z = self.torch.full((self.N,), float("nan"), dtype=self.torch.float64, device=self.device)
        self._check(self.L.rf_apply_precond(self.h, _ptr(r), _ptr(z)))
        return z

    # --- measurement --------------------------------------------------------
    KERNELS = ("coeff", "resid", "spmv", "update", "apply_h", "accept", "decide", "begin")

    def _timing_mask(self, kernels):
        if kernels is True:
            return 0xff
        mask = 0
        for k in (kernels or ()):
            mask |= 1 << self.KERNELS.index(k)
        return mask

    def set_timing(self, kernels=True):
        """kernels: True (all), False/None (off) or an iterable of kernel names."""
        self._check(self.L.rf_set_timing(self.h, self._timing_mask(kernels)))

    def select_timing(self, kernels=True, every=1):
        """Like set_timing, in the next step planned and every `every`-th one
        after it, keeping the counters."""
        self._check(self.L.rf_select_timing(self.h, self._timing_mask(kernels), int(every)))

    def get_timing(self) -> dict:
        tm = RfTiming()
        self._check(self.L.rf_get_timing(self.h, C.byref(tm)))
        out = {"cells": tm.cells}
        for k in range(RF_NKERNELS):
            name = tm.name[k].decode() if tm.name[k] else ""
            if name:
                out[name] = {"launches": tm.launches[k], "ms": tm.ms[k],
                             "idle_launches": tm.idle_launches[k], "idle_ms": tm.idle_ms[k]}
        return out


def _struct_dict(st):
    return {name: getattr(st, name) for name, _ in st._fields_}


class Ensemble:
    """Many independent 1-D columns (include/rf_ensemble.h) on one GPU.

    lengths: cells per column; soil: ncol x 6 (theta_r, theta_s, alpha, n,
    Ks, S); the packed state is column after column, bottom cell first."""

    def __init__(self, lengths, dz, soil, model=RF_VGM, device: int = 0, stream=None):
        import numpy as np
        import torch
        self.torch = torch
        self.L = load_library()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        s = self.L.rf_ens_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if s != RF_OK:
            raise RfError(s, "rf_ens_create failed")
        self.h = h
        self.lengths = np.ascontiguousarray(lengths, dtype=np.int32)
        self.offsets = np.concatenate([[0], np.cumsum(self.lengths)[:-1]]).astype(np.int64)
        sp = np.ascontiguousarray(np.atleast_2d(soil), dtype=np.float64)
        self._check(self.L.rf_ens_setup(self.h, len(self.lengths),
                                        self.lengths.ctypes.data_as(C.c_void_p), float(dz), model,
                                        sp.ctypes.data_as(C.c_void_p)))
        n = C.c_long()
        self._check(self.L.rf_ens_cells(self.h, C.byref(n)))
        self.ncell = n.value
        self.ncol = len(self.lengths)
        self.ws = None

    def close(self):
        if getattr(self, "h", None):
            self.L.rf_ens_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, s):
        if s != RF_OK:
            raise RfError(s, self.L.rf_ens_last_error(self.h).decode())
        return s

    def last_error(self) -> str:
        return self.L.rf_ens_last_error(self.h).decode()

    def set_bc(self, face, kind, value=0.0):
        self._check(self.L.rf_ens_set_bc(self.h, face, kind, float(value)))

    def set_options(self, **kw):
        o = RfOptions()
        self.L.rf_default_options(C.byref(o))
        for k, v in kw.items():
            if not hasattr(o, k):
                raise KeyError(k)
            setattr(o, k, v)
        self._check(self.L.rf_ens_set_options(self.h, C.byref(o)))

    def set_tile(self, waves_per_block, blocks_per_cu=0):
        t = RfEnsTile(waves_per_block, blocks_per_cu)
        self._check(self.L.rf_ens_set_tile(self.h, C.byref(t)))

    def get_tile(self):
        t = RfEnsTile()
        self._check(self.L.rf_ens_get_tile(self.h, C.byref(t)))
        return (t.waves_per_block, t.blocks_per_cu)

    def set_limits(self, max_steps, max_seconds):
        self._check(self.L.rf_ens_set_limits(self.h, int(max_steps), float(max_seconds)))

    def bind(self):
        n = C.c_size_t()
        self._check(self.L.rf_ens_workspace_bytes(self.h, C.byref(n)))
        self.ws = self.torch.empty(n.value, dtype=self.torch.uint8, device=self.device)
        self._check(self.L.rf_ens_bind_workspace(self.h, _ptr(self.ws), n.value))

    def set_state(self, h, t=0.0):
        return self.L.rf_ens_set_state(self.h, _ptr(h), float(t))

    def get_state(self):
        out = self.torch.empty(self.ncell, dtype=self.torch.float64, device=self.device)
        self._check(self.L.rf_ens_get_state(self.h, _ptr(out)))
        return out

    def run(self, t_end):
        sm = RfEnsSummary()
        s = self.L.rf_ens_run(self.h, float(t_end), C.byref(sm))
        return s, _struct_dict(sm)

    def columns(self):
        arr = (RfEnsColumn * self.ncol)()
        self._check(self.L.rf_ens_get_columns(self.h, arr))
        return [_struct_dict(c) for c in arr]

    def autotune(self, t_span):
        t = RfEnsTile()
        s = self.L.rf_ens_autotune(self.h, float(t_span), C.byref(t))
        return s, (t.waves_per_block, t.blocks_per_cu)


class Guess:
    """The learned Picard initial guess (include/rf_guess.h) on one grid."""

    def __init__(self, nx, ny, nz, seed=0, device: int = 0, stream=None):
        import torch
        self.torch = torch
        self.L = load_library()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        s = self.L.rf_guess_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if s != RF_OK:
            raise RfError(s, "rf_guess_create failed")
        self.h = h
        self.N = nx * ny * nz
        self.shape = (nx, ny, nz)
        self._check(self.L.rf_guess_setup(self.h, nx, ny, nz, seed))
        n = C.c_size_t()
        self._check(self.L.rf_guess_workspace_bytes(self.h, C.byref(n)))
        self.ws = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        self._check(self.L.rf_guess_bind_workspace(self.h, _ptr(self.ws), n.value))
        self.nparams = self.L.rf_guess_param_count()

    def close(self):
        if getattr(self, "h", None):
            self.L.rf_guess_destroy(self.h)
            self.h = None

    __del__ = close

    def _check(self, s):
        if s != RF_OK:
            raise RfError(s, self.L.rf_guess_last_error(self.h).decode())
        return s

    def set_params(self, p):
        import numpy as np
        a = np.ascontiguousarray(p, dtype=np.float32)
        assert a.size == self.nparams
        self._check(self.L.rf_guess_set_params(self.h, a.ctypes.data_as(C.c_void_p)))

    def get_params(self):
        import numpy as np
        a = np.empty(self.nparams, np.float32)
        self._check(self.L.rf_guess_get_params(self.h, a.ctypes.data_as(C.c_void_p)))
        return a

    def predict(self, hn, hprev, lnks, rain, out=None):
        if out is None:
            out = self.torch.empty(self.N, dtype=self.torch.float64, device=self.device)
        self._check(self.L.rf_guess_predict(self.h, _ptr(hn), _ptr(hprev), _ptr(lnks), float(rain),
                                            _ptr(out)))
        return out

    def gradient(self, hn, hprev, lnks, rain, target):
        import numpy as np
        g = np.empty(self.nparams, np.float32)
        loss = C.c_double()
        self._check(self.L.rf_guess_gradient(self.h, _ptr(hn), _ptr(hprev), _ptr(lnks), float(rain),
                                             _ptr(target), C.byref(loss), g.ctypes.data_as(C.c_void_p)))
        return loss.value, g

    def train_step(self, hn, hprev, lnks, rain, target, lr):
        loss = C.c_double()
        self._check(self.L.rf_guess_train_step(self.h, _ptr(hn), _ptr(hprev), _ptr(lnks), float(rain),
                                               _ptr(target), float(lr), C.byref(loss)))
        return loss.value
