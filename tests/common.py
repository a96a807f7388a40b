"""Helpers shared by the tests: build the oracle and the GPU solver from one
seeded workload, and compare states."""
import numpy as np

from paper_1809_10895_amd import workloads as W

PARITY_OPTS = dict(tol_picard=1e-6, tol_cg=1e-13, max_picard=100, max_cg=20000)


def make_oracle(orc, w, **opts):
    P = orc.Problem(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, ktop=w.ktop, grad_elev=w.grad_elev)
    W.configure(w, P)
    o = dict(PARITY_OPTS, dt0=w.dt, dt_max=w.dt_max, ebats=int(w.ebats))
    o.update(opts)
    P.set_options(**o)
    assert P.set_state(w.h0) == 0
    return P


def make_solver(w, precond=1, **opts):
    import torch
    from paper_1809_10895_amd import Solver
    S = Solver()
    S.setup_grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.ktop, w.grad_elev)
    W.configure(w, S)
    o = dict(PARITY_OPTS, dt0=w.dt, dt_max=w.dt_max, ebats=int(w.ebats), precond=precond)
    o.update(opts)
    S.set_options(**o)
    S.bind()
    h0 = torch.tensor(w.h0, dtype=torch.float64, device="cuda")
    assert S.set_state(h0) == 0, S.last_error()
    return S


def rel_err(h_gpu, h_ref, mask):
    """max |h_gpu - h_ref| / max(max |h_ref|, 1 m) over active cells."""
    d = np.abs(h_gpu[mask] - h_ref[mask]).max() if mask.any() else 0.0
    return d / max(np.abs(h_ref[mask]).max(), 1.0)
