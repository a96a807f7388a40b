"""rf_bind_static_workspace (the entry point that allocates nothing): the
library's static device workspace bound in place of a caller's buffer gives
the same steps, bit for bit, as rf_bind_workspace with a torch buffer; two
binds in a row, the second on a smaller grid; and a grid too large for it is
refused."""
import numpy as np
import pytest

from paper_1809_10895_amd import Solver, workloads as W
from tests.common import PARITY_OPTS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _solver(w, static):
    S = Solver()
    S.setup_grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.ktop, w.grad_elev)
    W.configure(w, S)
    S.set_options(**dict(PARITY_OPTS, dt0=w.dt, dt_max=w.dt_max, ebats=1))
    if static:
        assert S.bind_static() == 0, S.last_error()
    else:
        S.bind()
    assert S.set_state(torch.tensor(w.h0, dtype=torch.float64, device="cuda")) == 0, S.last_error()
    return S


def _run(S, t_end):
    s, rs = S.run(t_end)
    assert s == 0, S.last_error()
    h, t = S.get_state()
    return rs, h.cpu().numpy(), t, S.mass_balance()


@pytest.mark.parametrize("shape", [(24, 20, 48), (13, 9, 30)])   # the second call is smaller
def test_static_workspace_equals_caller_workspace(shape):
    nx, ny, nz = shape
    w = W.watershed(nx=nx, ny=ny, nz=nz, kmin=nz // 2)
    w.h0 = np.where(w.active_mask(), -1.5, 0.0)
    ref = _run(_solver(w, static=False), 3 * 3600.0)
    S = _solver(w, static=True)
    got = _run(S, 3 * 3600.0)
    assert got[0] == ref[0]                              # accepted, rejected, Picard, PCG totals
    assert np.array_equal(got[1], ref[1])                # heads bit for bit
    assert got[2] == ref[2]
    assert got[3] == ref[3]                              # water balance
    assert ref[0]["accepted"] > 5 and ref[0]["picard_total"] > ref[0]["accepted"]


def test_static_workspace_refuses_a_grid_too_large():
    w = W.hillslope(nx=64, ny=64, nz=64)                 # 262144 cells: fits
    S = Solver()
    S.setup_grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz)
    W.configure(w, S)
    assert S.bind_static() == 0, S.last_error()
    S2 = Solver()
    S2.setup_grid(128, 128, 64, 1.0, 1.0, 0.1)           # 1 M cells: about 150 MB of workspace
    S2.set_soil(np.array([W.SOIL_HILLSLOPE]))
    assert S2.bind_static() == -4                         # RF_ERR_NOMEM
    assert "needed" in S2.last_error()
