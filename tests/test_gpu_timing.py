"""Host-side step machinery.  Per-kernel timing (rf_set_timing /
rf_get_timing): each launch that did work is counted once under its kernel,
launches enqueued ahead of need that returned at once are counted apart,
durations are positive and add up to no more than the wall time of the
steps, and timing changes no result.  The host's two ways of waiting for a
step (polling, blocking) give the same results."""
import time

import numpy as np
import pytest

from paper_1809_10895_amd import workloads as W
from tests.common import make_solver

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def small_hillslope():
    return W.hillslope(nx=24, ny=20, nz=40, seed=3)


@pytest.mark.parametrize("precision", [0, 1])
def test_timing_counts_every_working_launch(precision):
    w = small_hillslope()
    S = make_solver(w, precond=1, tol_cg=1e-8, precision=precision)
    assert S.step(w.dt)[0] == 0
    S.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nstep, picard, cg = 4, 0, 0
    for _ in range(nstep):
        s, st = S.step(w.dt)
        assert s == 0, S.last_error()
        picard += st["picard_iters"]
        cg += st["cg_iters_total"]
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    tm = S.get_timing()
    assert tm["cells"] == int(w.active_mask().sum())
    assert tm["begin"]["launches"] == nstep
    assert tm["accept"]["launches"] == nstep
    assert tm["coeff"]["launches"] == picard
    assert tm["resid"]["launches"] == picard
    assert tm["spmv"]["launches"] == cg
    assert tm["update"]["launches"] == cg
    assert tm["apply_h"]["launches"] == picard
    kernels = [v for v in tm.values() if isinstance(v, dict)]
    for v in kernels:
        if v["launches"]:
            assert v["ms"] > 0.0
        assert v["ms"] >= 0.0 and v["idle_ms"] >= 0.0
    assert sum(v["ms"] + v["idle_ms"] for v in kernels) <= wall_ms


def test_timing_changes_no_result():
    w = small_hillslope()
    out = []
    for mask in (False, True, ["update"]):
        S = make_solver(w, precond=1, tol_cg=1e-8)
        S.set_timing(mask)
        for _ in range(3):
            assert S.step(w.dt)[0] == 0, S.last_error()
        out.append(S.get_state()[0].cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_timing_reset_and_off():
    w = small_hillslope()
    S = make_solver(w, precond=1, tol_cg=1e-8)
    S.set_timing(["spmv", "update"])
    assert S.step(w.dt)[0] == 0
    tm = S.get_timing()
    assert tm["spmv"]["launches"] > 0 and tm["coeff"]["launches"] == 0
    S.set_timing(False)
    assert S.step(w.dt)[0] == 0
    tm = S.get_timing()
    assert all(v["launches"] == 0 and v["idle_launches"] == 0
               for v in tm.values() if isinstance(v, dict))


def test_host_wait_modes_agree():
    from paper_1809_10895_amd.binding import RF_WAIT_BLOCK, RF_WAIT_SPIN
    w = small_hillslope()
    out = []
    for mode in (RF_WAIT_SPIN, RF_WAIT_BLOCK):
        S = make_solver(w, precond=1, tol_cg=1e-8, host_wait=mode)
        for _ in range(3):
            assert S.step(w.dt)[0] == 0, S.last_error()
        s, rs = S.run(S.get_state()[1] + 2 * w.dt)
        assert s == 0, S.last_error()
        out.append(S.get_state()[0].cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_select_timing_keeps_counters_and_times_a_sample():
    w = small_hillslope()
    S = make_solver(w, precond=1, tol_cg=1e-8)
    assert S.step(w.dt)[0] == 0
    S.set_timing(["update"])
    cg_timed = 0
    for i in range(6):
        S.select_timing(["update"] if i % 3 == 0 else False)
        s, st = S.step(w.dt)
        assert s == 0, S.last_error()
        if i % 3 == 0:
            cg_timed += st["cg_iters_total"]
    tm = S.get_timing()
    assert tm["update"]["launches"] == cg_timed and tm["update"]["ms"] > 0.0
    assert tm["spmv"]["launches"] == 0
    # a stride: steps 0, 3, 6 of nine
    S.select_timing(["update"], every=3)
    for i in range(9):
        s, st = S.step(w.dt)
        assert s == 0, S.last_error()
        if i % 3 == 0:
            cg_timed += st["cg_iters_total"]
    assert S.get_timing()["update"]["launches"] == cg_timed
