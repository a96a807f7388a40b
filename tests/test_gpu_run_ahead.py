"""rf_run with fixed steps enqueues each step before it waits for the step
ahead of it; on the device the new step starts only if that step was
accepted by the work enqueued for it up front, and otherwise does nothing and
is enqueued again.  Its states, statistics and water balance must equal those
of one rf_step call per step: with a jump in the rain rate (a step that needs
more Picard and PCG work than the one before it, so the step behind it finds
it not yet accepted), steps clipped at that forcing change and at t_end, the
extrapolated first iterate, mixed precision, a grid whose reductions need the
fold kernel, timing of a sample of the steps, and a step that fails."""
import math

import numpy as np
import pytest

from paper_1809_10895_amd import workloads as W
from tests.common import make_solver

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def rainy(nx=24, ny=20, nz=40, jump=3.5, q2=2e-6):
    """Small hillslope whose rain rises from 1e-7 to q2 m/s at jump * dt."""
    w = W.hillslope(nx=nx, ny=ny, nz=nz, seed=3)
    w.forcing = {W.ZMAX: (np.array([0.0, jump * w.dt]), np.array([1e-7, q2]))}
    return w


def before(t, t_end):
    return t < t_end * (1.0 - 1e-15) - 1e-12


def fixed_dt(w, t, t_end):
    """The fixed-step rule: dt0 clipped at the next forcing change and t_end."""
    dt = w.dt
    tf = math.inf
    for s in w.forcing[W.ZMAX][0]:
        if s > t * (1.0 + 1e-15) + 1e-12 and s < tf:
            tf = float(s)
    if t + dt > tf:
        dt = tf - t
    if t + dt > t_end:
        dt = t_end - t
    return dt


def by_steps(w, t_end, **opts):
    """One rf_step call per step; (solver, step stats, status of the last call)."""
    S = make_solver(w, ebats=0, **opts)
    sts, t = [], 0.0
    while before(t, t_end):
        s, st = S.step(fixed_dt(w, t, t_end))
        sts.append(st)
        if s != 0:
            return S, sts, s
        t = S.get_state()[1]
    return S, sts, 0


def by_run(w, t_end, timing=None, **opts):
    S = make_solver(w, ebats=0, **opts)
    if timing:
        S.set_timing(timing[0])
        S.select_timing(timing[0], every=timing[1])
    s, rs = S.run(t_end)
    return S, rs, s


def state(S):
    h, t = S.get_state()
    return h.cpu().numpy(), t


def compare(w, t_end, timing=None, **opts):
    Sa, sts, sa = by_steps(w, t_end, **opts)
    Sb, rs, sb = by_run(w, t_end, timing, **opts)
    assert sa == sb, (sa, sb, Sb.last_error())
    ok = [st for st in sts if st["converged"]]
    assert rs["accepted"] == len(ok)
    assert rs["rejected"] == (1 if sa else 0)
    assert rs["picard_total"] == sum(st["picard_iters"] for st in sts)
    assert rs["cg_total"] == sum(st["cg_iters_total"] for st in sts)
    ha, ta = state(Sa)
    hb, tb = state(Sb)
    assert ta == tb and np.array_equal(ha, hb)
    assert Sa.mass_balance() == Sb.mass_balance()
    return Sa, Sb, sts, rs


def test_run_ahead_matches_single_steps():
    w = rainy()
    _, _, sts, rs = compare(w, 8 * w.dt, precond=1, tol_cg=1e-8)
    # the rain jump: a clipped step, and steps that needed more Picard
    # iterations than the step before them
    dts = [st["dt"] for st in sts]
    assert 0.5 * w.dt in dts
    its = [st["picard_iters"] for st in sts]
    assert any(b > a for a, b in zip(its, its[1:])), its


def test_run_ahead_clipped_at_t_end_jacobi():
    w = rainy(jump=2.0)
    compare(w, 6.25 * w.dt, precond=0, tol_cg=1e-8)


def test_run_ahead_extrapolated_first_iterate():
    w = rainy()
    compare(w, 8 * w.dt, precond=1, tol_cg=1e-8, first_iterate=1)


def test_run_ahead_mixed_precision():
    w = rainy()
    compare(w, 6 * w.dt, precond=1, tol_cg=1e-8, precision=1, cg_rel_tol=1e-3)


def test_run_ahead_with_fold_kernels():
    # one column per wavefront over 72 x 64 columns: 576 blocks, more than a
    # consumer kernel combines, so every reduction goes through the fold
    w = rainy(nx=72, ny=64, nz=16)
    compare(w, 5 * w.dt, precond=1, tol_cg=1e-8, cols_per_wave=1)


def test_run_ahead_timing_a_sample_of_steps():
    w = rainy()
    _, Sb, _, _ = compare(w, 8 * w.dt, timing=(["update", "coeff"], 3), precond=1, tol_cg=1e-8)
    tm = Sb.get_timing()
    assert tm["update"]["launches"] > 0 and tm["coeff"]["launches"] > 0
    assert tm["spmv"]["launches"] == 0


def test_run_ahead_failing_step_leaves_last_accepted_state():
    # two Picard iterations are not enough for these steps: the run stops at
    # the first step, as one rf_step per step does, with the state rolled back
    w = rainy()
    Sa, Sb, sts, rs = compare(w, 8 * w.dt, precond=1, tol_cg=1e-8, max_picard=2)
    assert not sts[-1]["converged"]
    # the solver goes on from there once allowed more iterations
    for S in (Sa, Sb):
        S.set_options(tol_picard=1e-6, tol_cg=1e-8, max_picard=50, max_cg=20000, ebats=0,
                      dt0=w.dt, precond=1)
    ra, rb = Sa.step(w.dt), Sb.step(w.dt)
    assert ra[0] == 0 and rb[0] == 0
    assert ra[1]["picard_iters"] == rb[1]["picard_iters"]
    assert np.array_equal(state(Sa)[0], state(Sb)[0])


@pytest.mark.parametrize("max_iters,precision,first", [(4, 0, 0), (8, 0, 0), (8, 1, 0), (4, 0, 1)])
def test_run_ahead_under_ebats_matches_single_steps(max_iters, precision, first):
    """rf_run with EBATS runs ahead while the step in flight cannot lengthen
    dt; it must take the steps that the same rules take one rf_step at a
    time (learned.ebats_run without a network): same accepted and rejected
    steps, Picard totals and heads.  With at most four Picard iterations per
    step, and with eight, the rain jump makes steps fail and rerun (about 240
    and 50 steps over the six hours; a heavier rain that ponds the surface
    drives dt down to tens of thousands of steps); with eight also in mixed
    precision, and with four from the extrapolated first iterate, whose ratio
    follows dt through the reruns."""
    from paper_1809_10895_amd import learned
    w = rainy(jump=3.5, q2=2.5e-6)
    t_end = 6 * 3600.0
    seg = w.forcing[W.ZMAX]
    out = []
    for driver in ("rf_run", "steps"):
        S = make_solver(w, precond=1, tol_cg=1e-8, ebats=1, dt0=w.dt, dt_max=3600.0,
                        max_iters=max_iters, max_picard=max_iters if driver == "steps" else 50,
                        precision=precision, first_iterate=first)
        if driver == "rf_run":
            s, rs = S.run(t_end)
            assert s == 0, S.last_error()
            r = (rs["accepted"], rs["rejected"], rs["picard_total"])
        else:
            e = learned.ebats_run(S, seg, t_end, w.dt, 3600.0, max_iters=max_iters)
            r = (e["accepted"], e["rejected"], e["picard_total"])
        out.append((r, state(S)))
    assert out[0][0] == out[1][0], (out[0][0], out[1][0])
    assert out[0][1][1] == out[1][1][1] and np.array_equal(out[0][1][0], out[1][1][0])
    assert out[0][0][1] > 0, out[0][0]          # some steps were rerun
