"""Pins of the oracle's whole Picard step and time loop against results fixed
by the mathematics: hydrostatic equilibrium, the closed-form steady Gardner
profile of Appendix A (Eq. A8), the exact discrete steady state found by
shooting, the unit-gradient free-drainage state, the water balance, 1-D/3-D
equivalence, symmetry and the EBATS rules (Sec. 2.2)."""
import numpy as np
import pytest

from tests.golden_data import SOILS


def column(orc, nz, dz, soil, model=0, nx=1, ny=1, dx=1.0, dy=1.0):
    P = orc.Problem(nx, ny, nz, dx, dy, dz)
    P.set_soil(np.array([soil]), model=model)
    return P


def steady(P, h0, tol=1e-13, chunk=1e6, nchunks=200):
    """March to steady state with EBATS (Picard with explicit gravity does not
    converge for one huge step on steep curves), until a whole chunk of
    simulated time changes h by less than tol."""
    P.set_options(tol_picard=1e-12, tol_cg=1e-15, max_picard=500, max_cg=100000, ebats=1,
                  dt0=100.0, dt_max=1e7, dt_min=1e-8, max_iters=12)
    P.set_state(h0)
    prev, t = None, 0.0
    for _ in range(nchunks):
        t += chunk
        s, rs = P.run(t)
        assert s == 0, rs
        h, _ = P.get_state()
        if prev is not None and np.max(np.abs(h - prev)) < tol:
            return h
        prev = h
    raise AssertionError("no steady state")


def test_hydrostatic_invariance_3d(orc):
    nx, ny, nz, dx, dy, dz = 4, 3, 12, 0.5, 0.5, 0.05
    g = np.array([0.25, -0.15, 0.956556])
    P = orc.Problem(nx, ny, nz, dx, dy, dz, grad_elev=g)
    rng = np.random.default_rng(0)
    P.set_soil(np.array([SOILS["loam_sec3_1"], SOILS["eq5_layer2"]]),
               rng.integers(0, 2, P.N).astype(np.uint8), rng.normal(0, 1, P.N))
    i = np.arange(nx)[None, :, None]
    j = np.arange(ny)[:, None, None]
    k = np.arange(nz)[None, None, :]
    elev = g[0] * (i + .5) * dx + g[1] * (j + .5) * dy + g[2] * (k + .5) * dz
    h = (0.3 - elev).ravel()                   # saturated below, unsaturated above
    P.set_options(tol_picard=1e-9, tol_cg=1e-12, max_picard=20, ebats=0, dt0=3600.0)
    P.set_state(h)
    for dt in (1.0, 3600.0, 1e6):
        s, st = P.step(dt)
        assert s == 0 and st["picard_iters"] == 1 and st["cg_iters_total"] == 0
    h1, _ = P.get_state()
    assert np.max(np.abs(h1 - h)) <= 1e-13
    mb = P.mass_balance()
    assert abs(mb["error"]) <= 1e-14 * mb["storage"]


def gardner_profile(z, Ks, alpha, q_in):
    """Steady h(z) above a water table (h = 0 at z = 0) with a constant
    downward flux q_in (Appendix A, Eq. A8 with the flux counted positive
    downward; the text's 'positive = evaporation' is the opposite sign)."""
    return np.log((q_in + (Ks - q_in) * np.exp(-alpha * z)) / Ks) / alpha


@pytest.mark.parametrize("alpha,q_in", [(3.0, 5e-7), (3.0, -2e-8), (1.0, 8e-7), (0.06, 5e-7),
                                        (0.06, -1e-7)])
def test_gardner_closed_form_second_order(orc, alpha, q_in):
    Ks, L = 1e-6, 1.0
    soil = (0.05, 0.40, alpha, 2.0, Ks, 1e-5)
    errs = []
    for nz in (50, 100, 200):
        dz = L / nz
        P = column(orc, nz, dz, soil, model=orc.GARDNER)
        P.set_bc(orc.ZMIN, orc.DIRICHLET, 0.0)
        P.set_bc(orc.ZMAX, orc.FLUX, q_in)
        z = (np.arange(nz) + 0.5) * dz
        h = steady(P, -0.5 * z)
        errs.append(np.max(np.abs(h - gardner_profile(z, Ks, alpha, q_in))))
    if alpha >= 1.0:
        order = np.log2(errs[0] / errs[1]), np.log2(errs[1] / errs[2])
        assert 1.8 < order[0] < 2.2 and 1.8 < order[1] < 2.2, (errs, order)
    assert errs[1] < 1e-3 * max(1.0, alpha), errs


def shoot(orc, soil, nz, dz, h_bottom, q_in):
    """Exact discrete steady state of the 1-D scheme: every face carries the
    same downward flux q_in.  Bottom Dirichlet face (half cell): solved in
    closed form; each interior face (K_f = mean of the two cells): solved for
    the upper cell by bisection to the last bit."""
    K = lambda h: orc.conductivity([h], soil)[0]
    Kb = K(h_bottom)
    h = [h_bottom - 0.5 * dz * (1.0 - q_in / Kb)]
    for _ in range(nz - 1):
        hk, Kk = h[-1], K(h[-1])
        f = lambda hn: 0.5 * (Kk + K(hn)) * ((hn - hk) / dz + 1.0) - q_in
        lo, hi = hk - dz, hk + 50.0
        assert f(lo) < 0 < f(hi)
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if f(mid) < 0:
                lo = mid
            else:
                hi = mid
        h.append(0.5 * (lo + hi))
    return np.array(h)


@pytest.mark.parametrize("soil_name,q_frac", [("column100", 0.2), ("loam_sec3_1", 0.5),
                                              ("steep_n3", 0.05)])
def test_discrete_steady_state_by_shooting(orc, soil_name, q_frac):
    soil = SOILS[soil_name]
    nz, dz, hb = 60, 0.02, -0.1
    q_in = q_frac * orc.conductivity([hb], soil)[0]
    h_ref = shoot(orc, soil, nz, dz, hb, q_in)
    P = column(orc, nz, dz, soil)
    P.set_bc(orc.ZMIN, orc.DIRICHLET, hb)
    P.set_bc(orc.ZMAX, orc.FLUX, q_in)
    h = steady(P, np.full(nz, -0.5))
    assert np.max(np.abs(h - h_ref)) <= 1e-9, np.max(np.abs(h - h_ref))


def test_free_drainage_unit_gradient(orc):
    """Top flux q over a free-draining base: the steady state is uniform with
    K(h) = q (gravity-only flow)."""
    soil = SOILS["hillslope"]
    q = 1e-8
    lo, hi = -100.0, 0.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if orc.conductivity([mid], soil)[0] < q:
            lo = mid
        else:
            hi = mid
    P = column(orc, 40, 0.05, soil)
    P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
    P.set_bc(orc.ZMAX, orc.FLUX, q)
    h = steady(P, np.full(40, -1.0), tol=1e-12)
    assert np.max(np.abs(h - 0.5 * (lo + hi))) <= 1e-8


def test_water_balance_transient(orc):
    """Rain on the 1-D column over a shallow water table (a saturated band, so
    C = S is exercised): storage change equals cumulative boundary inflow up
    to the Picard tolerance."""
    soil = SOILS["column100"]
    P = column(orc, 100, 0.01, soil)
    P.set_bc(orc.ZMAX, orc.FLUX, 2e-6)
    P.set_bc(orc.ZMIN, orc.DIRICHLET, 0.2)       # water table 20 cm above the base
    P.set_options(tol_picard=1e-10, tol_cg=1e-13, ebats=1, dt0=1.0, dt_max=60.0, max_iters=20)
    z = (np.arange(100) + 0.5) * 0.01
    P.set_state(0.2 - z)
    s, rs = P.run(1800.0)
    assert s == 0 and rs["accepted"] > 20
    mb = P.mass_balance()
    dS = mb["storage"] - mb["storage0"]
    assert mb["inflow"][orc.ZMAX] == pytest.approx(1800 * 2e-6, rel=1e-12)
    assert abs(mb["error"]) <= 1e-9 * abs(dS), mb
    h, _ = P.get_state()
    assert (h > 0).sum() >= 10    # a saturated band exists, so S is exercised


def test_3d_homogeneous_equals_1d(orc):
    soil = SOILS["loam_sec3_1"]
    nz, dz = 30, 0.02
    P1 = column(orc, nz, dz, soil)
    P3 = column(orc, nz, dz, soil, nx=3, ny=2, dx=0.4, dy=0.6)
    for P in (P1, P3):
        P.set_bc(orc.ZMAX, orc.FLUX, 5e-7)
        P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
        P.set_options(tol_picard=1e-10, tol_cg=1e-14, max_picard=100, ebats=0, dt0=60.0)
    P1.set_state(np.full(nz, -1.0))
    P3.set_state(np.full(6 * nz, -1.0))
    assert P1.run(3600.0)[0] == 0 and P3.run(3600.0)[0] == 0
    h1, _ = P1.get_state()
    h3, _ = P3.get_state()
    assert np.max(np.abs(h3.reshape(6, nz) - h1[None, :])) <= 1e-11


def test_xy_symmetry(orc):
    nx = ny = 5
    nz = 6
    rng = np.random.default_rng(5)
    f = rng.normal(size=(nx, nx))
    f = f + f.T                                   # symmetric under i <-> j
    lnks = np.repeat(f.reshape(-1), nz)           # cell k + nz*(i + nx*j) -> f[j, i]
    P = orc.Problem(nx, ny, nz, 1.0, 1.0, 0.1)
    P.set_soil(np.array([SOILS["hillslope"]]), None, lnks)
    P.set_bc(orc.ZMAX, orc.FLUX, 1e-6)
    P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
    P.set_options(tol_picard=1e-10, tol_cg=1e-14, ebats=0, dt0=600.0)
    P.set_state(np.full(P.N, -2.0))
    assert P.run(6000.0)[0] == 0
    h, _ = P.get_state()
    h = h.reshape(ny, nx, nz)
    assert np.max(np.abs(h - h.transpose(1, 0, 2))) <= 1e-11


def test_step_failure_rolls_back(orc):
    soil = SOILS["column100"]
    P = column(orc, 100, 0.01, soil)
    P.set_bc(orc.ZMAX, orc.DIRICHLET, -0.75)
    P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
    P.set_options(tol_picard=1e-6, tol_cg=1e-10, max_picard=1, ebats=0, dt0=10.0)
    h0 = np.full(100, -10.0)
    P.set_state(h0)
    s, st = P.step(100.0)
    assert s == orc.ERR_NOT_CONVERGED and st["picard_iters"] == 1
    h, t = P.get_state()
    assert np.array_equal(h, h0) and t == 0.0
    assert P.mass_balance()["error"] == 0.0


def test_ebats_growth_rule(orc):
    """A system that always converges in one Picard iteration (hydrostatic):
    dt grows by `factor` after every `inc_after` steps, capped at dt_max."""
    nz, dz = 10, 0.1
    P = column(orc, nz, dz, SOILS["loam_sec3_1"])
    z = (np.arange(nz) + 0.5) * dz
    P.set_options(tol_picard=1e-8, tol_cg=1e-12, ebats=1, dt0=1.0, dt_max=2.0, factor=1.3,
                  inc_after=10, few_iters=3, max_iters=8)
    P.set_state(-z)
    t, dt, expect = 0.0, 1.0, 0
    for n in range(1, 45):
        t += dt
        expect += 1
        if n % 10 == 0:
            dt = min(dt * 1.3, 2.0)
    s, rs = P.run(t)
    assert s == 0 and rs["accepted"] == expect and rs["rejected"] == 0
    assert P.dt == pytest.approx(dt, rel=1e-14)


def test_ebats_shrinks_until_dt_min(orc):
    P = column(orc, 100, 0.01, SOILS["column100"])
    P.set_bc(orc.ZMAX, orc.DIRICHLET, -0.75)
    P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
    # max_iters = 1: every step that needs a second Picard iteration is rerun
    P.set_options(tol_picard=1e-6, tol_cg=1e-10, ebats=1, dt0=100.0, dt_min=1.0, factor=2.0,
                  max_iters=1)
    h0 = np.full(100, -10.0)
    P.set_state(h0)
    s, rs = P.run(1000.0)
    assert s == orc.ERR_NOT_CONVERGED
    assert rs["rejected"] == 7 and rs["accepted"] == 0    # 100 -> 50 ... -> 0.78 < dt_min
    h, t = P.get_state()
    assert np.array_equal(h, h0) and t == 0.0


def test_forcing_segments(orc):
    """Piecewise-constant rain: steps end on segment boundaries and the
    cumulative top inflow is the integral of the series."""
    P = column(orc, 40, 0.05, SOILS["hillslope"])
    P.set_bc(orc.ZMAX, orc.FLUX, 0.0)
    P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
    t0 = np.array([0.0, 1000.0, 1500.0, 4000.0])
    q = np.array([0.0, 2e-6, 0.0, 5e-7])
    P.set_forcing(orc.ZMAX, t0, q)
    P.set_options(tol_picard=1e-8, tol_cg=1e-12, ebats=1, dt0=300.0, dt_max=3600.0)
    P.set_state(np.full(40, -2.0))
    assert P.run(6000.0)[0] == 0
    expected = 500 * 2e-6 + 2000 * 5e-7
    assert P.mass_balance()["inflow"][orc.ZMAX] == pytest.approx(expected, rel=1e-12)


def test_picard_iterates_reproduce_the_step(orc):
    """The iterates exposed for inspection are the step's own: the last one is
    the accepted state, and their successive differences are the deltas the
    step reports."""
    soil = SOILS["column100"]
    P = column(orc, 100, 0.01, soil)
    P.set_bc(orc.ZMAX, orc.DIRICHLET, -0.75)
    P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
    P.set_options(tol_picard=1e-6, tol_cg=1e-13, ebats=0, dt0=10.0)
    h0 = np.full(100, -10.0)
    P.set_state(h0)
    s, st = P.step(10.0)
    assert s == 0 and st["picard_iters"] >= 3
    h1, _ = P.get_state()
    P.set_state(h0)
    its = [h0] + [P.picard_iterate(h0, 10.0, m) for m in range(1, st["picard_iters"] + 1)]
    assert np.array_equal(its[-1], h1)
    for m in range(st["picard_iters"]):
        assert np.abs(its[m + 1] - its[m]).max() == st["delta"][m]
    assert np.array_equal(P.get_state()[0], h0)          # state untouched
