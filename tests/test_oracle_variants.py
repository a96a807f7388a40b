"""Pins of the oracle on the paper's variant cases: the modified Picard
linearisation (Sec. 2.2), the loam infiltration column of Sec. 3.1 and the
steep-front heterogeneous block of Appendix B.

The modified scheme (Celia et al., cited in Sec. 2.2) keeps theta~(h^m) -
theta~(h^n) explicitly and takes the analytic capacity for the remaining
increment; the classical scheme takes the chord slope.  Both have the same
fixed point, the mass-conservative backward-Euler equation
V (theta~(h) - theta~(h^n)) / dt = net inflow, so their converged states
must agree to the Picard tolerance, and the converged state of either must
satisfy the other's linear system."""
import numpy as np
import pytest

from tests.golden_data import SOILS


def loam_column(orc, variant, nz=100, dz=0.01):
    """Sec. 3.1: 1 m of loam in 1 cm cells, h = -1 m initially, free drainage
    at the base, fixed head 0.01 m at the top."""
    P = orc.Problem(1, 1, nz, 1.0, 1.0, dz)
    P.set_soil(np.array([SOILS["loam_sec3_1"]]))
    P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE, 0.0)
    P.set_bc(orc.ZMAX, orc.DIRICHLET, 0.01)
    P.set_state(np.full(nz, -1.0))
    return P


def chord_residual(orc, P_template_args, h_prev, h_new, dt):
    """max |A h - b| / diag of the classical (chord-slope) system assembled
    at h^m = h_new for the step h_prev -> h_new."""
    P = P_template_args()
    P.set_options(picard_variant=orc.PICARD_CHORD)
    P.set_state(h_prev)
    sysd = P.assemble(h_new, dt)
    Ah = P.matvec(sysd, h_new)
    return np.max(np.abs(Ah - sysd["b"]) / sysd["diag"])


def test_modified_and_classical_picard_share_the_fixed_point(orc):
    dt = 300.0
    states = {}
    for v in (orc.PICARD_CHORD, orc.PICARD_MODIFIED):
        P = loam_column(orc, v)
        P.set_options(tol_picard=1e-11, tol_cg=1e-15, max_picard=200, max_cg=1000, ebats=0,
                      dt0=dt, picard_variant=v)
        hist = [P.get_state()[0]]
        iters = []
        for _ in range(12):
            s, st = P.step(dt)
            assert s == 0
            iters.append(st["picard_iters"])
            hist.append(P.get_state()[0])
        states[v] = (hist, iters, P.mass_balance())
    h_c, it_c, mb_c = states[orc.PICARD_CHORD]
    h_m, it_m, mb_m = states[orc.PICARD_MODIFIED]
    assert it_c != it_m                           # two different iterations ...
    assert np.max(np.abs(h_c[-1] - h_m[-1])) <= 1e-8   # ... one fixed point
    # the modified scheme's converged state solves the classical system
    for n in (1, 6, 12):
        r = chord_residual(orc, lambda: loam_column(orc, 0), h_m[n - 1], h_m[n], dt)
        assert r <= 1e-9, (n, r)
    for mb in (mb_c, mb_m):
        assert abs(mb["error"]) <= 1e-9 * (mb["storage"] - mb["storage0"])


def test_modified_picard_first_iterate_uses_the_analytic_capacity(orc):
    """One Picard iteration from h^0 = h^n: both schemes then take the
    analytic capacity C(h^n) (the chord is undefined) and give the same
    first iterate; they differ from the second on."""
    dt = 300.0
    out = {}
    for v in (orc.PICARD_CHORD, orc.PICARD_MODIFIED):
        P = loam_column(orc, v)
        P.set_options(tol_picard=1e-11, tol_cg=1e-15, max_picard=200, ebats=0, dt0=dt,
                      picard_variant=v)
        s, st = P.step(dt)
        assert s == 0
        out[v] = st["delta"]
    d_c, d_m = out[orc.PICARD_CHORD], out[orc.PICARD_MODIFIED]
    assert d_c[0] == d_m[0]
    assert d_c[1] != d_m[1]


def test_loam_column_sec3_1_infiltration(orc):
    """Sec. 3.1 run under EBATS (first step 5 min, largest 1 h) for 2 h:
    the balance closes, water enters through the top only, and the profile
    stays monotone (wetter towards the ponded top).  The ponded top cell
    crosses saturation, where the Picard iterates of the chord scheme swing
    between the saturated and unsaturated branches, so EBATS settles on
    steps of seconds (rejections included)."""
    P = loam_column(orc, orc.PICARD_CHORD)
    P.set_options(tol_picard=1e-6, tol_cg=1e-12, max_picard=50, ebats=1, dt0=300.0,
                  dt_max=3600.0)
    s, rs = P.run(2 * 3600.0)
    assert s == 0 and rs["accepted"] > 12 and rs["rejected"] > 0
    h, t = P.get_state()
    assert t == 2 * 3600.0
    assert np.all(np.diff(h) >= -1e-12)                 # h increases upwards
    assert h[-1] > -0.2 and h[0] < -0.9                 # front inside the column
    mb = P.mass_balance()
    gain = mb["storage"] - mb["storage0"]
    assert mb["inflow"][orc.ZMAX] > 0 and gain > 0
    assert abs(mb["error"]) <= 1e-6 * gain


def steep_block(orc, top, t_end, tol_cg=1e-6, variant=0, nx=8, ny=6, nz=40, d=0.25, seed=0):
    """Appendix B, scaled down: a block with an uncorrelated lognormal Ks
    (median 1e-6 m/s, sigma of log10 Ks = 1), a water table at mid height
    (hydrostatic start, fixed head at the base), fixed head `top` at the
    surface; PCG 1e-6 m, Picard 1e-4 m, first step 0.1 s."""
    P = orc.Problem(nx, ny, nz, d, d, d)
    rng = np.random.default_rng(seed)
    soil = np.array(SOILS["loam_sec3_1"])
    soil[4] = 1e-6
    P.set_soil(np.array([soil]), None, rng.normal(0.0, np.log(10.0), P.N))
    z = (np.arange(nz) + 0.5) * d
    H = nz * d / 2
    P.set_bc(orc.ZMIN, orc.DIRICHLET, H)
    P.set_bc(orc.ZMAX, orc.DIRICHLET, top)
    P.set_options(tol_picard=1e-4, tol_cg=tol_cg, max_picard=50, max_cg=20000, dt0=0.1,
                  dt_max=86400.0, ebats=1, picard_variant=variant)
    P.set_state(np.tile(H - z, nx * ny))
    s, rs = P.run(t_end)
    assert s == 0, rs
    return rs, P.mass_balance()


def test_appendix_b_steeper_fronts_need_more_iterations(orc):
    """The paper reports a strong growth of the PCG effort from the smooth
    (-0.1 m) to the steep (1 m) infiltration; the same ordering holds here,
    and every run closes its water balance."""
    cg, picard = [], []
    for top in (-0.1, 0.1, 1.0):
        rs, mb = steep_block(orc, top, 600.0)
        cg.append(rs["cg_total"])
        picard.append(rs["picard_total"])
        assert abs(mb["error"]) <= 1e-5 * (mb["storage"] - mb["storage0"])
    assert cg[0] < cg[1] < cg[2] and cg[2] > 10 * cg[0]
    assert picard[0] < picard[1] < picard[2]


@pytest.mark.parametrize("variant", [0, 1])
def test_appendix_b_both_linearisations_conserve_mass(orc, variant):
    rs, mb = steep_block(orc, 1.0, 120.0, tol_cg=1e-12, variant=variant)
    assert rs["accepted"] > 100
    assert abs(mb["error"]) <= 2e-5 * (mb["storage"] - mb["storage0"])
