"""The oracle's slab mode (block-Jacobi DIC over sub-domains of whole y-rows,
the 'simple' decomposition of Sec. 2.3, on OpenMP threads): it changes the
preconditioner, not the solution, so every Picard step must reach the heads
of the serial method to within the PCG tolerance, and a slab must never use a
coupling that crosses its boundary."""
import numpy as np
import pytest

from paper_1809_10895_amd import workloads as W


def _pair(orc, w, nslab, **opts):
    out = []
    for ns in (1, nslab):
        P = orc.Problem(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, ktop=w.ktop, grad_elev=w.grad_elev)
        W.configure(w, P)
        P.set_options(**opts)
        P.set_slabs(ns)
        assert P.set_state(w.h0) == 0
        out.append(P)
    return out


def test_slab_mode_reaches_the_serial_heads(orc):
    w = W.watershed(nx=24, ny=20, nz=16, kmin=6)
    ser, par = _pair(orc, w, 5, tol_picard=1e-9, tol_cg=1e-13, max_picard=100, max_cg=20000,
                     ebats=0, dt0=600.0)
    cg = [0, 0]
    for _ in range(4):
        s0, st0 = ser.step(600.0)
        s1, st1 = par.step(600.0)
        assert s0 == 0 and s1 == 0
        cg[0] += st0["cg_iters_total"]
        cg[1] += st1["cg_iters_total"]
    h0, _ = ser.get_state()
    h1, _ = par.get_state()
    m = ser.active_mask()
    assert np.abs(h1[m] - h0[m]).max() <= 1e-9
    # block Jacobi across slabs is a weaker preconditioner than the global DIC
    assert cg[1] > cg[0]
    mb0, mb1 = ser.mass_balance(), par.mass_balance()
    assert mb1["storage"] == pytest.approx(mb0["storage"], rel=1e-11)


def test_slab_preconditioner_is_block_diagonal(orc):
    """z = M^-1 r of a residual that is non-zero only inside slab s must be zero
    outside slab s (the slabs' DIC factors are independent)."""
    w = W.hillslope(nx=6, ny=8, nz=5)
    P = orc.Problem(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz)
    W.configure(w, P)
    P.set_state(w.h0)
    P.set_slabs(4)                      # rows {0,1}, {2,3}, {4,5}, {6,7}
    sysd = P.assemble(w.h0 + 0.01, 600.0)
    row = w.nx * w.nz
    r = np.zeros(P.N)
    r[2 * row:4 * row] = np.random.default_rng(3).normal(size=2 * row)
    z = P.dic_apply(sysd, r)
    assert np.all(z[:2 * row] == 0.0) and np.all(z[4 * row:] == 0.0)
    assert np.abs(z[2 * row:4 * row]).max() > 0.0
    # with one slab the same residual spreads over the whole grid
    P.set_slabs(1)
    z1 = P.dic_apply(sysd, r)
    assert np.abs(z1[:2 * row]).max() > 0.0
