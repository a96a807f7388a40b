"""The two ways of reaching lateral neighbours in the stencil kernels (LDS
tiles with a halo, and per-wave neighbour-column loads) on the same steps:
identical Picard and PCG counts and heads equal to rounding, on a masked,
tilted grid whose extent is not a whole number of tiles (partial tiles at
the +x and +y edges, empty columns, one-cell columns); and the tiled path
against the oracle."""
import numpy as np
import pytest

from paper_1809_10895_amd import workloads as W
from tests.common import make_oracle, make_solver, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def masked_grid(nx=37, ny=26, nz=64, seed=7):
    w = W.watershed(nx=nx, ny=ny, nz=nz, seeds=(seed, seed + 1, seed + 2), kmin=nz // 2)
    w.ktop[0] = 0
    w.ktop[nx + 3] = 1
    w.ktop[-1] = nz
    w.h0 = np.where(w.active_mask(), -2.0, 0.0)
    w.grad_elev = np.array([0.08, -0.05, 0.995])
    w.bcs.append((W.XMIN, W.DIRICHLET, -1.0))
    return w


@pytest.mark.parametrize("tile_rows", [2, 4])   # tiles of 8 x 2 and 8 x 4 columns
@pytest.mark.parametrize("precision", [0, 1])
def test_tiles_and_columns_take_the_same_steps(precision, tile_rows):
    w = masked_grid()
    opts = dict(ebats=1, dt0=300.0, precision=precision)
    S_t = make_solver(w, stencil=1, tile_rows=tile_rows, **opts)
    S_c = make_solver(w, stencil=0, **opts)
    s_t, r_t = S_t.run(4 * 3600.0)
    s_c, r_c = S_c.run(4 * 3600.0)
    assert s_t == 0 and s_c == 0, (S_t.last_error(), S_c.last_error())
    for k in ("accepted", "rejected", "picard_total", "cg_total"):
        assert r_t[k] == r_c[k], (k, r_t, r_c)
    m = w.active_mask()
    h_t = S_t.get_state()[0].cpu().numpy()
    h_c = S_c.get_state()[0].cpu().numpy()
    assert rel_err(h_t, h_c, m) <= 1e-12
    assert np.array_equal(h_t[~m], w.h0[~m])         # inactive cells untouched


def test_tiles_walked_per_block_on_a_large_grid():
    """A grid of more than 512 tiles (each block walks a run of tiles, the next
    one's loads in flight): the same steps as the per-wave column kernels."""
    w = masked_grid(nx=136, ny=130, nz=24, seed=5)      # 17 x 65 = 1105 tiles of 8 x 2
    opts = dict(ebats=0, dt0=900.0)
    S_t = make_solver(w, stencil=1, **opts)
    S_c = make_solver(w, stencil=0, **opts)
    for _ in range(3):
        s_t, st_t = S_t.step(900.0)
        s_c, st_c = S_c.step(900.0)
        assert s_t == 0 and s_c == 0
        assert st_t["picard_iters"] == st_c["picard_iters"]
        assert st_t["cg_iters"] == st_c["cg_iters"]
    m = w.active_mask()
    assert rel_err(S_t.get_state()[0].cpu().numpy(), S_c.get_state()[0].cpu().numpy(), m) <= 1e-12


@pytest.mark.parametrize("nz", [40, 33])   # 33: odd column height (cell pairs at odd offsets)
def test_tiled_steps_match_oracle(orc, nz):
    w = masked_grid(nx=21, ny=14, nz=nz, seed=11)
    P = make_oracle(orc, w)
    S = make_solver(w, stencil=1)
    m = w.active_mask()
    for n in range(6):
        s_o, st_o = P.step(600.0)
        s_g, st_g = S.step(600.0)
        assert s_o == 0 and s_g == 0, S.last_error()
        assert st_g["picard_iters"] == st_o["picard_iters"], (n, st_g, st_o)
        h_o, _ = P.get_state()
        h_g = S.get_state()[0].cpu().numpy()
        assert rel_err(h_g, h_o, m) <= 1e-8, n
    mb_g, mb_o = S.mass_balance(), P.mass_balance()
    assert mb_g["storage"] == pytest.approx(mb_o["storage"], rel=1e-10)


@pytest.mark.parametrize("stencil", [1, 0])   # tiles, column kernels
def test_every_column_height_matches_oracle(orc, stencil):
    """Columns of every active height 0..64 side by side: odd and even tops,
    one-cell columns, tops at the 16- and 32-lane boundaries of the half-waves
    that the short-column kernels scan over, full and empty columns.  Same
    Picard iterations as the oracle and heads to 1e-8 over three steps."""
    w = masked_grid(nx=65, ny=2, nz=64, seed=13)
    w.ktop = np.tile(np.arange(65, dtype=np.int32), 2)
    w.h0 = np.where(w.active_mask(), -2.0, 0.0)
    P = make_oracle(orc, w)
    S = make_solver(w, stencil=stencil)
    m = w.active_mask()
    for n in range(3):
        s_o, st_o = P.step(600.0)
        s_g, st_g = S.step(600.0)
        assert s_o == 0 and s_g == 0, S.last_error()
        assert st_g["picard_iters"] == st_o["picard_iters"], (n, st_g, st_o)
        h_o, _ = P.get_state()
        assert rel_err(S.get_state()[0].cpu().numpy(), h_o, m) <= 1e-8, n
