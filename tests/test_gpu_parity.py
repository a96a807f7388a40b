"""GPU parity: every stage of the HIP path, called through the C ABI, against
the FP64 CPU oracle on the same seeded inputs.  Sizes span several column
chunks and blocks with ragged tails (nz = 70 > 64, nx*ny not a multiple of
the block size) and masked columns."""
import numpy as np
import pytest

from paper_1809_10895_amd import workloads as W
from tests.common import make_oracle, make_solver, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def small_3d(nx=13, ny=11, nz=70, seed=0, mask=True, g=(0.1, -0.05, 0.99373)):
    rng = np.random.default_rng(seed)
    ktop = rng.integers(nz // 2, nz + 1, size=nx * ny).astype(np.int32) if mask else None
    if mask:
        ktop[3] = 0
        ktop[5] = 1
    N = nx * ny * nz
    layer = rng.integers(0, 3, N).astype(np.uint8)
    w = W.Workload(name="small3d", nx=nx, ny=ny, nz=nz, dx=0.7, dy=0.9, dz=0.05,
                   soil=np.array(W.SOIL_EQ5), h0=rng.uniform(-3.0, 0.3, N),
                   bcs=[(W.XMIN, W.DIRICHLET, -0.5), (W.XMAX, W.NOFLOW, 0.0),
                        (W.YMIN, W.FLUX, 3e-7), (W.YMAX, W.FREE_DRAINAGE, 0.0),
                        (W.ZMIN, W.DIRICHLET, 0.2), (W.ZMAX, W.FLUX, 1e-6)],
                   dt=30.0, t_end=300.0, ktop=ktop, grad_elev=np.array(g), layer=layer,
                   lnks=rng.normal(0, 1, N))
    return w, rng


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def test_soil_functions_match_oracle(orc):
    w, rng = small_3d()
    P = make_oracle(orc, w)
    S = make_solver(w)
    h = rng.uniform(-100.0, 1.0, w.N)
    h[::7] = -10 ** rng.uniform(-6, 3, h[::7].size)
    th, cap, k = (host(t) for t in S.eval_soil(dev(h)))
    th_o, cap_o, k_o = P.eval_cells(h)
    m = w.active_mask()
    for got, ref in ((th, th_o), (cap, cap_o), (k, k_o)):
        assert np.all(np.isnan(got[~m]))                  # inactive cells untouched
        nz = ref[m] != 0
        err = np.abs(got[m][nz] - ref[m][nz]) / np.abs(ref[m][nz])
        assert err.max() <= 1e-13, err.max()


@pytest.mark.parametrize("nz", [70, 48])   # 48: the LDS-tiled stencil kernels
@pytest.mark.parametrize("precond", [0, 1])
def test_assembly_operator_preconditioner_match_oracle(orc, precond, nz):
    w, rng = small_3d(seed=1, nz=nz)
    P = make_oracle(orc, w)
    S = make_solver(w, precond=precond)
    hm = w.h0 + rng.normal(0, 0.02, w.N)
    dt = 45.0
    sysd = P.assemble(hm, dt)
    diag, rhs = (host(t) for t in S.assemble(dev(hm), dt))
    m = w.active_mask()
    # The chord slope (theta(h^m) - theta(h^n)) / (h^m - h^n) carries the
    # rounding of the two water contents divided by |h^m - h^n|; one ulp of
    # theta on either side bounds the capacity difference by
    # 4 eps max(theta) / |dh|.  b_P and (A x)_P are sums of terms of size up to
    # A_PP |h| (or |x|): rounding-order differences scale with that row size.
    eps = 2.2e-16
    V = w.dx * w.dy * w.dz
    th_m, _, _ = P.eval_cells(hm)
    dC = 4 * eps * np.abs(th_m) / np.abs(hm - w.h0)
    d_o = sysd["diag"]
    tol_d = 1e-14 * d_o + V * dC / dt
    assert np.all(np.abs(diag[m] - d_o[m]) <= tol_d[m])
    row_b = d_o * (np.abs(w.h0) + np.abs(hm) + 1.0)
    tol_b = 1e-14 * row_b + V * dC / dt * np.abs(w.h0)
    assert np.all(np.abs(rhs[m] - sysd["b"][m]) <= tol_b[m])
    # operator on a random vector
    x = rng.normal(size=w.N)
    x[~m] = 0.0                                       # inactive entries are never read
    y = host(S.apply_operator(dev(x)))
    y_o = P.matvec(sysd, x)
    tol_y = 1e-14 * d_o * np.abs(x).max() + V * dC / dt * np.abs(x)
    assert np.all(np.abs(y[m] - y_o[m]) <= tol_y[m])
    # preconditioner
    r = rng.normal(size=w.N)
    z = host(S.apply_precond(dev(r)))
    assert np.all(np.isnan(z[~m]))                    # inactive cells untouched
    z = np.where(m, z, 0.0)
    if precond == 0:
        ref = r[m] / diag[m]                          # with the diagonal checked above
        assert np.all(np.abs(z[m] - ref) <= 2.3e-16 * np.abs(ref))
    else:
        # z-line: z solves T_col z = r per column, T_col = vertical part of A
        # (the diagonal checked above, -z/+z couplings of the oracle's matrix)
        off = sysd["off"]
        Tz = diag * z
        Tz[1:] += off[4][1:] * z[:-1]
        Tz[:-1] += off[5][:-1] * z[1:]
        za = np.abs(z)
        row = diag * (za + np.r_[0.0, za[:-1]] + np.r_[za[1:], 0.0])
        # pivots and sweeps are prefix scans over the column: rounding grows
        # with its length (nz = 70 here), a few hundred ulps at most
        assert np.max(np.abs(Tz[m] - r[m]) / row[m]) <= 64 * w.nz * 2.2e-16


def test_zline_equals_dic_on_a_column(orc):
    """On a single column both preconditioners are the exact inverse."""
    w = W.column100()
    P = make_oracle(orc, w)
    S = make_solver(w, precond=1)
    rng = np.random.default_rng(3)
    hm = w.h0 + rng.normal(0, 0.1, w.N)
    sysd = P.assemble(hm, 10.0)
    S.assemble(dev(hm), 10.0)
    r = rng.normal(size=w.N)
    z = host(S.apply_precond(dev(r)))
    z_o = P.dic_apply(sysd, r)
    # two exact solves of one tridiagonal system agree to cond(A) * eps
    A = P.dense_matrix(sysd)
    cond = np.linalg.cond(A)
    assert np.abs(z - z_o).max() <= 20 * cond * 2.2e-16 * np.abs(z_o).max()


@pytest.mark.parametrize("precond", [0, 1])
def test_column100_steps_match_oracle(orc, precond):
    w = W.column100()
    P = make_oracle(orc, w)
    S = make_solver(w, precond=precond)
    m = w.active_mask()
    for n in range(40):
        s_o, st_o = P.step(w.dt)
        s_g, st_g = S.step(w.dt)
        assert s_o == 0 and s_g == 0, S.last_error()
        assert st_g["picard_iters"] == st_o["picard_iters"], (n, st_g, st_o)
        h_o, _ = P.get_state()
        h_g = host(S.get_state()[0])
        assert rel_err(h_g, h_o, m) <= 1e-8, n
    if precond == 1:
        assert all(c <= 1 for c in st_g["cg_iters"])    # exact on a column
    mb_g, mb_o = S.mass_balance(), P.mass_balance()
    assert mb_g["storage"] == pytest.approx(mb_o["storage"], rel=1e-10)
    assert np.allclose(mb_g["inflow"], mb_o["inflow"], rtol=1e-8, atol=1e-15)


@pytest.mark.parametrize("nz", [70, 48])   # 48: the LDS-tiled stencil kernels
@pytest.mark.parametrize("precond", [0, 1])
def test_small_3d_mixed_bcs_steps_match_oracle(orc, precond, nz):
    w, _ = small_3d(seed=2, nz=nz)
    w.h0 = np.where(w.active_mask(), -1.0, 0.0)
    w.bcs[4] = (W.ZMIN, W.DIRICHLET, -0.2)
    P = make_oracle(orc, w)
    S = make_solver(w, precond=precond)
    m = w.active_mask()
    for n in range(4):
        s_o, st_o = P.step(w.dt)
        s_g, st_g = S.step(w.dt)
        assert s_o == 0 and s_g == 0, S.last_error()
        assert st_g["picard_iters"] == st_o["picard_iters"]
        h_o, _ = P.get_state()
        h_g = host(S.get_state()[0])
        assert rel_err(h_g, h_o, m) <= 1e-8
        assert np.array_equal(h_g[~m], w.h0[~m])      # inactive cells carried unchanged
    mb = S.mass_balance()
    assert abs(mb["error"]) <= 1e-6 * abs(mb["storage"])


@pytest.mark.parametrize("precond", [0, 1])
def test_saturated_water_table_steps_match_oracle(orc, precond):
    """A water table 30 cm above the base (h > 0 below it: C = S, K = Ks) under
    rain, layered heterogeneous soil: the saturated branch of Eqs. 2-4."""
    nx, ny, nz, dz = 9, 7, 40, 0.025
    rng = np.random.default_rng(8)
    z = (np.arange(nz) + 0.5) * dz
    h0 = np.tile(0.3 - z, nx * ny)
    w = W.Workload(name="watertable", nx=nx, ny=ny, nz=nz, dx=0.5, dy=0.5, dz=dz,
                   soil=np.array([W.SOIL_COLUMN100, W.SOIL_HILLSLOPE]), h0=h0,
                   bcs=[(W.ZMIN, W.DIRICHLET, 0.3), (W.ZMAX, W.FLUX, 2e-6)], dt=5.0,
                   t_end=50.0, layer=(rng.random(nx * ny * nz) < 0.3).astype(np.uint8),
                   lnks=rng.normal(0, 0.5, nx * ny * nz))
    P = make_oracle(orc, w)
    S = make_solver(w, precond=precond)
    m = w.active_mask()
    for n in range(6):
        s_o, st_o = P.step(w.dt)
        s_g, st_g = S.step(w.dt)
        assert s_o == 0 and s_g == 0, S.last_error()
        assert st_g["picard_iters"] == st_o["picard_iters"]
        h_o, _ = P.get_state()
        assert rel_err(host(S.get_state()[0]), h_o, m) <= 1e-8
    assert (h_o > 0).sum() > 100
    mb_g, mb_o = S.mass_balance(), P.mass_balance()
    assert mb_g["storage"] == pytest.approx(mb_o["storage"], rel=1e-10)
    assert np.allclose(mb_g["inflow"], mb_o["inflow"], rtol=1e-8, atol=1e-15)


def test_hillslope_slice_steps_match_oracle(orc):
    w = W.hillslope(nx=24, ny=20, nz=64)
    P = make_oracle(orc, w)
    S = make_solver(w, precond=1)
    m = w.active_mask()
    for n in range(3):
        s_o, st_o = P.step(w.dt)
        s_g, st_g = S.step(w.dt)
        assert s_o == 0 and s_g == 0
        assert st_g["picard_iters"] == st_o["picard_iters"]
        h_o, _ = P.get_state()
        assert rel_err(host(S.get_state()[0]), h_o, m) <= 1e-8


def test_watershed_slice_ebats_run_matches_oracle(orc):
    w = W.watershed(nx=24, ny=20, nz=64, t_end=6 * 3600.0)
    # a wet first hours so that the rain and EBATS clipping are exercised
    t0, q = w.forcing[W.ZMAX]
    q = q.copy()
    q[:3] = [2e-6, 0.0, 5e-6]
    w.forcing[W.ZMAX] = (t0, q)
    P = make_oracle(orc, w)
    S = make_solver(w, precond=1)
    s_o, rs_o = P.run(w.t_end)
    s_g, rs_g = S.run(w.t_end)
    assert s_o == 0 and s_g == 0, S.last_error()
    assert (rs_g["accepted"], rs_g["rejected"], rs_g["picard_total"]) == \
        (rs_o["accepted"], rs_o["rejected"], rs_o["picard_total"])
    m = w.active_mask()
    h_o, t_o = P.get_state()
    h_g, t_g = S.get_state()
    assert t_g == t_o
    assert rel_err(host(h_g), h_o, m) <= 1e-8
    mb_g, mb_o = S.mass_balance(), P.mass_balance()
    assert mb_g["inflow"][W.ZMAX] == pytest.approx(mb_o["inflow"][W.ZMAX], rel=1e-12)
    assert mb_g["storage"] == pytest.approx(mb_o["storage"], rel=1e-10)


def test_runs_are_deterministic():
    w = W.hillslope(nx=20, ny=18, nz=64)
    out = []
    for _ in range(2):
        S = make_solver(w, precond=1, tol_cg=1e-8)
        for _ in range(2):
            assert S.step(w.dt)[0] == 0
        out.append(host(S.get_state()[0]))
    assert np.array_equal(out[0], out[1])


def test_failed_step_rolls_back_bitwise():
    w = W.column100()
    S = make_solver(w, max_picard=1)
    h0 = host(S.get_state()[0])
    s, st = S.step(50.0)
    assert s == -5 and st["picard_iters"] == 1            # RF_ERR_NOT_CONVERGED
    h1, t = S.get_state()
    assert np.array_equal(host(h1), h0) and t == 0.0
    assert S.mass_balance()["error"] == 0.0


def test_error_paths():
    from paper_1809_10895_amd import Solver
    S = Solver()
    assert S.L.rf_step(S.h, 1.0, None, None) == -2          # RF_ERR_STATE before set-up
    w = W.column100()
    S2 = make_solver(w)
    bad = torch.full((w.N,), -1.0, dtype=torch.float64, device="cuda")
    bad[17] = float("nan")
    h_before = host(S2.get_state()[0])
    assert S2.set_state(bad) == -7                          # RF_ERR_NONFINITE
    assert np.array_equal(host(S2.get_state()[0]), h_before)
    assert S2.L.rf_step(S2.h, -1.0, None, None) == -1       # RF_ERR_ARG


@pytest.mark.parametrize("precond,variant", [(1, 0), (0, 0), (1, 1)])
def test_hillslope_full_size_one_step(orc, precond, variant):
    """The 128x128x64 hillslope in the launch shape the benchmark times: one
    600 s step against the oracle (tight PCG tolerance on both sides, so the
    result does not depend on the preconditioner), with the z-line and the
    Jacobi preconditioner on the GPU, and with the modified Picard
    linearisation on both sides."""
    w = W.hillslope()
    P = make_oracle(orc, w, picard_variant=variant)
    S = make_solver(w, precond=precond, picard_variant=variant)
    s_o, st_o = P.step(w.dt)
    s_g, st_g = S.step(w.dt)
    assert s_o == 0 and s_g == 0
    assert st_g["picard_iters"] == st_o["picard_iters"]
    h_o, _ = P.get_state()
    assert rel_err(host(S.get_state()[0]), h_o, w.active_mask()) <= 1e-8


def test_hillslope_steps_match_oracle_at_bench_options(orc):
    """The full 128 x 128 x 64 hillslope at the benchmark's FP64 options (PCG
    tolerance 1e-8 m, the paper's 1/100 of the Picard tolerance): eight 600 s
    steps, the same Picard counts, every active head within 1e-8 relative
    after every step (measured: the difference grows to 1.9e-9, the solves'
    errors at tol_cg adding up over the steps)."""
    w = W.hillslope()
    P = make_oracle(orc, w, tol_cg=1e-8)
    S = make_solver(w, precond=1, tol_cg=1e-8)
    m = w.active_mask()
    for n in range(8):
        s_o, st_o = P.step(w.dt)
        s_g, st_g = S.step(w.dt)
        assert s_o == 0 and s_g == 0, S.last_error()
        assert st_g["picard_iters"] == st_o["picard_iters"], (n, st_g["delta"], st_o["delta"])
        assert rel_err(host(S.get_state()[0]), P.get_state()[0], m) <= 1e-8, n

