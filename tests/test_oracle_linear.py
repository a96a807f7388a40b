"""Pins of the oracle's assembly and DIC-PCG solve: symmetry, the exact
hydrostatic null-flux state, LAPACK dense solves, and the exactness of DIC on
tridiagonal (1-D) systems."""
import numpy as np
import pytest
import scipy.linalg

from tests.golden_data import SOILS


def make_problem(orc, nx, ny, nz, seed=0, mask=False, g=None, dx=0.5, dy=0.7, dz=0.1):
    rng = np.random.default_rng(seed)
    ktop = None
    if mask:
        ktop = rng.integers(nz // 2, nz + 1, size=nx * ny).astype(np.int32)
        ktop[0] = 0  # one empty column
    P = orc.Problem(nx, ny, nz, dx, dy, dz, ktop=ktop, grad_elev=g)
    params = np.array([SOILS["eq5_layer1"], SOILS["eq5_layer2"], SOILS["hillslope"]])
    layer = rng.integers(0, 3, size=P.N).astype(np.uint8)
    lnks = rng.normal(0.0, 1.0, size=P.N)
    P.set_soil(params, layer, lnks)
    return P, rng


def mixed_bcs(orc, P):
    P.set_bc(orc.XMIN, orc.DIRICHLET, -0.4)
    P.set_bc(orc.XMAX, orc.NOFLOW)
    P.set_bc(orc.YMIN, orc.FLUX, 2e-7)
    P.set_bc(orc.YMAX, orc.FREE_DRAINAGE)
    P.set_bc(orc.ZMIN, orc.DIRICHLET, 0.3)
    P.set_bc(orc.ZMAX, orc.FLUX, 1e-6)


@pytest.mark.parametrize("mask", [False, True])
def test_assembly_symmetric_and_diagonally_dominant(orc, mask):
    P, rng = make_problem(orc, 4, 3, 5, mask=mask, g=[0.2, -0.1, 0.97])
    mixed_bcs(orc, P)
    h = rng.uniform(-3.0, 0.5, P.N)
    P.set_state(h)
    hm = h + rng.normal(0, 0.05, P.N)
    sysd = P.assemble(hm, 60.0)
    A = P.dense_matrix(sysd)
    assert np.array_equal(A, A.T)
    # weakly diagonally dominant, strictly where the capacity is positive
    off = np.abs(A).sum(axis=1) - np.abs(np.diag(A))
    assert np.all(np.diag(A) >= off)
    assert np.all(np.linalg.eigvalsh(A) > 0)


@pytest.mark.parametrize("g", [None, [0.3, 0.2, 0.932737905308882]])
def test_hydrostatic_state_has_zero_residual(orc, g):
    """h + z = const carries no flux through any face (Appendix A, zero-flux
    case); with h^n = h^m = hydrostatic, b - A h must vanish to round-off."""
    P, rng = make_problem(orc, 5, 4, 6, seed=3, mask=True, g=g)
    nx, ny, nz = P.shape
    gv = np.array(g if g is not None else [0, 0, 1.0])
    dx, dy, dz = 0.5, 0.7, 0.1
    i = np.arange(nx)[None, :, None]
    j = np.arange(ny)[:, None, None]
    k = np.arange(nz)[None, None, :]
    elev = gv[0] * (i + 0.5) * dx + gv[1] * (j + 0.5) * dy + gv[2] * (k + 0.5) * dz
    h = (0.2 - elev).reshape(-1)            # order (j, i, k) == k + nz*(i + nx*j)
    # the only non-trivial boundary: Dirichlet bottom at the hydrostatic value
    # of the bottom face is column-dependent, so keep Dirichlet off and use
    # no-flow everywhere (total flux zero, gravity included)
    P.set_state(h)
    sysd = P.assemble(h, 1e3)
    r = sysd["b"] - P.matvec(sysd, h)
    assert np.max(np.abs(r)) <= 1e-12 * np.max(np.abs(sysd["b"]))


def test_hydrostatic_with_dirichlet_bottom(orc):
    P, rng = make_problem(orc, 3, 2, 8, seed=4)
    dz = 0.1
    z = (np.arange(8) + 0.5) * dz
    h = np.tile(-0.5 - z, 6)
    P.set_bc(orc.ZMIN, orc.DIRICHLET, -0.5)      # h + z = -0.5 at the bottom face z = 0
    P.set_state(h)
    sysd = P.assemble(h, 1e3)
    r = sysd["b"] - P.matvec(sysd, h)
    assert np.max(np.abs(r)) <= 1e-12 * np.max(np.abs(sysd["b"]))


@pytest.mark.parametrize("mask", [False, True])
def test_pcg_matches_lapack(orc, mask):
    P, rng = make_problem(orc, 4, 3, 5, seed=7, mask=mask, g=[0.1, 0.0, 0.995])
    mixed_bcs(orc, P)
    h = rng.uniform(-2.0, 0.2, P.N)
    P.set_state(h)
    sysd = P.assemble(h + 0.01, 30.0)
    A = P.dense_matrix(sysd)
    x_ref = np.linalg.solve(A, sysd["b"])
    x, its = P.pcg(sysd, h, tol=1e-14)
    assert its > 0
    assert np.max(np.abs(x - x_ref)) <= 1e-11 * max(1.0, np.max(np.abs(x_ref)))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dic_exact_on_tridiagonal(orc, axis):
    """With couplings along one axis only, DIC keeps every entry of the
    Cholesky factor, so M = A: one PCG iteration and M^-1 r = A^-1 r
    (checked with LAPACK's banded solver)."""
    n = 9
    shape = [1, 1, 1]
    shape[axis] = n
    P, rng = make_problem(orc, *shape, seed=11)
    P.set_bc(orc.ZMIN, orc.DIRICHLET, -0.2)
    P.set_bc(orc.XMIN, orc.DIRICHLET, -0.1)
    h = rng.uniform(-2.0, -0.1, P.N)
    P.set_state(h)
    sysd = P.assemble(h * 1.01, 100.0)
    A = P.dense_matrix(sysd)
    ab = np.zeros((3, n))
    ab[0, 1:] = np.diag(A, 1)
    ab[1] = np.diag(A)
    ab[2, :-1] = np.diag(A, -1)
    r = rng.normal(size=n)
    z = P.dic_apply(sysd, r)
    z_ref = scipy.linalg.solve_banded((1, 1), ab, r)
    assert np.allclose(z, z_ref, rtol=1e-12, atol=0)
    x, its = P.pcg(sysd, h, tol=1e-13)
    assert its == 1


def test_dic_is_spd_preconditioner(orc):
    """M^-1 must be symmetric positive definite for PCG: z1.r2 == z2.r1."""
    P, rng = make_problem(orc, 4, 4, 4, seed=2)
    mixed_bcs(orc, P)
    h = rng.uniform(-2.0, 0.0, P.N)
    P.set_state(h)
    sysd = P.assemble(h, 10.0)
    r1, r2 = rng.normal(size=P.N), rng.normal(size=P.N)
    z1, z2 = P.dic_apply(sysd, r1), P.dic_apply(sysd, r2)
    assert z1 @ r2 == pytest.approx(z2 @ r1, rel=1e-12)
    assert z1 @ r1 > 0
