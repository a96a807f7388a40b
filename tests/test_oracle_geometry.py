"""Pins of the oracle's lateral face geometry (Sec. 2.2, last paragraph: face
conductivity by linear interpolation, transmissivity A_f K_f / d_f, explicit
gravity A_f K_f (g . n_f)) on grids with dx != dy != dz.

The face area A_f multiplies both the transmissivity and the gravity term, so
it cancels from hydrostatic equilibrium, from every steady state (each face
carries the same flux) and from the water balance.  Two pins that do not
cancel it:

* the same transient 1-D problem laid along x, along y and along z, with the
  three spacings permuted so that the cell volume and the area of the faces
  across the flow are the same in all three runs: the heads must agree;
* a face-by-face NumPy assembly of the Picard system written here from the
  paper (no code shared with the oracle), compared entry by entry with the
  oracle's assembly on a small anisotropic, masked, tilted grid with mixed
  boundary conditions.
"""
import numpy as np
import pytest

from tests.golden_data import SOILS

# spacing along the flow, and the two spacings across it (all different)
D_ALONG, A_ACROSS, B_ACROSS = 0.02, 0.7, 1.3


def _axis_run(orc, axis, soil, nseg):
    """nseg cells along `axis`; the other two spacings are A_ACROSS and
    B_ACROSS in cyclic order, so the cross-section is A_ACROSS * B_ACROSS and
    the cell volume D_ALONG * A_ACROSS * B_ACROSS in every orientation."""
    n = [1, 1, 1]
    d = [0.0, 0.0, 0.0]
    n[axis] = nseg
    d[axis] = D_ALONG
    d[(axis + 1) % 3] = A_ACROSS
    d[(axis + 2) % 3] = B_ACROSS
    g = [0.0, 0.0, 0.0]
    g[axis] = 1.0                     # "up" along the axis of the column
    P = orc.Problem(n[0], n[1], n[2], d[0], d[1], d[2], grad_elev=np.array(g))
    P.set_soil(np.array([soil]))
    lo, hi = 2 * axis, 2 * axis + 1   # XMIN/XMAX, YMIN/YMAX or ZMIN/ZMAX
    P.set_bc(lo, orc.FREE_DRAINAGE)
    P.set_bc(hi, orc.FLUX, 3e-6)
    return P


@pytest.mark.parametrize("soil_name", ["loam_sec3_1", "column100"])
def test_axis_permutation_transient(orc, soil_name):
    """Rain into a dry column through its top face with a free-draining base:
    the transient heads depend on the ratio of face area to cell volume, and
    must be identical whichever grid axis the column lies along."""
    soil = SOILS[soil_name]
    nseg = 40
    h0 = np.linspace(-3.0, -0.5, nseg)          # wetter towards the top
    out = []
    for axis in range(3):
        P = _axis_run(orc, axis, soil, nseg)
        P.set_options(tol_picard=1e-11, tol_cg=1e-14, max_picard=200, ebats=0, dt0=30.0)
        assert P.set_state(h0) == 0
        s, rs = P.run(1800.0)
        assert s == 0 and rs["accepted"] == 60, rs
        h, _ = P.get_state()
        mb = P.mass_balance()
        out.append((h, mb))
    # the run moves water: the heads change by far more than the bar below
    assert np.abs(out[0][0] - h0).max() > 0.05
    for h, mb in out[1:]:
        assert np.abs(h - out[0][0]).max() <= 1e-12
        assert mb["storage"] == pytest.approx(out[0][1]["storage"], rel=1e-13)
    # the top inflow is the prescribed rate times the cross-section
    inflow_top = out[2][1]["inflow"][orc.ZMAX]
    assert inflow_top == pytest.approx(3e-6 * 1800.0 * A_ACROSS * B_ACROSS, rel=1e-12)
    assert out[0][1]["inflow"][orc.XMAX] == pytest.approx(inflow_top, rel=1e-12)
    assert out[1][1]["inflow"][orc.YMAX] == pytest.approx(inflow_top, rel=1e-12)


def test_lateral_flow_slice_transposes(orc):
    """Lateral flow in a vertical slice along x on a grid with dy != dx, and
    the same slice laid along y with dx and dy swapped: the heads must be the
    same.  Pins the lateral coupling's indexing and the Dirichlet side face
    on a non-square grid (the face areas themselves are pinned by the axis
    permutation and the face-by-face assembly)."""
    soil = SOILS["hillslope"]
    nl, nz = 6, 8
    dl, dw, dz = 0.5, 1.7, 0.1                 # along the slice, across it, vertical
    rng = np.random.default_rng(12)
    lnks = rng.normal(0.0, 0.8, (nl, nz))
    h0 = -1.0 - 0.3 * rng.random((nl, nz))
    res = []
    for axis in (0, 1):
        if axis == 0:
            P = orc.Problem(nl, 1, nz, dl, dw, dz)
            ln = lnks.reshape(-1)              # cell k + nz*i
            hh = h0.reshape(-1)
            P.set_bc(orc.XMIN, orc.DIRICHLET, -0.2)
        else:
            P = orc.Problem(1, nl, nz, dw, dl, dz)
            ln = lnks.reshape(-1)              # cell k + nz*j (nx = 1)
            hh = h0.reshape(-1)
            P.set_bc(orc.YMIN, orc.DIRICHLET, -0.2)
        P.set_soil(np.array([soil]), None, ln)
        P.set_bc(orc.ZMAX, orc.FLUX, 1e-6)
        P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
        P.set_options(tol_picard=1e-11, tol_cg=1e-14, max_picard=200, ebats=0, dt0=120.0)
        assert P.set_state(hh) == 0
        assert P.run(3600.0)[0] == 0
        res.append((P.get_state()[0], P.mass_balance()))
    assert np.abs(res[0][0] - h0.reshape(-1)).max() > 0.01
    assert np.abs(res[0][0] - res[1][0]).max() <= 1e-12
    assert res[0][1]["inflow"][orc.XMIN] == pytest.approx(res[1][1]["inflow"][orc.YMIN], rel=1e-11)


# ---------------------------------------------------------------------------
# independent face-by-face assembly (NumPy), written from Sec. 1 and Sec. 2.2
# ---------------------------------------------------------------------------

def _vg(h, tr, ts, alpha, n, ks, S):
    """theta~, C, K of Eqs. 2-4 as printed (Se^(1/m) with 1/m = n/(n-1)),
    plus S h above saturation for theta~ and C = S there."""
    m = 1.0 - 1.0 / n
    if h >= 0.0:
        return ts + S * h, S, ks
    x = (alpha * -h) ** n
    se = (1.0 + x) ** (-m)
    theta = tr + (ts - tr) * se
    cap = (ts - tr) * alpha * n * m * (alpha * -h) ** (n - 1.0) * (1.0 + x) ** (-m - 1.0)
    k = ks * np.sqrt(se) * (1.0 - (1.0 - se ** (1.0 / m)) ** m) ** 2
    return theta, cap, k


def _reference_system(nx, ny, nz, dx, dy, dz, ktop, g, layers, layer_of, lnks, bcs, hm, hn, dt,
                      chord_eps=1e-9):
    """diag, off[6][N], b of one Picard iteration, face by face.

    Cell (i,j,k) is index k + nz*(i + nx*j).  Directions 0..5 = -x,+x,-y,+y,
    -z,+z.  For an interior face between active P and N:
      T = A K_f / d with K_f = (K_P + K_N)/2,  diag_P += T,  off = -T,
      b_P += A K_f (g . n)  (explicit gravity, outward normal n).
    Boundary faces: Dirichlet h_b -> T_b = A K(h_b) / (d/2), diag += T_b,
    b += T_b h_b + A K(h_b) (g . n); flux q -> b += A q; free drainage ->
    b += A K_P (g . n); no flow and faces to masked cells -> nothing.
    Storage: chord slope C = (theta~(h^m) - theta~(h^n)) / (h^m - h^n)
    (Eq. 3 when |h^m - h^n| < chord_eps); diag += V C / dt, b += V C h^n / dt."""
    N = nx * ny * nz
    V = dx * dy * dz
    spacing = {0: dx, 1: dy, 2: dz}
    # area of a face normal to each axis: the product of the other two spacings
    face_area = {0: dy * dz, 1: dx * dz, 2: dx * dy}
    diag = np.zeros(N)
    off = np.zeros((6, N))
    b = np.zeros(N)
    K = np.zeros(N)

    def idx(i, j, k):
        return k + nz * (i + nx * j)

    def active(i, j, k):
        return 0 <= i < nx and 0 <= j < ny and 0 <= k < ktop[i + nx * j]

    def params(c):
        p = list(layers[layer_of[c]])
        p[4] = p[4] * np.exp(lnks[c])
        return p

    for j in range(ny):
        for i in range(nx):
            for k in range(nz):
                c = idx(i, j, k)
                if not active(i, j, k):
                    diag[c] = 1.0
                    b[c] = hm[c]
                    continue
                p = params(c)
                th_m, cap_m, K[c] = _vg(hm[c], *p)
                th_n, _, _ = _vg(hn[c], *p)
                dh = hm[c] - hn[c]
                C = (th_m - th_n) / dh if abs(dh) >= chord_eps else cap_m
                diag[c] = V * C / dt
                b[c] = V * C * hn[c] / dt
    steps = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    for j in range(ny):
        for i in range(nx):
            for k in range(nz):
                if not active(i, j, k):
                    continue
                c = idx(i, j, k)
                for d, (di, dj, dk) in enumerate(steps):
                    axis = d // 2
                    outward = 1.0 if d % 2 else -1.0
                    gn = outward * g[axis]
                    A = face_area[axis]
                    dist = spacing[axis]
                    i2, j2, k2 = i + di, j + dj, k + dk
                    inside_box = 0 <= i2 < nx and 0 <= j2 < ny and k2 >= 0
                    top_of_column = d == 5 and k2 >= ktop[i + nx * j]
                    if inside_box and not top_of_column:
                        if not active(i2, j2, k2):
                            continue
                        Kf = 0.5 * (K[c] + K[idx(i2, j2, k2)])
                        T = A * Kf / dist
                        diag[c] += T
                        off[d, c] = -T
                        b[c] += A * Kf * gn
                        continue
                    kind, value = bcs.get(d, ("noflow", 0.0))
                    if kind == "dirichlet":
                        Kb = _vg(value, *params(c))[2]
                        Tb = A * Kb / (0.5 * dist)
                        diag[c] += Tb
                        b[c] += Tb * value + A * Kb * gn
                    elif kind == "flux":
                        b[c] += A * value
                    elif kind == "free":
                        b[c] += A * K[c] * gn
    return diag, off, b


def test_assembly_matches_face_by_face_reference(orc):
    nx, ny, nz = 4, 3, 5
    dx, dy, dz = 0.9, 0.35, 0.12
    g = np.array([0.2, -0.1, 0.974679])
    ktop = np.array([5, 4, 5, 3,
                     5, 5, 2, 5,
                     1, 5, 4, 0], np.int32)
    layers = [SOILS["eq5_layer2"], SOILS["loam_sec3_1"]]
    rng = np.random.default_rng(21)
    N = nx * ny * nz
    layer_of = rng.integers(0, 2, N).astype(np.uint8)
    lnks = rng.normal(0.0, 0.7, N)
    hn = -0.2 - 1.5 * rng.random(N)
    hm = hn + rng.uniform(-0.3, 0.3, N)
    hm[7] = hn[7]                 # the analytic capacity branch
    hm[20] = 0.05                 # a saturated cell (C = S side of the chord)
    P = orc.Problem(nx, ny, nz, dx, dy, dz, ktop=ktop, grad_elev=g)
    P.set_soil(np.array(layers), layer_of, lnks)
    P.set_bc(orc.XMIN, orc.DIRICHLET, -0.4)
    P.set_bc(orc.XMAX, orc.FREE_DRAINAGE)
    P.set_bc(orc.YMIN, orc.FLUX, 2e-6)
    P.set_bc(orc.YMAX, orc.DIRICHLET, 0.1)
    P.set_bc(orc.ZMIN, orc.FREE_DRAINAGE)
    P.set_bc(orc.ZMAX, orc.FLUX, -4e-7)
    P.set_state(hn)
    dt = 45.0
    sysd = P.assemble(hm, dt)
    bcs = {0: ("dirichlet", -0.4), 1: ("free", 0.0), 2: ("flux", 2e-6), 3: ("dirichlet", 0.1),
           4: ("free", 0.0), 5: ("flux", -4e-7)}
    diag, off, b = _reference_system(nx, ny, nz, dx, dy, dz, ktop, g, layers, layer_of, lnks,
                                     bcs, hm, hn, dt)
    act = P.active_mask()
    assert act.sum() > 40 and (~act).sum() > 5
    # inactive cells: identity rows carrying h^m
    assert np.array_equal(sysd["diag"][~act], diag[~act])
    assert np.array_equal(sysd["b"][~act], b[~act])
    # active rows, against the size of the active diagonal (Eq. 4 as printed
    # and the oracle's cancellation-free form differ by a few ulps)
    scale = np.abs(diag[act]).max()
    assert np.abs(sysd["diag"][act] - diag[act]).max() <= 1e-12 * scale
    assert np.abs(sysd["off"] - off).max() <= 1e-12 * scale
    # b mixes V C h^n / dt with the face terms: compare against its own size
    bscale = np.abs(b[act]).max()
    assert np.abs(sysd["b"][act] - b[act]).max() <= 1e-12 * bscale
    # every lateral direction is exercised, with different areas per axis
    for d in range(6):
        assert (off[d] != 0).sum() > 0
