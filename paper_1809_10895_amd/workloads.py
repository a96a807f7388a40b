"""Seeded synthetic inputs for the Richards-equation workloads.

This module only draws inputs (grids, soil fields, surfaces, rain series,
initial states); it holds none of the solver's arithmetic, so that the HIP
library and the CPU oracle are fed identical bytes.  Every generator takes
an explicit seed (numpy.random.default_rng).

Workloads (the paper's own field and benchmark data are not available; these
synthetic stand-ins carry the shapes and parameter ranges of its cases):

* column100  -- 1-D vertical infiltration column, 1x1x100 cells of 1 cm,
  van Genuchten theta_r 0.102, theta_s 0.368, alpha 3.35 1/m, n 2,
  Ks 9.22e-5 m/s; h0 = -10 m, top Dirichlet -0.75 m, free drainage; dt 10 s.
* hillslope  -- 128x128x64 cells of 1 x 1 x 0.1 m, lognormal Ks (ln-sigma 1,
  Gaussian-smoothed white noise with an 8-cell correlation length), n 1.6,
  alpha 2 1/m with the loam water contents of Sec. 3.1; h0 = -2 m, rain
  1e-7 m/s on top, no-flow sides, free drainage below; dt 600 s.
* watershed  -- 512x512x64 cells of 2 x 2 x 0.2 m (the mesh resolution of
  Sec. 4.2), fractal (Hurst 0.8) surface masking the cells above it, three
  soil layers with the parameters of Eq. 5 plus a lognormal Ks field, hourly
  rain (10% wet hours, exponential depths of mean 2 mm); EBATS from 60 s up
  to 3600 s.
* ensemble   -- 4096 independent 1-D columns of 1 cm cells, lengths uniform
  in 50..400 cells, per-column van Genuchten n in [1.3, 3], alpha in
  [0.5, 5] 1/m, log10 Ks in [-7, -4] (uniform), theta_r/theta_s of column100;
  h0 = -10 m, top Dirichlet -0.75 m, free drainage (the column100 set-up);
  EBATS from 10 s.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Face and boundary-type numbering of the C ABI (include/rf.h).
XMIN, XMAX, YMIN, YMAX, ZMIN, ZMAX = range(6)
NOFLOW, DIRICHLET, FLUX, FREE_DRAINAGE = range(4)

# (theta_r, theta_s, alpha [1/m], n, Ks [m/s], S [1/m])
SOIL_COLUMN100 = (0.102, 0.368, 3.35, 2.0, 9.22e-5, 1e-5)
SOIL_HILLSLOPE = (0.078, 0.43, 2.0, 1.6, 2.89e-6, 1e-5)
SOIL_EQ5 = ((0.08, 0.45, 2.3, 1.2, 1e-3, 1e-5),    # Sec. 3.2, Eq. 5, layer 1
            (0.20, 0.50, 2.1, 2.4, 1e-5, 1e-5),    # layer 2
            (0.15, 0.55, 1.7, 1.9, 1e-6, 1e-5))    # layer 3
EQ5_LAYER_BOTTOMS = (0.4, 2.0)   # depth [m] below the local surface where layers 2 and 3 start


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    soil: np.ndarray                     # nlayer x 6
    h0: np.ndarray                       # N
    bcs: list                            # [(face, type, value)]
    dt: float                            # fixed step (or EBATS dt0)
    t_end: float
    ktop: np.ndarray | None = None       # nx*ny int32
    grad_elev: np.ndarray | None = None
    layer: np.ndarray | None = None      # N uint8
    lnks: np.ndarray | None = None       # N float64
    forcing: dict = field(default_factory=dict)   # face -> (t_start, flux)
    ebats: bool = False
    dt_max: float = 3600.0
    model: int = 0

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def active_mask(self):
        kt = self.ktop if self.ktop is not None else np.full(self.nx * self.ny, self.nz)
        return (np.arange(self.nz)[None, :] < kt[:, None]).reshape(-1)

    @property
    def active_cells(self):
        return int(self.active_mask().sum())


def gaussian_field(shape, corr_cells, seed):
    """Standard-normal white noise (shape given as (ny, nx, nz) in memory order)
    convolved, periodically, with an isotropic Gaussian of standard deviation
    corr_cells (index units), re-standardised to mean 0 and variance 1."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    ks = [np.fft.fftfreq(n) for n in shape]
    kk = np.meshgrid(*ks, indexing="ij")
    k2 = sum(k * k for k in kk)
    kernel = np.exp(-2.0 * (np.pi ** 2) * (corr_cells ** 2) * k2)
    f = np.fft.ifftn(np.fft.fftn(w) * kernel).real
    f -= f.mean()
    f /= f.std()
    return f


def fbm_surface(nx, ny, hurst, seed):
    """Fractional-Brownian surface by spectral synthesis: random phases,
    amplitude |k|^-(H+1), normalised to [0, 1].  Shape (ny, nx)."""
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(nx)[None, :]
    ky = np.fft.fftfreq(ny)[:, None]
    k = np.sqrt(kx * kx + ky * ky)
    k[0, 0] = 1.0
    amp = k ** (-(hurst + 1.0))
    amp[0, 0] = 0.0
    phase = rng.uniform(0.0, 2.0 * np.pi, size=(ny, nx))
    noise = rng.standard_normal((ny, nx))
    s = np.fft.ifft2(amp * noise * np.exp(1j * phase)).real
    s -= s.min()
    s /= s.max()
    return s


def rain_series(t_end, seg=3600.0, p_wet=0.1, mean_depth=2e-3, seed=4):
    """Piecewise-constant rain: each `seg` seconds is wet with probability
    p_wet, with an exponential depth of mean `mean_depth` metres spread over
    the segment.  Returns (t_start, flux [m/s])."""
    rng = np.random.default_rng(seed)
    n = int(np.ceil(t_end / seg))
    wet = rng.random(n) < p_wet
    depth = rng.exponential(mean_depth, n)
    t0 = np.arange(n) * seg
    return t0, np.where(wet, depth / seg, 0.0)


def column100(t_end=86400.0):
    nz = 100
    return Workload(name="column100", nx=1, ny=1, nz=nz, dx=1.0, dy=1.0, dz=0.01,
                    soil=np.array([SOIL_COLUMN100]), h0=np.full(nz, -10.0),
                    bcs=[(ZMAX, DIRICHLET, -0.75), (ZMIN, FREE_DRAINAGE, 0.0)],
                    dt=10.0, t_end=t_end)


def hillslope(nx=128, ny=128, nz=64, seed=1, t_end=86400.0, rain=1e-7):
    f = gaussian_field((ny, nx, nz), 8.0, seed)          # memory order j, i, k
    return Workload(name="hillslope", nx=nx, ny=ny, nz=nz, dx=1.0, dy=1.0, dz=0.1,
                    soil=np.array([SOIL_HILLSLOPE]), h0=np.full(nx * ny * nz, -2.0),
                    bcs=[(ZMAX, FLUX, rain), (ZMIN, FREE_DRAINAGE, 0.0)],
                    dt=600.0, t_end=t_end, lnks=f.reshape(-1).astype(np.float64))


def watershed(nx=512, ny=512, nz=64, seeds=(2, 3, 4), t_end=86400.0, kmin=None):
    s_surf, s_ks, s_rain = seeds
    kmin = nz // 2 if kmin is None else kmin
    surf = fbm_surface(nx, ny, 0.8, s_surf)              # (ny, nx)
    ktop = (kmin + np.rint(surf * (nz - kmin))).astype(np.int32).reshape(-1)
    dz = 0.2
    k = np.arange(nz)[None, :]
    depth = (ktop[:, None] - k - 0.5) * dz               # below the local surface
    layer = np.where(depth < EQ5_LAYER_BOTTOMS[0], 0,
                     np.where(depth < EQ5_LAYER_BOTTOMS[1], 1, 2)).astype(np.uint8)
    lnks = gaussian_field((ny, nx, nz), 8.0, s_ks).reshape(-1)
    active = (k < ktop[:, None]).reshape(-1)
    h0 = np.where(active, -2.0, 0.0)
    t0, q = rain_series(t_end, seed=s_rain)
    return Workload(name="watershed", nx=nx, ny=ny, nz=nz, dx=2.0, dy=2.0, dz=dz,
                    soil=np.array(SOIL_EQ5), h0=h0,
                    bcs=[(ZMAX, FLUX, 0.0), (ZMIN, FREE_DRAINAGE, 0.0)],
                    dt=60.0, t_end=t_end, ktop=ktop, layer=layer.reshape(-1), lnks=lnks,
                    forcing={ZMAX: (t0, q)}, ebats=True, dt_max=3600.0)


def configure(w: Workload, target):
    """Hands a workload's soil, boundary conditions and forcing to any object
    with set_soil / set_bc / set_forcing methods of the C ABI's shape (the
    grid is given at construction or through setup_grid).  Returns target."""
    target.set_soil(w.soil, w.layer, w.lnks, model=w.model)
    for face, kind, value in w.bcs:
        target.set_bc(face, kind, value)
    for face, (t0, q) in w.forcing.items():
        target.set_forcing(face, t0, q)
    return target


@dataclass
class EnsembleWorkload:
    name: str
    lengths: np.ndarray                  # ncol int32
    dz: float
    soil: np.ndarray                     # ncol x 6
    h0: np.ndarray                       # packed, sum(lengths)
    bcs: list                            # [(face, type, value)], faces ZMIN / ZMAX
    dt: float                            # dt0
    t_end: float
    ebats: bool = True
    dt_max: float = 3600.0

    @property
    def ncol(self):
        return len(self.lengths)

    @property
    def offsets(self):
        return np.concatenate([[0], np.cumsum(self.lengths)[:-1]]).astype(np.int64)

    def column(self, c):
        """(length, soil row, initial heads) of column c."""
        o = self.offsets[c]
        return int(self.lengths[c]), self.soil[c], self.h0[o:o + self.lengths[c]]


def ensemble(ncol=4096, seed=5, lmin=50, lmax=400, t_end=3600.0, dt_max=3600.0):
    rng = np.random.default_rng(seed)
    lengths = rng.integers(lmin, lmax + 1, size=ncol).astype(np.int32)
    n = rng.uniform(1.3, 3.0, ncol)
    alpha = rng.uniform(0.5, 5.0, ncol)
    ks = 10.0 ** rng.uniform(-7.0, -4.0, ncol)
    tr, ts, _, _, _, S = SOIL_COLUMN100
    soil = np.stack([np.full(ncol, tr), np.full(ncol, ts), alpha, n, ks, np.full(ncol, S)], 1)
    return EnsembleWorkload(name="ensemble", lengths=lengths, dz=0.01, soil=soil,
                            h0=np.full(int(lengths.sum()), -10.0),
                            bcs=[(ZMAX, DIRICHLET, -0.75), (ZMIN, FREE_DRAINAGE, 0.0)],
                            dt=10.0, t_end=t_end, ebats=True, dt_max=dt_max)


def configure_ensemble(w: EnsembleWorkload, target):
    """Hands an ensemble's boundary conditions to an object with set_bc."""
    for face, kind, value in w.bcs:
        target.set_bc(face, kind, value)
    return target
