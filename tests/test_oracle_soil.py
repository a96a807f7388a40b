"""Pins of the oracle's soil functions (Eqs. 2-4) against values that do not
come from the oracle: a 50-digit `decimal` evaluation of the equations exactly
as printed, analytic limits, and the derivative relation C = d theta / dh."""
from decimal import Decimal, getcontext

import numpy as np
import pytest

# Soil parameter sets (theta_r, theta_s, alpha, n, Ks, S) quoted in the paper
# or in the benchmark configurations; see tests/golden/soils.txt.
from tests.golden_data import SOILS

H_GRID = [-1e3, -1e2, -31.6, -10.0, -3.0, -1.0, -0.75, -0.3, -0.1, -0.03, -1e-2, -1e-3,
          -1e-4, -1e-6]


def _dec_eqs(h, p):
    """Eqs. 2-4 as printed, with the n/(n-1) exponent, in 50-digit decimal."""
    getcontext().prec = 50
    tr, ts, a, n, Ks, S = (Decimal(float(v)) for v in p)
    h = Decimal(float(h))
    one = Decimal(1)
    if h >= 0:
        return ts + S * h, S, Ks
    m = one - one / n
    u = (-a * h) ** n
    Se = (one + u) ** (-m)
    theta = (ts - tr) * Se + tr
    C = (ts - tr) * a * n * m * (-a * h) ** (n - one) * (one + u) ** (-(2 - one / n))
    K = Ks * Se.sqrt() * (one - (one - Se ** (n / (n - one))) ** m) ** 2
    return theta, C, K


@pytest.mark.parametrize("name", list(SOILS))
def test_vg_against_decimal(orc, name):
    p = SOILS[name]
    th = orc.theta(H_GRID, p)
    cap = orc.capacity(H_GRID, p)
    k = orc.conductivity(H_GRID, p)
    for idx, h in enumerate(H_GRID):
        t_ref, c_ref, k_ref = (float(v) for v in _dec_eqs(h, p))
        assert th[idx] == pytest.approx(t_ref, rel=2e-15, abs=0), (name, h)
        assert cap[idx] == pytest.approx(c_ref, rel=2e-14, abs=0), (name, h)
        if k_ref > 1e-300:
            assert k[idx] == pytest.approx(k_ref, rel=5e-14, abs=0), (name, h)


@pytest.mark.parametrize("name", list(SOILS))
def test_vg_limits(orc, name):
    p = SOILS[name]
    tr, ts, a, n, Ks, S = p
    # saturated branch: theta = theta_s + S h, C = S, K = Ks
    assert orc.theta([0.0], p)[0] == ts
    assert orc.theta([0.5], p)[0] == pytest.approx(ts + 0.5 * S, rel=1e-15)
    assert orc.capacity([0.5], p)[0] == S
    assert orc.conductivity([0.0, 2.0], p).tolist() == [Ks, Ks]
    # continuity at h = 0^-
    assert orc.theta([-1e-12], p)[0] == pytest.approx(ts, rel=1e-9)
    assert orc.conductivity([-1e-30], p)[0] == pytest.approx(Ks, rel=1e-4)
    # dry limit: theta -> theta_r, K -> 0, K increasing in h
    # theta - theta_r = (ts-tr)(1+u)^-m <= (ts-tr) u^-m = (ts-tr)(alpha|h|)^-(n-1)
    hd = -1e9
    excess = orc.theta([hd], p)[0] - tr
    assert 0 <= excess <= (ts - tr) * (a * abs(hd)) ** (-(n - 1)) * (1 + 1e-12) + 1e-16
    kk = orc.conductivity(H_GRID, p)
    assert np.all(np.diff(kk) > 0)
    assert np.all(np.diff(orc.theta(H_GRID, p)) > 0)


@pytest.mark.parametrize("name", list(SOILS))
def test_capacity_is_derivative_of_theta(orc, name):
    """Eq. 3 must be the derivative of Eq. 2: Richardson-extrapolated central
    differences of the oracle's theta."""
    p = SOILS[name]
    for h in [-10.0, -3.0, -1.0, -0.4, -0.1, -0.02]:
        def d(step):
            return (orc.theta([h + step], p)[0] - orc.theta([h - step], p)[0]) / (2 * step)
        e = 1e-3 * abs(h)
        der = (4 * d(e / 2) - d(e)) / 3
        assert orc.capacity([h], p)[0] == pytest.approx(der, rel=1e-7), (name, h)


def test_gardner(orc):
    p = (0.05, 0.4, 3.0, 2.0, 1e-6, 1e-5)
    h = np.array([-2.0, -0.5, -1e-3])
    assert np.allclose(orc.conductivity(h, p, model=orc.GARDNER), 1e-6 * np.exp(3.0 * h),
                       rtol=1e-15, atol=0)
    assert orc.conductivity([0.1], p, model=orc.GARDNER)[0] == 1e-6
