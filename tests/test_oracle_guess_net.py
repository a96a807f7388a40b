"""Pins of the CPU reference of the learned-guess network (oracle/guess_net.py)
against definitions it does not share code with: a brute-force per-cell
convolution written from the tap convention of include/rf_guess.h, central
finite differences of its FP64 loss, and the BF16 rounding rule."""
import numpy as np
import pytest

from oracle import guess_net as G


def brute_conv(x, W, shape):
    """y[cell, co] = sum over taps and ci of W[co, tap, ci] x[nbr(cell, tap), ci],
    with cell = k + nz (i + nx j) and tap = 9 (di+1) + 3 (dj+1) + (dk+1)."""
    nx, ny, nz = shape
    xf = x.reshape(-1, x.shape[-1])
    y = np.zeros((nx * ny * nz, W.shape[0]))
    for j in range(ny):
        for i in range(nx):
            for k in range(nz):
                c = k + nz * (i + nx * j)
                for di in (-1, 0, 1):
                    for dj in (-1, 0, 1):
                        for dk in (-1, 0, 1):
                            ii, jj, kk = i + di, j + dj, k + dk
                            if not (0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz):
                                continue
                            t = (di + 1) * 9 + (dj + 1) * 3 + (dk + 1)
                            y[c] += W[:, t, :] @ xf[kk + nz * (ii + nx * jj)]
    return y


def test_conv_matches_brute_force_definition():
    rng = np.random.default_rng(0)
    shape = (3, 4, 5)
    x = rng.normal(size=(4, 3, 5, 6))              # (ny, nx, nz, C)
    W = rng.normal(size=(7, 27, 6))
    y = G.conv(x, W).reshape(-1, 7)
    assert np.allclose(y, brute_conv(x, W, shape), rtol=1e-12, atol=1e-12)


def test_single_tap_picks_the_right_neighbour():
    """A weight only at tap (di, dj, dk) = (1, 0, -1) copies x(i+1, j, k-1)."""
    shape = (4, 3, 5)
    nx, ny, nz = shape
    x = np.arange(nx * ny * nz, dtype=float).reshape(ny, nx, nz, 1)
    W = np.zeros((1, 27, 1))
    W[0, 2 * 9 + 1 * 3 + 0, 0] = 1.0
    y = G.conv(x, W)[..., 0]
    for j in range(ny):
        for i in range(nx):
            for k in range(nz):
                want = x[j, i + 1, k - 1, 0] if (i + 1 < nx and k - 1 >= 0) else 0.0
                assert y[j, i, k] == want


def test_transpose_is_the_adjoint():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 4, 6, 5))
    d = rng.normal(size=(3, 4, 6, 2))
    W = rng.normal(size=(2, 27, 5))
    assert np.isclose(np.sum(G.conv(x, W) * d), np.sum(x * G.conv_transpose(d, W)), rtol=1e-12)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    shape = (3, 2, 5)
    N = 30
    p = G.init_params(seed=3, scale_out=1.0)
    hn = rng.uniform(-3, -0.5, N)
    hp = hn - rng.normal(0, 0.01, N)
    lnks = rng.normal(0, 1, N)
    target = hn + rng.normal(0, 0.01, N)
    loss, g = G.loss_and_grad(p, hn, hp, lnks, 2e-7, target, shape)
    idx = []
    for wo, bo in G.OFFSETS:
        idx += list(rng.choice(np.arange(wo, bo), 8, replace=False)) + [bo]
    for e in idx:
        h = 1e-5 * max(1.0, abs(p[e]))
        pp, pm = p.copy(), p.copy()
        pp[e] += h
        pm[e] -= h
        lp, _ = G.loss_and_grad(pp, hn, hp, lnks, 2e-7, target, shape)
        lm, _ = G.loss_and_grad(pm, hn, hp, lnks, 2e-7, target, shape)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[e]) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (e, fd, g[e])


def test_untrained_output_layer_gives_the_extrapolation():
    """y = 0: h^n + (h^n - h^{n-1}), which is h^n when the two states agree."""
    rng = np.random.default_rng(4)
    shape = (2, 2, 3)
    p = G.init_params(seed=1, scale_out=0.0)
    wo, bo = G.OFFSETS[3]
    p[bo] = 0.0
    hn = rng.uniform(-2, -1, 12)
    hp = hn - rng.normal(0, 0.01, 12)
    assert np.array_equal(G.predict(p, hn, hn, None, 0.0, shape), hn)
    assert np.array_equal(G.predict(p, hn, hp, None, 0.0, shape), hn + (hn - hp))


@pytest.mark.parametrize("x,want", [(1.0, 1.0), (1.00390625, 1.0), (1.01171875, 1.015625),
                                     (3.0e-39, 3.0e-39), (-2.5, -2.5), (65504.0, 65536.0)])
def test_bf16_rounding(x, want):
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins
    got = G.bf16(np.array([x]))[0]
    if x == 3.0e-39:
        assert abs(got - x) <= 2.0 ** -133
    else:
        assert got == want
