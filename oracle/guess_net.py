"""CPU reference of the learned Picard guess network (test infrastructure
only: used by tests/, never by the library).

Plain NumPy in FP64: each 3x3x3 convolution is the sum over the 27 taps of
the zero-padded, shifted input times that tap's weight matrix; the backward
pass applies the chain rule layer by layer (the transposed convolution is
the same sum with the taps mirrored).  Optionally every stored quantity is
rounded to BF16 where the GPU stores it (weights, features, activations,
output-gradient, layer gradients), so that the GPU gradients can be compared
at the precision they are computed in.  The network and its parameter
vector are the ones described in include/rf_guess.h; the network is an
extension of the paper's Picard loop, not part of its method, so there is no
passage of the paper to follow, and the reference is pinned by finite
differences of its own FP64 loss (tests/test_oracle_guess_net.py).
"""
import numpy as np

TAPS = 27
CIN = (4, 32, 32, 32)
COUT = (32, 32, 32, 1)
H_SCALE, DH_SCALE, RAIN_SCALE, OUT_SCALE = 10.0, 100.0, 1e7, 0.01


def param_offsets():
    """[(w_offset, b_offset)] per layer and the total count."""
    out, o = [], 0
    for ci, co in zip(CIN, COUT):
        out.append((o, o + co * TAPS * ci))
        o += co * TAPS * ci + co
    return out, o


OFFSETS, NPARAMS = param_offsets()


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params, rnd):
    Ws, bs = [], []
    for l, (wo, bo) in enumerate(OFFSETS):
        W = np.asarray(params[wo:bo], np.float64).reshape(COUT[l], TAPS, CIN[l])
        Ws.append(bf16(W) if rnd else W)
        bs.append(np.asarray(params[bo:bo + COUT[l]], np.float64))   # biases stay FP32
    return Ws, bs


def taps():
    for di in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for dk in (-1, 0, 1):
                yield (di + 1) * 9 + (dj + 1) * 3 + (dk + 1), di, dj, dk


def shifted(x, di, dj, dk):
    """out[j, i, k] = x[j + dj, i + di, k + dk] (zero outside); x is (ny, nx, nz, C)."""
    ny, nx, nz, _ = x.shape
    p = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    return p[1 + dj:1 + dj + ny, 1 + di:1 + di + nx, 1 + dk:1 + dk + nz, :]


def conv(x, W):
    """sum over taps of shifted(x) @ W[:, tap, :].T; x (ny, nx, nz, Cin), W (Cout, 27, Cin)."""
    out = np.zeros(x.shape[:3] + (W.shape[0],))
    for t, di, dj, dk in taps():
        out += shifted(x, di, dj, dk) @ W[:, t, :].T
    return out


def conv_transpose(d, W):
    """Gradient of conv with respect to its input: sum over taps of the
    mirrored shift of d times W[:, tap, :]."""
    out = np.zeros(d.shape[:3] + (W.shape[2],))
    for t, di, dj, dk in taps():
        out += shifted(d, -di, -dj, -dk) @ W[:, t, :]
    return out


def conv_weight_grad(x, d):
    """dW[co, tap, ci] = sum over cells of d[cell, co] x[cell + tap, ci]."""
    g = np.zeros((d.shape[3], TAPS, x.shape[3]))
    dd = d.reshape(-1, d.shape[3])
    for t, di, dj, dk in taps():
        g[:, t, :] = dd.T @ shifted(x, di, dj, dk).reshape(-1, x.shape[3])
    return g


def features(hn, hprev, lnks, rain, shape):
    nx, ny, nz = shape
    f = np.zeros((len(hn), 4))
    f[:, 0] = np.asarray(hn) / H_SCALE
    f[:, 1] = (np.asarray(hn) - np.asarray(hprev)) * DH_SCALE
    f[:, 2] = 0.0 if lnks is None else np.asarray(lnks)
    f[:, 3] = rain * RAIN_SCALE
    return f.reshape(ny, nx, nz, 4)


def forward(params, f, rnd=False):
    """Returns y (ny, nx, nz) and the list [x0, a1, a2, a3] of layer inputs."""
    Ws, bs = unpack(params, rnd)
    x = bf16(f) if rnd else f
    xs = [x]
    for l in range(3):
        a = np.maximum(conv(x, Ws[l]) + bs[l], 0.0)
        x = bf16(a) if rnd else a
        xs.append(x)
    y = conv(x, Ws[3])[..., 0] + bs[3][0]
    return y, xs


def first_iterate(hn, hprev, y):
    """h^{n+1,0} = h^n + (h^n - h^{n-1}) + 0.01 m y: the network's output y
    corrects the linear extrapolation in time."""
    hn, hprev = np.asarray(hn, dtype=np.float64), np.asarray(hprev, dtype=np.float64)
    return hn + (hn - hprev) + OUT_SCALE * np.asarray(y, dtype=np.float64).reshape(hn.shape)


def predict(params, hn, hprev, lnks, rain, shape, rnd=False):
    y, _ = forward(params, features(hn, hprev, lnks, rain, shape), rnd)
    return first_iterate(hn, hprev, y.reshape(-1))


def loss_and_grad(params, hn, hprev, lnks, rain, target, shape, rnd=False):
    """Loss 0.5/N sum ((h^{n+1,0} - target) / 0.01 m)^2 and its parameter gradient."""
    nx, ny, nz = shape
    N = nx * ny * nz
    f = features(hn, hprev, lnks, rain, shape)
    Ws, bs = unpack(params, rnd)
    y, xs = forward(params, f, rnd)
    r = (first_iterate(hn, hprev, y.reshape(-1)).reshape(ny, nx, nz)
         - np.asarray(target).reshape(ny, nx, nz)) / OUT_SCALE
    loss = 0.5 * np.sum(r * r) / N
    d = (r / N)[..., None]
    if rnd:
        d = bf16(d)
    grad = np.zeros(NPARAMS)
    for l in (3, 2, 1, 0):
        wo, bo = OFFSETS[l]
        grad[wo:bo] = conv_weight_grad(xs[l], d).reshape(-1)
        grad[bo:bo + COUT[l]] = d.reshape(-1, COUT[l]).sum(0)
        if l > 0:
            dx = conv_transpose(d, Ws[l]) * (xs[l] > 0)
            d = bf16(dx) if rnd else dx
    return loss, grad


def init_params(seed=0, scale_out=0.0):
    """He-normal hidden layers; the output layer scaled by scale_out."""
    rng = np.random.default_rng(seed)
    p = np.zeros(NPARAMS)
    for l, (wo, bo) in enumerate(OFFSETS):
        sd = np.sqrt(2.0 / (TAPS * CIN[l])) * (scale_out if l == 3 else 1.0)
        p[wo:bo] = rng.normal(0.0, sd, bo - wo)
        p[bo:bo + COUT[l]] = rng.normal(0.0, 0.05, COUT[l])
    return p


def loss_grad_abs(params, hn, hprev, lnks, rain, target, shape):
    """loss_and_grad with the BF16 roundings (rnd=True), and for every
    parameter the sum of the magnitudes of the terms its gradient adds up:
    sum over cells of |d| |x| for a weight, of |d| for a bias.  A difference
    between two evaluations that round their operands to BF16 (2^-8 relative)
    and add in different orders is bounded by a few 2^-8 times that sum."""
    nx, ny, nz = shape
    N = nx * ny * nz
    f = features(hn, hprev, lnks, rain, shape)
    Ws, bs = unpack(params, True)
    y, xs = forward(params, f, True)
    r = (first_iterate(hn, hprev, y.reshape(-1)).reshape(ny, nx, nz)
         - np.asarray(target).reshape(ny, nx, nz)) / OUT_SCALE
    loss = 0.5 * np.sum(r * r) / N
    d = bf16((r / N)[..., None])
    grad, mag = np.zeros(NPARAMS), np.zeros(NPARAMS)
    for l in (3, 2, 1, 0):
        wo, bo = OFFSETS[l]
        grad[wo:bo] = conv_weight_grad(xs[l], d).reshape(-1)
        mag[wo:bo] = conv_weight_grad(np.abs(xs[l]), np.abs(d)).reshape(-1)
        grad[bo:bo + COUT[l]] = d.reshape(-1, COUT[l]).sum(0)
        mag[bo:bo + COUT[l]] = np.abs(d).reshape(-1, COUT[l]).sum(0)
        if l > 0:
            d = bf16(conv_transpose(d, Ws[l]) * (xs[l] > 0))
    return loss, grad, mag


def predict_abs(params, hn, hprev, lnks, rain, shape):
    """The network output y (BF16 roundings) and, per cell, the sum of the
    magnitudes of the terms of the output layer: sum over taps and channels of
    |W| |x| plus |b|."""
    Ws, bs = unpack(params, True)
    y, xs = forward(params, features(hn, hprev, lnks, rain, shape), True)
    mag = conv(np.abs(xs[3]), np.abs(Ws[3]))[..., 0] + abs(bs[3][0])
    return y.reshape(-1), mag.reshape(-1)

