"""Training and use of the learned Picard initial guess (include/rf_guess.h).

The network predicts the first Picard iterate of a backward-Euler step from
h^n, h^{n-1}, the ln Ks field and the rain rate; plain Picard then runs from
it to the same tolerance.  Data come from the solver itself: trajectories
of the hillslope workload (one seeded Ks field and rain series per seed),
each step's converged state being the target of the step before.  Training
runs on random lateral crops (the network's receptive field is 9 x 9 x 9
cells), evaluation on the full grid of held-out seeds.

Everything numeric runs in the HIP library (Solver for the steps, Guess for
the network's forward, backward and Adam kernels); PyTorch only holds the
device arrays and cuts the crops.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import workloads as W
from .binding import Guess, Solver

SOLVER_OPTS = dict(tol_picard=1e-6, tol_cg=1e-8, max_picard=50, ebats=0)


def rain_steps(seed, nsteps, dt, seg=3600.0, p_wet=0.4, mean_rate=3e-7, cap=2e-6):
    """Piecewise-constant rain of one seed: each `seg` seconds is wet with
    probability p_wet at an exponential rate of mean `mean_rate` (capped).
    Returns (segment starts, rates) for the forcing table."""
    rng = np.random.default_rng(seed + 7919)
    n = int(np.ceil(nsteps * dt / seg)) + 1
    wet = rng.random(n) < p_wet
    rate = np.minimum(rng.exponential(mean_rate, n), cap)
    return np.arange(n) * seg, np.where(wet, rate, 0.0)


@dataclass
class Trajectory:
    seed: int
    states: object          # torch (nsteps + 1, N) float64 on the device
    rain: np.ndarray        # rate during step n
    lnks: object            # torch (N,) float64
    picard: np.ndarray      # Picard iterations of each step (plain start)


def make_solver(w, t0q, precision=0, first_iterate=0):
    import torch
    S = Solver(0)
    S.setup_grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.ktop, w.grad_elev)
    W.configure(w, S)
    S.set_forcing(W.ZMAX, *t0q)
    S.set_options(dt0=w.dt, precond=1, precision=precision, first_iterate=first_iterate,
                  **SOLVER_OPTS)
    S.bind()
    assert S.set_state(torch.tensor(w.h0, dtype=torch.float64, device="cuda")) == 0, S.last_error()
    return S


def trajectory(seed, nsteps, nx=128, ny=128, nz=64, dt=600.0):
    """nsteps plain steps of the hillslope with Ks field and rain of `seed`."""
    import torch
    w = W.hillslope(nx=nx, ny=ny, nz=nz, seed=seed)
    w.dt = dt
    t0q = rain_steps(seed, nsteps, dt)
    S = make_solver(w, t0q)
    states = torch.empty((nsteps + 1, w.N), dtype=torch.float64, device="cuda")
    states[0] = S.get_state()[0]
    picard = np.zeros(nsteps, np.int64)
    rain = np.zeros(nsteps)
    for n in range(nsteps):
        rain[n] = t0q[1][min(int(n * dt // 3600.0), len(t0q[1]) - 1)]
        s, st = S.step(dt)
        assert s == 0, S.last_error()
        picard[n] = st["picard_iters"]
        states[n + 1] = S.get_state()[0]
    lnks = torch.tensor(w.lnks, dtype=torch.float64, device="cuda")
    return Trajectory(seed, states, rain, lnks, picard), w


def crop(t, shape, x0, y0, cx, cy):
    """Lateral crop [y0, y0+cy) x [x0, x0+cx) of a (..., N) tensor, contiguous."""
    nx, ny, nz = shape
    v = t.reshape(t.shape[:-1] + (ny, nx, nz))[..., y0:y0 + cy, x0:x0 + cx, :]
    return v.reshape(t.shape[:-1] + (cy * cx * nz,)).contiguous()


def train(trajs, shape, steps, crop_xy=(32, 32), lr=1e-3, seed=0, log_every=0, init=None,
          decay=0.3):
    """Adam on random (trajectory, step, crop) samples; returns the trained
    parameters and the loss history.  The step size is lr, then falls
    linearly to zero over the last `decay` fraction of the steps: at a
    constant rate the loss of single samples swings by more than an order of
    magnitude from one stretch of steps to the next, and the parameters
    depend on where training happens to stop."""
    nx, ny, nz = shape
    cx, cy = crop_xy
    rng = np.random.default_rng(seed)
    G = Guess(cx, cy, nz, seed=seed)
    if init is not None:
        G.set_params(init)
    losses = []
    for it in range(steps):
        tr = trajs[rng.integers(len(trajs))]
        n = int(rng.integers(len(tr.rain)))
        x0 = int(rng.integers(nx - cx + 1))
        y0 = int(rng.integers(ny - cy + 1))
        hn = crop(tr.states[n], shape, x0, y0, cx, cy)
        hp = crop(tr.states[max(n - 1, 0)], shape, x0, y0, cx, cy)
        tg = crop(tr.states[n + 1], shape, x0, y0, cx, cy)
        lk = crop(tr.lnks, shape, x0, y0, cx, cy)
        left = steps - it
        rate = lr * min(1.0, left / (decay * steps)) if decay > 0 else lr
        losses.append(G.train_step(hn, hp, lk, tr.rain[n], tg, rate))
        if log_every and (it + 1) % log_every == 0:
            print("train step %d loss %.4e" % (it + 1, np.mean(losses[-log_every:])), flush=True)
    return G.get_params(), np.array(losses)


def evaluate(params, seed, nsteps, nx=128, ny=128, nz=64, dt=600.0, precision=0,
             modes=("plain", "learned")):
    """The same nsteps with h^n as first iterate ("plain"), with the learned
    guess ("learned") and with the library's extrapolated first iterate
    ("extrapolate"); returns Picard totals, wall times and the largest state
    difference from the plain run."""
    import torch
    w = W.hillslope(nx=nx, ny=ny, nz=nz, seed=seed)
    w.dt = dt
    t0q = rain_steps(seed, nsteps, dt)
    lnks = torch.tensor(w.lnks, dtype=torch.float64, device="cuda")
    out = {}
    finals = {}
    for mode in modes:
        S = make_solver(w, t0q, precision=precision, first_iterate=1 if mode == "extrapolate" else 0)
        G = Guess(nx, ny, nz) if mode == "learned" else None
        if G is not None:
            G.set_params(params)
        h_prev = S.get_state()[0]
        h_now = torch.empty_like(h_prev)
        guess = torch.empty_like(h_prev)
        picard = 0
        t_pred = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for n in range(nsteps):
            rain = t0q[1][min(int(n * dt // 3600.0), len(t0q[1]) - 1)]
            if G is not None:
                S.get_state(out=h_now)
                tp = time.perf_counter()
                G.predict(h_now, h_prev, lnks, rain, out=guess)
                t_pred += time.perf_counter() - tp
                h_prev, h_now = h_now, h_prev
                s, st = S.step(dt, guess)
            else:
                s, st = S.step(dt)
            assert s == 0, S.last_error()
            picard += st["picard_iters"]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        finals[mode] = S.get_state()[0]
        out[mode] = {"picard_total": picard, "picard_per_step": picard / nsteps, "wall_s": el,
                     "wall_s_per_simulated_day": el / (nsteps * dt) * 86400.0,
                     "predict_s": t_pred}
    for mode in modes:
        if mode != "plain":
            out["max_abs_h_diff_m" + ("" if mode == "learned" else "_" + mode)] = float(
                (finals["plain"] - finals[mode]).abs().max())
    return out
