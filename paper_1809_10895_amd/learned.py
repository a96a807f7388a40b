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
from .binding import RF_ERR_LINEAR, RF_ERR_NONFINITE, RF_ERR_NOT_CONVERGED, Guess, Solver

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


def ebats_run(S, t0q, t_end, dt0, dt_max, G=None, lnks=None, few_iters=3, inc_after=10,
              max_iters=8, factor=1.3, dt_min=1e-6):
    """The library's adaptive time loop (rf_run with EBATS, Sec. 2.2) driven
    from here, one rf_step per attempt, so that a step can start from the
    network's first iterate.  The network corrects the linear extrapolation
    h^n + (h^n - h^{n-1}) of equal steps, so it is used when dt equals the
    last accepted step's; otherwise (dt grown, or clipped at a change of the
    rain rate or at t_end) the step is left to the solver's own first
    iterate (h^n, or the extrapolation scaled by dt/dt_prev when the solver
    has first_iterate = 1).  S must have max_picard = max_iters.  Returns
    the counts of the run and the seconds spent in the network."""
    import torch
    seg_t, seg_q = np.asarray(t0q[0], np.float64), np.asarray(t0q[1], np.float64)

    def before(t):
        return t < t_end * (1.0 - 1e-15) - 1e-12

    def next_change(t):
        later = seg_t[seg_t > t * (1.0 + 1e-15) + 1e-12]
        return float(later.min()) if later.size else np.inf

    def rain_at(t):
        k = np.nonzero(seg_t <= t)[0]
        return float(seg_q[k[-1]]) if k.size else 0.0

    h_now, t = S.get_state()
    h_prev = torch.empty_like(h_now)
    guess = torch.empty_like(h_now)
    dt_cur, dt_prev, easy = dt0, 0.0, 0
    out = {"accepted": 0, "rejected": 0, "picard_total": 0, "learned_steps": 0, "predict_s": 0.0}
    while before(t):
        dt, clipped = dt_cur, False
        tf = next_change(t)
        if t + dt > tf:
            dt, clipped = tf - t, True
        if t + dt > t_end:
            dt, clipped = t_end - t, True
        g = None
        if G is not None and dt_prev > 0.0 and dt == dt_prev:
            tp = time.perf_counter()
            G.predict(h_now, h_prev, lnks, rain_at(t), out=guess)
            out["predict_s"] += time.perf_counter() - tp
            g = guess
        s, st = S.step(dt, g)
        out["picard_total"] += st["picard_iters"]
        if s != 0:
            if s not in (RF_ERR_NOT_CONVERGED, RF_ERR_LINEAR, RF_ERR_NONFINITE):
                raise RuntimeError(S.last_error())
            out["rejected"] += 1
            dt_cur, easy = dt / factor, 0
            if dt_cur < dt_min:
                raise RuntimeError("EBATS: dt %g fell below dt_min" % dt_cur)
            continue
        out["accepted"] += 1
        out["learned_steps"] += g is not None
        h_prev, h_now = h_now, h_prev
        t = S.get_state(out=h_now)[1]
        dt_prev = dt
        if not clipped:
            dt_cur = dt
        if st["picard_iters"] <= few_iters:
            easy += 1
            if easy >= inc_after:
                dt_cur, easy = min(dt_cur * factor, dt_max), 0
        else:
            easy = 0
    return out


def evaluate_ebats(params, seed, days=1.0, nx=128, ny=128, nz=64, dt0=600.0, dt_max=3600.0):
    """A simulated day (or `days`) of the hillslope with the rain series of
    `seed` under EBATS from its initial state, tol 1e-6 m: the paper's loop
    in FP64 through rf_run, the same loop driven from here (ebats_run), the
    extrapolated first iterate with mixed precision through rf_run, and the
    learned first iterate with mixed precision through ebats_run.  Wall time
    per simulated day, counts, and the water-balance error of each run."""
    import torch
    w = W.hillslope(nx=nx, ny=ny, nz=nz, seed=seed)
    w.dt = dt0
    t_end = days * 86400.0
    t0q = rain_steps(seed, int(np.ceil(t_end / 600.0)) + 1, 600.0)
    lnks = torch.tensor(w.lnks, dtype=torch.float64, device="cuda")
    runs = (("plain_fp64", 0, 0, "rf_run"), ("plain_fp64_loop", 0, 0, "loop"),
            ("extrapolate_mixed", 1, 1, "rf_run"), ("learned_mixed", 1, 1, "loop"))
    out = {"workload": "hillslope %dx%dx%d seed %d with its rain series, EBATS %g s to %g s, "
                       "%g simulated day(s)" % (nx, ny, nz, seed, dt0, dt_max, days)}
    for name, prec, fi, driver in runs:
        S = make_solver(w, t0q, precision=prec, first_iterate=fi)
        S.set_options(dt0=dt0, dt_max=dt_max, precond=1, precision=prec, first_iterate=fi,
                      tol_picard=1e-6, tol_cg=1e-8, ebats=1,
                      max_picard=8 if driver == "loop" else 50)
        G = None
        if name == "learned_mixed":
            G = Guess(nx, ny, nz)
            G.set_params(params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if driver == "rf_run":
            s, rs = S.run(t_end)
            if s != 0:
                raise RuntimeError(S.last_error())
            r = {"accepted": rs["accepted"], "rejected": rs["rejected"],
                 "picard_total": rs["picard_total"]}
        else:
            r = ebats_run(S, t0q, t_end, dt0, dt_max, G=G, lnks=lnks)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        mb = S.mass_balance()
        r["wall_s_per_simulated_day"] = el / days
        r["water_balance_error_m3"] = mb["error"]
        r["storage_change_m3"] = mb["storage"] - mb["storage0"]
        out[name] = r
    base = out["plain_fp64"]["wall_s_per_simulated_day"]
    for name in ("plain_fp64_loop", "extrapolate_mixed", "learned_mixed"):
        out[name]["speedup_vs_plain_fp64"] = base / out[name]["wall_s_per_simulated_day"]
    return out


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
