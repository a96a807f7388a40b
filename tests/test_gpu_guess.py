"""GPU checks of the learned Picard guess (include/rf_guess.h): the MFMA
forward pass and the hand-written gradients against the CPU reference
(oracle/guess_net.py, with the same BF16 roundings), training, and what a
trained network gains over plain Picard on held-out seeds."""
import os

import numpy as np
import pytest

from oracle import guess_net as R
from paper_1809_10895_amd import learned
from paper_1809_10895_amd import workloads as W
from paper_1809_10895_amd.binding import Guess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def sample(shape, seed):
    rng = np.random.default_rng(seed)
    N = int(np.prod(shape))
    hn = rng.uniform(-3.0, -0.2, N)
    hp = hn - rng.normal(0, 0.02, N)
    lnks = rng.normal(0, 1, N)
    target = hn + rng.normal(0, 0.01, N)
    return hn, hp, lnks, target


# 70 cells in z: one full 64-cell tile and a ragged one; 11 x 9 columns
SHAPE = (11, 9, 70)


def test_forward_matches_reference():
    p = R.init_params(seed=5, scale_out=1.0).astype(np.float32)
    hn, hp, lnks, _ = sample(SHAPE, 1)
    G = Guess(*SHAPE)
    G.set_params(p)
    got = G.predict(dev(hn), dev(hp), dev(lnks), 3e-7).cpu().numpy()
    want = R.predict(p.astype(np.float64), hn, hp, lnks, 3e-7, SHAPE, rnd=True)
    base = hn + (hn - hp)                     # the extrapolation the network corrects
    y_g, y_r = (got - base) / R.OUT_SCALE, (want - base) / R.OUT_SCALE
    # Per cell: both sides round the same stored quantities to BF16, and FP32
    # and FP64 sums can move an activation across a BF16 rounding boundary
    # (2^-8 relative), so each output differs by at most about 2^-8 times the
    # sum of the magnitudes of its output layer's terms (sum |W| |x| + |b|;
    # measured 2.5e-4 of it).
    y_m, mag = R.predict_abs(p.astype(np.float64), hn, hp, lnks, 3e-7, SHAPE)
    assert np.allclose(y_m, y_r, rtol=0, atol=1e-12)
    assert np.all(np.abs(y_g - y_r) <= 2.0 ** -8 * mag)
    assert np.corrcoef(y_g, y_r)[0, 1] >= 0.9999


def test_gradient_matches_reference():
    shape = (6, 5, 70)
    p = R.init_params(seed=6, scale_out=1.0).astype(np.float32)
    hn, hp, lnks, target = sample(shape, 2)
    G = Guess(*shape)
    G.set_params(p)
    loss_g, grad_g = G.gradient(dev(hn), dev(hp), dev(lnks), 3e-7, dev(target))
    loss_r, grad_r, mag = R.loss_grad_abs(p.astype(np.float64), hn, hp, lnks, 3e-7, target, shape)
    assert loss_g == pytest.approx(loss_r, rel=1e-3)
    g = grad_g.astype(np.float64)
    # Per parameter: a gradient is a sum over cells of (upstream gradient) x
    # (activation), both rounded to BF16 on both sides; an operand that lands
    # on the other side of a BF16 rounding boundary moves its term by 2^-8,
    # and upstream gradients carry such differences from the layers above, so
    # every element stays within a few 2^-8 of the sum of the magnitudes of
    # its terms (measured: at most 3.0 x 2^-8, in layer 1).
    assert np.all(np.abs(g - grad_r) <= 2.0 ** -5 * mag), \
        float(np.max(np.abs(g - grad_r) / np.maximum(mag, 1e-300)))
    # Per tap of every layer (a wrong tap or channel moves a whole block, not
    # single elements), and per output channel: relative L2 error.
    for l, (wo, bo) in enumerate(R.OFFSETS):
        gw = g[wo:bo].reshape(R.COUT[l], R.TAPS, R.CIN[l])
        rw = grad_r[wo:bo].reshape(R.COUT[l], R.TAPS, R.CIN[l])
        for t in range(R.TAPS):
            rel = np.linalg.norm(gw[:, t] - rw[:, t]) / np.linalg.norm(rw[:, t])
            assert rel <= 3e-2, (l, t, rel)
        for co in range(R.COUT[l]):
            rel = np.linalg.norm(gw[co] - rw[co]) / np.linalg.norm(rw[co])
            assert rel <= 3e-2, (l, co, rel)
        gb, rb = g[bo:bo + R.COUT[l]], grad_r[bo:bo + R.COUT[l]]
        assert np.all(np.abs(gb - rb) <= 2.0 ** -5 * mag[bo:bo + R.COUT[l]]), l


def test_untrained_network_returns_the_extrapolation():
    hn, hp, lnks, _ = sample(SHAPE, 3)
    G = Guess(*SHAPE, seed=1)
    got = G.predict(dev(hn), dev(hp), dev(lnks), 0.0).cpu().numpy()
    assert np.array_equal(got, hn + (hn - hp))


def test_training_fits_one_solver_step():
    trajs, w = [], None
    tr, w = learned.trajectory(100, 3, nx=32, ny=32, nz=64)
    shape = (32, 32, 64)
    G = Guess(*shape, seed=0)
    hn, hp, tg = tr.states[1], tr.states[0], tr.states[2]
    losses = [G.train_step(hn, hp, tr.lnks, tr.rain[1], tg, 2e-3) for _ in range(150)]
    assert np.isfinite(losses).all()
    assert np.mean(losses[-10:]) < 0.3 * losses[0], (losses[0], losses[-10:])


def test_learned_guess_cuts_picard_iterations():
    """Trained on eight seeds of a 48 x 48 x 64 hillslope (24 steps each, 6000
    Adam steps), evaluated on a held-out seed.  The network corrects the
    linear extrapolation in time (its zero-parameter form), and its first
    iterate is far closer to the converged state than that extrapolation;
    plain Picard from it needs fewer iterations than from h^n and no more
    than from the extrapolation, and the converged states agree."""
    nx, ny, nz, nsteps = 48, 48, 64, 24
    trajs = [learned.trajectory(s, nsteps, nx=nx, ny=ny, nz=nz)[0] for s in range(100, 108)]
    params, losses = learned.train(trajs, (nx, ny, nz), 6000, crop_xy=(32, 32), lr=3e-4)
    val, _ = learned.trajectory(200, nsteps, nx=nx, ny=ny, nz=nz)
    G = Guess(nx, ny, nz)

    def val_loss(p):
        G.set_params(p)
        return np.mean([G.gradient(val.states[n], val.states[max(n - 1, 0)], val.lnks, val.rain[n],
                                   val.states[n + 1])[0] for n in range(nsteps)])

    extrap = val_loss(np.zeros_like(params))      # y = 0: the extrapolated first iterate
    trained = val_loss(params)
    assert trained < 0.2 * extrap, (trained, extrap)
    ev = learned.evaluate(params, 200, nsteps, nx=nx, ny=ny, nz=nz,
                          modes=("plain", "learned", "extrapolate"))
    assert ev["learned"]["picard_total"] < ev["plain"]["picard_total"], ev
    assert ev["learned"]["picard_total"] <= ev["extrapolate"]["picard_total"], ev
    # the runs converge every step to tol_picard = 1e-6 from different first
    # iterates; their states differ by the Picard stopping error only
    assert ev["max_abs_h_diff_m"] <= 2e-5, ev


def test_ebats_loop_from_python_equals_rf_run():
    """learned.ebats_run drives the library's adaptive time loop one rf_step
    at a time: without a network it takes the same steps as rf_run (same
    accepted and rejected steps, Picard totals and heads, bit for bit), with
    a change of the rain rate inside the run."""
    nx, ny, nz = 32, 24, 64
    w = W.hillslope(nx=nx, ny=ny, nz=nz, seed=201)
    t_end = 6 * 3600.0
    t0q = learned.rain_steps(201, 40, 600.0)
    out = []
    for driver in ("rf_run", "loop"):
        S = learned.make_solver(w, t0q)
        S.set_options(dt0=600.0, dt_max=3600.0, precond=1, tol_picard=1e-6, tol_cg=1e-8, ebats=1,
                      max_picard=8 if driver == "loop" else 50)
        if driver == "rf_run":
            s, rs = S.run(t_end)
            assert s == 0, S.last_error()
            r = (rs["accepted"], rs["rejected"], rs["picard_total"])
        else:
            e = learned.ebats_run(S, t0q, t_end, 600.0, 3600.0)
            r = (e["accepted"], e["rejected"], e["picard_total"])
        out.append((r, S.get_state()[0].cpu().numpy()))
    assert out[0][0] == out[1][0], (out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])


def test_learned_guess_under_ebats_closes_the_water_balance():
    """The committed network as the first iterate of the adaptive loop, with
    mixed precision: every step converges to tol_picard, the network starts
    most steps, and the water balance closes as in the plain run."""
    params = np.fromfile(os.path.join(ROOT, "paper_1809_10895_amd", "data", "guess_hillslope.f32"),
                         dtype=np.float32)
    ev = learned.evaluate_ebats(params, 202, days=0.25, nx=48, ny=48, nz=64)
    for k in ("plain_fp64", "plain_fp64_loop", "extrapolate_mixed", "learned_mixed"):
        r = ev[k]
        assert r["accepted"] > 0
        assert abs(r["water_balance_error_m3"]) <= 1e-6 * max(abs(r["storage_change_m3"]), 1.0), (k, r)
    assert ev["plain_fp64_loop"]["picard_total"] == ev["plain_fp64"]["picard_total"]
    lm = ev["learned_mixed"]
    assert lm["learned_steps"] >= 0.5 * lm["accepted"], lm
