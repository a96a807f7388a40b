"""Trains the learned Picard initial guess on solver trajectories of the
128 x 128 x 64 hillslope and evaluates it on held-out seeds.

    python -m paper_1809_10895_amd.train_guess --out guess_hillslope.f32 [--json results.json]
    python -m paper_1809_10895_amd.train_guess --params guess_hillslope.f32 --json results.json

(--params: evaluate saved parameters only, keeping the training record of
an existing --json file.)

Training data: --steps-per-seed backward-Euler steps (dt 600 s, Picard tol
1e-6) of each training seed (Ks field and rain series of that seed).
Training: Adam on random 32 x 32 x 64 crops.  Evaluation: the same number of
steps on each held-out seed, plain Picard, with the learned first iterate
and with the extrapolated one (h^n + (h^n - h^{n-1})), in FP64 and in mixed
precision; Picard totals, wall time per simulated day and the largest head
difference from the plain run.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

if __package__ in (None, ""):
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_1809_10895_amd import learned  # noqa: E402


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-seeds", default="100-119")
    ap.add_argument("--eval-seeds", default="200-204")
    ap.add_argument("--steps-per-seed", type=int, default=100)
    ap.add_argument("--eval-steps", type=int, default=100)
    ap.add_argument("--train-steps", type=int, default=20000)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--crop", type=int, default=32)
    ap.add_argument("--grid", default="128,128,64")
    ap.add_argument("--out", default=None, help="where to write the FP32 parameters")
    ap.add_argument("--params", default=None, help="evaluate these FP32 parameters (no training)")
    ap.add_argument("--json", default=None, help="where to write the results")
    return ap.parse_args()


def seeds(s):
    a, b = s.split("-")
    return list(range(int(a), int(b) + 1))


def train(args, nx, ny, nz):
    t0 = time.perf_counter()
    trajs = []
    for s in seeds(args.train_seeds):
        tr, _ = learned.trajectory(s, args.steps_per_seed, nx=nx, ny=ny, nz=nz)
        trajs.append(tr)
        print("trajectory seed %d: %.2f Picard/step" % (s, tr.picard.mean()), flush=True)
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    params, losses = learned.train(trajs, (nx, ny, nz), args.train_steps,
                                   crop_xy=(args.crop, args.crop), lr=args.lr,
                                   log_every=max(args.train_steps // 10, 1))
    t_train = time.perf_counter() - t0
    params.astype(np.float32).tofile(args.out)
    res = {"grid": [nx, ny, nz], "train_seeds": args.train_seeds,
           "samples": len(seeds(args.train_seeds)) * args.steps_per_seed,
           "train_steps": args.train_steps, "lr": args.lr, "crop": args.crop,
           "data_s": round(t_data, 2), "train_s": round(t_train, 2),
           "loss_first_1000": float(np.mean(losses[:1000])),
           "loss_last_1000": float(np.mean(losses[-1000:]))}
    return params, res


def main():
    args = parse()
    nx, ny, nz = (int(v) for v in args.grid.split(","))
    if args.params:
        params = np.fromfile(args.params, dtype=np.float32)
        res = {}
        if args.json and os.path.exists(args.json):
            with open(args.json) as f:
                res = json.load(f)
        res["eval_command"] = "python -m paper_1809_10895_amd.train_guess --params %s --json %s" % (
            args.params, args.json)
    else:
        if not args.out:
            raise SystemExit("--out (where to write the trained parameters) or --params is required")
        params, res = train(args, nx, ny, nz)
    res["eval"] = {}
    modes = ("plain", "learned", "extrapolate")
    for s in seeds(args.eval_seeds):
        for prec, name in ((0, "fp64"), (1, "mixed")):
            ev = learned.evaluate(params, s, args.eval_steps, nx=nx, ny=ny, nz=nz, precision=prec,
                                  modes=modes)
            res["eval"]["%d_%s" % (s, name)] = ev
            print("seed %d %s: Picard %d / %d / %d (plain / learned / extrapolated), "
                  "wall/day %.3f / %.3f / %.3f s, max |dh| %.2e / %.2e" % (
                      s, name, *(ev[m]["picard_total"] for m in modes),
                      *(ev[m]["wall_s_per_simulated_day"] for m in modes),
                      ev["max_abs_h_diff_m"], ev["max_abs_h_diff_m_extrapolate"]), flush=True)
    if args.json:
        with open(args.json, "w") as f:
            json.dump(res, f, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "eval"}))


if __name__ == "__main__":
    main()
