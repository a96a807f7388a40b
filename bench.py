#!/usr/bin/env python3
"""Benchmark of the Richards-equation hot path on one MI355X.

One step = one backward-Euler time step with its whole Picard loop (soil
coefficients, assembly, PCG solve, Picard exit test, step acceptance) of the
watershed workload: 512 x 512 x 64 cells of 2 x 2 x 0.2 m under a fractal
surface (12.46 M active cells), three soil layers (Eq. 5) with a lognormal Ks
field, hourly seeded rain, adaptive steps (EBATS) from 60 s up to 3600 s,
FP64; inputs resident in HBM.  Prints ONE JSON line with the throughput in
cell-steps/s, the roofline of the dominant kernel (HIP events on the library
stream, inside the timed region; also against device copies measured on the
same box, outside it) and the CPU oracle timed on a bounded sample (the
serial method and the multi-core slab mode).

    python bench.py [--gpus 1] [--steps 40] [--warmup 5] [--workload watershed]
                    [--precision fp64|mixed]

The timed steps are the run's steps warmup+1 .. warmup+steps, taken from the
initial state by the library's own adaptive time loop (rf_run_steps).  The
one-time costs of a process (code objects, the first long queue of work) are
paid on a separate context before.  The same steps are then timed in the
other precision ("other_precision"), and a whole simulated day is timed with
the paper's loop, mixed precision and the extrapolated first iterate
("ebats_day").
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_TFLOPS = 78.6

# Algorithmic bytes per active cell and launch (one pass over each array;
# neighbour values are reuse, not extra traffic).  Kernel -> (jacobi, zline).
ALGO_BYTES = {
    "fp64": {
        # read r, diag (z), p_old, K, Dd, e; write p, q, e (the last update's
        # e += alpha p rides on the spmv kernel, which reads p_old anyway)
        "spmv": (72, 64),
        "update": (32, 48),    # read r, q, diag (Jacobi) / r, q, rdp, tz (z-line); write r (+ z)
        "coeff": (56, 56),     # read h^m, h^n, theta^n, Ks; write K, Dd, bst
        # read K, h^m, Dd, bst; write r, diag (Jacobi) / r, tz, rdp, z (z-line,
        # diag rebuilt later from the factors)
        "resid": (48, 64),
        "apply_h": (32, 32),   # read e, p (the last alpha p), h^m; write h^m
        "accept": (24, 24),    # read h^m; write h^n, theta^n
    },
    # PCG vectors and the operator / preconditioner copies in FP32
    "mixed": {
        "spmv": (36, 32),      # as above, 4 B each
        "update": (16, 24),    # read r, q, diag / r, q, rdp, tz; write r (+ z), 4 B each
        "coeff": (56, 56),     # FP64 as above
        "resid": (48, 56),     # read K, h^m, Dd, bst (8 B); write r, diag / r, tz, rdp, z, and K, Dd (4 B)
        "apply_h": (24, 24),   # read e, p (4 B), h^m; write h^m
        "accept": (24, 24),
    },
}
PRECISION = {"fp64": 0, "mixed": 1}
STENCIL = {"columns": 0, "tiles": 1, "auto": 2}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="watershed", choices=["watershed", "hillslope", "column100"])
    ap.add_argument("--precond", default="zline", choices=["zline", "jacobi"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="arithmetic of the timed line (fp64 = the paper's)")
    ap.add_argument("--cg-rel-tol", type=float, default=0.0,
                    help="relative PCG exit test (0 = absolute tol_cg only)")
    ap.add_argument("--no-extras", action="store_true",
                    help="time the headline line only (no other precision, adaptive-step day or "
                         "learned guess): profiler runs")
    ap.add_argument("--learned-steps", type=int, default=24,
                    help="steps of the learned-guess comparison (0 = skip)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="budget of the CPU-oracle sample in slab mode on all threads (0 = skip)")
    ap.add_argument("--cpu-serial-steps", type=int, default=1,
                    help="steps of the one-thread CPU-oracle sample (0 = skip)")
    ap.add_argument("--no-timing", action="store_true", help="no per-kernel HIP events")
    ap.add_argument("--ebats-days", type=float, default=1.0,
                    help="simulated days of the adaptive-step extra (0: skip)")
    ap.add_argument("--timing-every", type=int, default=4,
                    help="time the dominant kernel in every N-th step of the timed region")
    ap.add_argument("--driver", choices=("run", "step"), default="run",
                    help="timed steps through rf_run (default) or one rf_step call per step")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="copy this many MiB with torch before the steps (reference kernel of "
                         "known traffic for hardware-counter runs)")
    ap.add_argument("--stencil", default="auto", choices=["auto", "tiles", "columns"],
                    help="how the stencil kernels reach lateral neighbours (LDS tiles or "
                         "per-wave neighbour columns)")
    ap.add_argument("--tile-rows", type=int, default=0, choices=[0, 2, 4],
                    help="columns of a stencil tile along y (0 = chosen by the library)")
    ap.add_argument("--cols-per-wave", type=int, default=0,
                    help="launch shape of the PCG kernels (0 = chosen from the grid size)")
    return ap.parse_args()


def make_workload(name):
    from paper_1809_10895_amd import workloads as W
    if name == "watershed":
        w = W.watershed()
        desc = ("watershed 512x512x64 cells of 2x2x0.2 m, fractal (Hurst 0.8) surface mask, three "
                "Eq.-5 layers with lognormal Ks (ln-sigma 1), hourly seeded rain (10% wet, "
                "exponential depths of mean 2 mm), EBATS dt 60 s -> 3600 s, FP64 PCG tol 1e-8 m")
    elif name == "hillslope":
        w = W.hillslope()
        desc = "hillslope 128x128x64, 1x1x0.1 m cells, lognormal Ks (ln-sigma 1), rain 1e-7 m/s, dt 600 s"
    else:
        w = W.column100()
        desc = "1-D column 1x1x100, dz 1 cm, top Dirichlet -0.75 m, dt 10 s"
    return w, desc


def host_info():
    """CPU model, sockets and cores of this host (lscpu), and os.cpu_count()."""
    import subprocess
    info = {"os_cpu_count": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(w, seconds, serial_steps):
    """The oracle as it stands on the first steps of the same workload from its
    initial state (each of the workload's first step size, dt0 = EBATS's
    first step): as many steps as fit in `seconds` in the slab mode (block-
    Jacobi DIC over one sub-domain of whole y-rows per thread, the 'simple'
    decomposition of Sec. 2.3) on every OpenMP thread, and `serial_steps`
    steps of the serial method (natural-order DIC-PCG, one thread)."""
    import oracle
    from paper_1809_10895_amd import workloads as W

    def run(nslab, budget, nmax):
        P = oracle.Problem(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, ktop=w.ktop, grad_elev=w.grad_elev)
        W.configure(w, P)
        P.set_options(tol_picard=1e-6, tol_cg=1e-8, max_picard=50, ebats=0, dt0=w.dt)
        P.set_slabs(nslab)
        P.set_state(w.h0)
        t0 = time.perf_counter()
        n = 0
        while n < nmax:
            s, _ = P.step(w.dt)
            if s != 0:
                break
            n += 1
            if time.perf_counter() - t0 >= budget:
                break
        return n, time.perf_counter() - t0

    nthr = oracle.threads()
    out = {"unit": "cell-steps/s", "kind": "oracle", "host": host_info()}
    if seconds > 0:
        nslab = max(1, min(nthr, w.ny))
        n, el = run(nslab, seconds, 10 ** 9)
        out.update({"value": w.active_cells * n / el, "cores": nthr,
                    "sample": "%d backward-Euler steps of %g s of the same workload from its initial "
                              "state, DIC-PCG with block-Jacobi DIC over %d slabs of whole y-rows "
                              "(the 'simple' decomposition), %d OpenMP threads (%.1f s)"
                              % (n, w.dt, nslab, nthr, el)})
    if serial_steps > 0:
        n, el = run(1, 0.0, serial_steps)
        one = {"value": w.active_cells * n / el, "cores": 1,
               "sample": "%d backward-Euler step(s) of %g s from the initial state, DIC-PCG in "
                         "natural order, one thread (%.1f s)" % (n, w.dt, el)}
        if "value" in out:
            out["one_thread"] = one
        else:
            out.update(one)
    return out if "value" in out else None


def host_stream_copy(threads, mib=512, reps=5):
    """Host memory bandwidth: a copy of `mib` MiB between two NumPy arrays in
    `threads` slices on as many threads (NumPy releases the GIL in copyto),
    best of `reps`; bytes counted as read + write."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor
    n = mib * (1 << 20) // 8
    src = np.ones(n)
    dst = np.zeros(n)
    edges = [n * i // threads for i in range(threads + 1)]

    def part(i):
        np.copyto(dst[edges[i]:edges[i + 1]], src[edges[i]:edges[i + 1]])

    best = float("inf")
    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(part, range(threads)))                     # first touch
        for _ in range(reps):
            t0 = time.perf_counter()
            list(ex.map(part, range(threads)))
            best = min(best, time.perf_counter() - t0)
    return 2.0 * n * 8 / best / 1e9


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("rf_kernels.hip", "rf_internal.h"):
        with open(os.path.join(ROOT, "paper_1809_10895_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, kernel, precision):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    tag = "" if precision == "fp64" else "_" + precision
    path = os.path.join(ROOT, "profiles", "pmc_%s_%s%s.json" % (kernel, workload, tag))
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_hash():
        return None
    return d.get("bytes_per_launch")


def timed_case(args, w, precision):
    """`args.warmup` untimed steps, then `args.steps` timed steps of `w` from its
    initial state in the given precision, through the library's time loop
    (rf_run_steps: EBATS when the workload adapts its steps, else fixed dt).
    Returns the measured figures and the final state (host copy)."""
    import torch
    from paper_1809_10895_amd import Solver, workloads as W
    pc = 1 if args.precond == "zline" else 0
    h0 = torch.tensor(w.h0, dtype=torch.float64, device="cuda:0")
    far = 1e12          # the runs stop on their step counts

    def solver():
        S = Solver(0)
        S.setup_grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.ktop, w.grad_elev)
        W.configure(w, S)
        S.set_options(tol_picard=1e-6, tol_cg=1e-8, max_picard=50, precond=pc, dt0=w.dt,
                      dt_max=w.dt_max, ebats=int(w.ebats), cols_per_wave=args.cols_per_wave,
                      precision=PRECISION[precision], cg_rel_tol=args.cg_rel_tol,
                      stencil=STENCIL[args.stencil], tile_rows=args.tile_rows)
        S.bind()
        assert S.set_state(h0) == 0, S.last_error()
        return S

    algo_bytes = ALGO_BYTES[precision]
    # One-time costs of the process, on a context of its own: the first step
    # (code objects loaded, scratch set up at a kernel's first launch), then
    # steps 2-5 with every kernel timed (the per-kernel table, which names the
    # dominant kernel), then 48 steps through the time loop, whose first long
    # queue of enqueued-ahead work the HIP runtime sets up once per process
    # (a few ms in all).
    S = solver()
    s, st = S.step(w.dt)
    assert s == 0, S.last_error()
    S.set_timing(True)
    for _ in range(4):
        s, st = S.step(w.dt)
        assert s == 0, S.last_error()
    tm_all = S.get_timing()
    S.set_timing(False)
    s, rs = S.run(far, max_steps=48)
    assert s == 0 and rs["accepted"] == 48, S.last_error()
    tot_all = sum(v["ms"] for v in tm_all.values() if isinstance(v, dict))
    kern = max((k for k in algo_bytes if k in tm_all and tm_all[k]["launches"]),
               key=lambda k: tm_all[k]["ms"], default=None)
    del S
    # the measured context: from the initial state, warmup steps, then the
    # timed ones, all through the same adaptive time loop
    S = solver()
    if args.warmup > 0:
        s, rs = S.run(far, max_steps=args.warmup)
        assert s == 0 and rs["accepted"] == args.warmup, S.last_error()
    t_start = S.get_state()[1]
    # timed region: HIP events time the dominant kernel's launches in every
    # timing_every-th step (a timed launch costs some overhead of its own)
    timed = [kern] if (kern and not args.no_timing) else False
    S.set_timing(timed)
    S.select_timing(timed, every=max(1, args.timing_every))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if args.driver == "run":
        s, rs = S.run(far, max_steps=args.steps)
        if s != 0 or rs["accepted"] != args.steps:
            raise SystemExit("run failed: %s %s" % (rs, S.last_error()))
        picard, cg, rejected = rs["picard_total"], rs["cg_total"], rs["rejected"]
    else:
        # one rf_step call per step, with the step sizes of the time loop
        # (fixed-step workloads only)
        if w.ebats:
            raise SystemExit("--driver step needs a fixed-step workload")
        picard = cg = rejected = 0
        for i in range(args.steps):
            s, st = S.step(w.dt)
            if s != 0:
                raise SystemExit("step failed: " + S.last_error())
            picard += st["picard_iters"]
            cg += st["cg_iters_total"]
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    t_stop = S.get_state()[1]
    tm = S.get_timing()
    cells = w.active_cells

    roof = None
    if kern is not None and not args.no_timing and tm[kern]["launches"]:
        avg_s = tm[kern]["ms"] / tm[kern]["launches"] * 1e-3
        algo = algo_bytes[kern][pc] * cells
        achieved = algo / avg_s / 1e9
        traffic = measured_traffic(args.workload, kern, precision)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": kern, "avg_us": round(avg_s * 1e6, 2),
                "timed_launches": tm[kern]["launches"],
                "timed_steps": "every %d%s step of the timed region" % (
                    args.timing_every, {1: "st", 2: "nd", 3: "rd"}.get(args.timing_every, "th"))
                if args.timing_every > 1 else "every step of the timed region",
                "algorithmic_bytes_per_launch": algo}
    # per-kernel breakdown from the warm-up steps (all kernels timed there),
    # with each kernel's algorithmic rate against the same peak
    kernels = {}
    for k, v in tm_all.items():
        if not isinstance(v, dict):
            continue
        avg = v["ms"] / v["launches"] * 1e-3 if v["launches"] else None
        e = {"launches": v["launches"], "avg_us": round(avg * 1e6, 2) if avg else None,
             "share": round(v["ms"] / tot_all, 3) if tot_all > 0 else None,
             "idle_launches": v["idle_launches"]}
        if avg and k in algo_bytes:
            gbs = algo_bytes[k][pc] * cells / avg / 1e9
            e.update({"algorithmic_GBps": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                      "traffic": measured_traffic(args.workload, k, precision)})
        kernels[k] = e
    h = S.get_state()[0].cpu().numpy()
    return {"value": cells * args.steps / el, "ms_per_step": el / args.steps * 1e3,
            "picard_per_step": picard / args.steps, "cg_per_picard": cg / max(picard, 1),
            "rejected_steps": rejected, "simulated_s": [t_start, t_stop],
            "mean_dt_s": (t_stop - t_start) / args.steps,
            "wall_s_per_simulated_day": el / (t_stop - t_start) * 86400.0,
            "roofline": roof, "kernels_warmup": kernels}, h


def ebats_day(args, w, days, dt0):
    """Wall time per simulated day with adaptive steps (EBATS, Sec. 2.2: dt
    from dt0 up to dt_max, x1.3 after ten easy steps, /1.3 and rerun above
    eight Picard iterations) from the workload's initial state: the paper's
    loop in FP64 and in mixed precision, and the extrapolated first iterate
    with mixed precision; the largest head difference from the FP64 run."""
    import numpy as np
    import torch
    from paper_1809_10895_amd import Solver, workloads as W
    pc = 1 if args.precond == "zline" else 0
    h0 = torch.tensor(w.h0, dtype=torch.float64, device="cuda:0")
    out = {"days": days, "dt0_s": dt0, "dt_max_s": w.dt_max}
    finals = {}
    m = w.active_mask()
    for name, prec, fi in (("plain_fp64", 0, 0), ("plain_mixed", 1, 0), ("extrapolate_mixed", 1, 1)):
        S = Solver(0)
        S.setup_grid(w.nx, w.ny, w.nz, w.dx, w.dy, w.dz, w.ktop, w.grad_elev)
        W.configure(w, S)
        S.set_options(tol_picard=1e-6, tol_cg=1e-8, max_picard=50, precond=pc, dt0=dt0,
                      dt_max=w.dt_max, ebats=1, precision=prec, first_iterate=fi,
                      cols_per_wave=args.cols_per_wave, stencil=STENCIL[args.stencil],
                      tile_rows=args.tile_rows)
        S.bind()
        assert S.set_state(h0) == 0, S.last_error()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s, rs = S.run(days * 86400.0)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"status": s, "wall_s_per_simulated_day": el / days,
                     "accepted": rs["accepted"], "rejected": rs["rejected"],
                     "picard_total": rs["picard_total"], "cg_total": rs["cg_total"],
                     "dt_last_s": rs["dt_last"]}
        finals[name] = S.get_state()[0].cpu().numpy()
        del S
    out["max_abs_h_diff_m"] = {k: float(np.abs(v[m] - finals["plain_fp64"][m]).max())
                               for k, v in finals.items() if k != "plain_fp64"}
    base = out["plain_fp64"]["wall_s_per_simulated_day"]
    out["speedup_vs_plain_fp64"] = {k: base / out[k]["wall_s_per_simulated_day"]
                                    for k in ("plain_mixed", "extrapolate_mixed")}
    return out


def copy_reference(nbytes, reps=20):
    """Same-box reference rate: a device-to-device copy (the runtime's copy
    kernel) of nbytes, read + write counted, GB/s."""
    import torch
    n = max(int(nbytes) // 16, 1)                     # nbytes moved = read n*8 + write n*8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 16.0 * n * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    return round(gbs, 1)


def add_copy_reference(roof):
    """The roofline against copies measured on the same box: one moving the
    dominant kernel's algorithmic bytes per launch (MALL-resident when the
    working set is) and one of 1 GiB (from HBM)."""
    if roof is None:
        return
    same = copy_reference(roof["algorithmic_bytes_per_launch"])
    big = copy_reference(1 << 30)
    roof["copy_reference_GBps"] = {"same_bytes": same, "1GiB": big}
    roof["frac_of_copy"] = {"same_bytes": round(roof["achieved"] / same, 4),
                            "1GiB": round(roof["achieved"] / big, 4)}


def learned_guess(nsteps):
    """The committed network (trained on seeds 100-119) on held-out seed 200
    of the hillslope with its rain series: plain Picard in FP64 against the
    learned first iterate with mixed precision, same Picard tolerance."""
    import numpy as np
    from paper_1809_10895_amd import learned
    path = os.path.join(ROOT, "paper_1809_10895_amd", "data", "guess_hillslope.f32")
    params = np.fromfile(path, dtype=np.float32)
    modes = ("plain", "learned", "extrapolate")
    fp64 = learned.evaluate(params, 200, nsteps, precision=0, modes=modes)
    mixed = learned.evaluate(params, 200, nsteps, precision=1, modes=modes)
    base = fp64["plain"]["wall_s_per_simulated_day"]
    return {"workload": "hillslope 128x128x64 seed 200 with its rain series, dt 600 s, %d steps" % nsteps,
            "wall_s_per_simulated_day": {
                "plain_fp64": base,
                "learned_fp64": fp64["learned"]["wall_s_per_simulated_day"],
                "extrapolate_fp64": fp64["extrapolate"]["wall_s_per_simulated_day"],
                "plain_mixed": mixed["plain"]["wall_s_per_simulated_day"],
                "learned_mixed": mixed["learned"]["wall_s_per_simulated_day"],
                "extrapolate_mixed": mixed["extrapolate"]["wall_s_per_simulated_day"]},
            "picard_total": {m: fp64[m]["picard_total"] for m in modes},
            "predict_ms_per_step": mixed["learned"]["predict_s"] / nsteps * 1e3,
            "learned_mixed_vs_plain_fp64": base / mixed["learned"]["wall_s_per_simulated_day"],
            "extrapolate_mixed_vs_plain_fp64": base / mixed["extrapolate"]["wall_s_per_simulated_day"],
            "max_abs_h_diff_m": max(fp64["max_abs_h_diff_m"], mixed["max_abs_h_diff_m"],
                                    fp64["max_abs_h_diff_m_extrapolate"],
                                    mixed["max_abs_h_diff_m_extrapolate"]),
            # the paper's adaptive steps (EBATS) over a simulated day
            "ebats_day": learned.evaluate_ebats(params, 200, days=1.0)}


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w, desc = make_workload(args.workload)
    cells = w.active_cells
    progress("%s %s" % (args.workload, args.precision))
    main_r, h_main = timed_case(args, w, args.precision)
    variant = learned_res = ebats_res = None
    if not args.no_extras:
        other = "mixed" if args.precision == "fp64" else "fp64"
        progress("%s %s" % (args.workload, other))
        r, h_other = timed_case(args, w, other)
        m = w.active_mask()
        variant = {"precision": other, "value": r["value"], "ms_per_step": r["ms_per_step"],
                   "picard_per_step": r["picard_per_step"], "cg_per_picard": r["cg_per_picard"],
                   "max_abs_h_diff_m": float(np.abs(h_other[m] - h_main[m]).max()),
                   "roofline": r["roofline"]}

    if not args.no_extras and args.ebats_days > 0:
        progress("EBATS day")
        # adaptive steps from the workload's own first step
        ebats_res = ebats_day(args, w, args.ebats_days, w.dt)
    if not args.no_extras and args.learned_steps > 0:
        progress("learned guess")
        learned_res = learned_guess(args.learned_steps)
    add_copy_reference(main_r["roofline"])
    progress("cpu baseline")
    cpu = cpu_baseline(w, args.cpu_seconds, args.cpu_serial_steps)
    if cpu is not None and cpu.get("cores", 1) > 1:
        # the host's own bandwidth, and what share of it the oracle's rate
        # would be if it moved the GPU path's algorithmic bytes per cell-step
        pc = 1 if args.precond == "zline" else 0
        ab = ALGO_BYTES[args.precision]
        pic, cgp = main_r["picard_per_step"], main_r["cg_per_picard"]
        per_cell_step = (pic * cgp * (ab["spmv"][pc] + ab["update"][pc])
                         + pic * (ab["coeff"][pc] + ab["resid"][pc] + ab["apply_h"][pc])
                         + ab["accept"][pc])
        bw = host_stream_copy(cpu["cores"])
        cpu["host_stream_copy_GBps"] = round(bw, 1)
        cpu["gpu_path_bytes_per_cell_step"] = round(per_cell_step, 1)
        cpu["stream_fraction"] = round(cpu["value"] * per_cell_step / 1e9 / bw, 4)
    out = {
        "metric": "cell-steps/s at Picard tol 1e-6", "value": main_r["value"], "unit": "cell-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "active_cells": cells, "grid": [w.nx, w.ny, w.nz],
                   "dt0_s": w.dt, "dt_max_s": w.dt_max if w.ebats else w.dt,
                   "ebats": bool(w.ebats), "tol_picard_m": 1e-6, "tol_cg_m": 1e-8,
                   "cg_rel_tol": args.cg_rel_tol, "precision": args.precision,
                   "precond": args.precond, "stencil": args.stencil, "tile_rows": args.tile_rows,
                   "cols_per_wave": args.cols_per_wave,
                   "driver": "rf_run_steps" if args.driver == "run" else "rf_step per step",
                   "picard_per_step": main_r["picard_per_step"],
                   "cg_per_picard": main_r["cg_per_picard"],
                   "rejected_steps": main_r["rejected_steps"],
                   "simulated_s": main_r["simulated_s"], "mean_dt_s": main_r["mean_dt_s"],
                   "wall_s_per_simulated_day": main_r["wall_s_per_simulated_day"]},
        "roofline": main_r["roofline"],
        "kernels_warmup": main_r["kernels_warmup"],
        "other_precision": variant,
        "ebats_day": ebats_res,
        "learned_guess": learned_res,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
