"""Case files of the CPU emulation driver (tests/simt/driver.cpp) and the
parsing of its output.  Test infrastructure only."""
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def _fmt(xs):
    return " ".join(repr(float(x)) for x in np.ravel(xs))


def solver_case(path, w, nsteps, dt, tol_picard=1e-6, tol_cg=1e-13, max_picard=100, max_cg=20000,
                precond=1, ebats=0, dt0=None, dt_max=3600.0, precision=0, stencil=2, tile_rows=0,
                cols_per_wave=0, use_static=0, cg_rel_tol=0.0, zline_refactor=0):
    lines = ["%d %d %d %r %r %r" % (w.nx, w.ny, w.nz, w.dx, w.dy, w.dz)]
    lines.append("1 " + _fmt(w.ktop) if w.ktop is not None else "0")
    g = w.grad_elev if w.grad_elev is not None else (0.0, 0.0, 1.0)
    lines.append(_fmt(g))
    soil = np.atleast_2d(w.soil)
    lines.append("%d %d %s" % (w.model, soil.shape[0], _fmt(soil)))
    lines.append("1 " + _fmt(w.layer) if w.layer is not None else "0")
    lines.append("1 " + _fmt(w.lnks) if w.lnks is not None else "0")
    lines.append("%d %s" % (len(w.bcs), " ".join("%d %d %r" % (f, k, float(v)) for f, k, v in w.bcs)))
    lines.append("%r %r %d %d %d %d %r %r %d %d %d %d %r %d" % (
        tol_picard, tol_cg, max_picard, max_cg, precond, ebats, dt0 if dt0 else dt, dt_max, precision,
        stencil, tile_rows, cols_per_wave, cg_rel_tol, zline_refactor))
    lines.append("%d %r" % (nsteps, dt))
    lines.append(_fmt(w.h0))
    lines.append("%d" % use_static)
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def ens_case(path, w, t_ends, tol_picard=1e-6, max_picard=50, chord_eps=1e-9, dt_min=1e-6,
             inc_after=10, few_iters=3, max_iters=8, factor=1.3, precision=0, picard_variant=0,
             model=0, max_steps=10 ** 8, max_seconds=1e6, waves_per_block=4, blocks_per_cu=0,
             run_steps=()):
    bc = {4: (0, 0.0), 5: (0, 0.0)}
    for face, kind, value in w.bcs:
        bc[face] = (kind, value)
    lines = ["%d %r %d" % (w.ncol, w.dz, model), _fmt(w.lengths), _fmt(w.soil)]
    lines.append("%d %r %d %r" % (bc[4][0], float(bc[4][1]), bc[5][0], float(bc[5][1])))
    lines.append("%r %d %r %r %r %r %d %d %d %d %r %d %d" % (
        tol_picard, max_picard, chord_eps, w.dt, w.dt_max, dt_min, int(w.ebats), inc_after, few_iters,
        max_iters, factor, precision, picard_variant))
    lines.append("%d %r" % (max_steps, max_seconds))
    lines.append("%d %d" % (waves_per_block, blocks_per_cu))
    lines.append("%d %s" % (len(t_ends), _fmt(t_ends)))
    lines.append("%d %s" % (len(run_steps), _fmt(run_steps)))   # per-run step budgets
    lines.append(_fmt(w.h0))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def run(exe, mode, path, timeout=900, fill=0):
    """Runs the driver on a case file; `fill` is the byte the driver writes
    into every device buffer before the library sees it."""
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", SIMT_FILL=str(fill))
    r = subprocess.run([exe, mode, path], capture_output=True, text=True, timeout=timeout, env=env)
    if r.returncode != 0:
        raise RuntimeError("driver exited with %d:\n%s\n%s" % (r.returncode, r.stdout[-3000:],
                                                               r.stderr[-6000:]))
    out = {"steps": [], "runs": [], "cols": []}
    for line in r.stdout.splitlines():
        tok = line.split()
        if not tok:
            continue
        if tok[0] == "step":
            out["steps"].append({"status": int(tok[1]), "picard_iters": int(tok[2]),
                                 "cg_iters_total": int(tok[3]), "delta": [float(x) for x in tok[4:]]})
        elif tok[0] == "runstats":
            out["runstats"] = dict(zip(("status", "accepted", "rejected", "picard_total", "cg_total", "t"),
                                       [int(tok[1]), int(tok[2]), int(tok[3]), int(tok[4]), int(tok[5]),
                                        float(tok[6])]))
        elif tok[0] == "mass":
            out["mass"] = {"storage": float(tok[1]), "storage0": float(tok[2]), "error": float(tok[3])}
        elif tok[0] == "run":
            out["runs"].append({"status": int(tok[1]), "accepted": int(tok[2]), "rejected": int(tok[3]),
                                "picard_total": int(tok[4]), "cell_steps": int(tok[5]),
                                "failed": int(tok[6]), "t_min": float(tok[7]),
                                "max_balance_error": float(tok[8])})
        elif tok[0] == "col":
            v = tok[2:]
            out["cols"].append({"status": int(v[0]), "accepted": int(v[1]), "rejected": int(v[2]),
                                "easy": int(v[3]), "picard_total": int(v[4]), "t": float(v[5]),
                                "dt_next": float(v[6]), "storage0": float(v[7]), "storage": float(v[8]),
                                "inflow_top": float(v[9]), "inflow_bottom": float(v[10])})
        elif tok[0] == "h":
            out["h"] = np.array([float(x) for x in tok[1:]])
        elif tok[0] == "error":
            raise RuntimeError(line)
    return out
