"""Writes the rocprofv3 summaries under profiles/ from the CSV output of
profiled bench.py runs (run on any machine, after the runs):

  stats: `rocprofv3 --kernel-trace --stats --output-format csv` of one run
         -> profiles/kernel_stats_<workload>[_mixed].md
  pmc:   two `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs with
         `bench.py --calibrate-copy-mib M` (a plain device copy of M MiB
         before the solver, whose counters give the KiB -> byte scales)
         -> profiles/pmc_<workload>[_mixed].md and one
            profiles/pmc_<kernel>_<workload>[_mixed].json per solver kernel,
            which bench.py reports as the kernel's measured HBM traffic while
            the kernel source hash in it matches the current source.

A dispatch "did work" when it is not one of the launches the step driver
enqueues past the end of a PCG solve or of the Picard loop, which return at
once: for durations, longer than 30 % of the kernel's 90th percentile and
4.5 us; for counters, at least 10 % of the kernel's largest FETCH_SIZE.
"""
import argparse
import csv
import glob
import hashlib
import json
import os
import re

ROOT = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("rf_kernels.hip", "rf_internal.h"):
        with open(os.path.join(ROOT, "paper_1809_10895_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short_name(name):
    """A kernel's name without return type and argument list."""
    name = name.strip().replace("(anonymous namespace)", "{anon}")
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def kernel_key(name):
    """bench.py's name of a solver kernel ('spmv' for rf::k_spmv<..> and
    rf::k_spmv_tile<..>), or None."""
    m = re.match(r"rf::k_([a-z_]+?)(_tile)?(<|$)", short_name(name))
    return m.group(1) if m else None


def find_csv(d, suffix):
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise SystemExit("no *%s under %s" % (suffix, d))
    return hits[-1]


def read_csv(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def title(workload, precision):
    return "%s workload, %s" % (workload, "FP64" if precision == "fp64" else "mixed precision")


def tag(precision):
    return "" if precision == "fp64" else "_" + precision


def stats(args):
    st = read_csv(find_csv(args.dir, "kernel_stats.csv"))
    tr = read_csv(find_csv(args.dir, "kernel_trace.csv"))
    out = ["# rocprofv3 kernel statistics -- " + title(args.workload, args.precision), "",
           "Command (from the repository root on the GPU box):", "", "```", args.command, "```", "",
           "Kernel source sha256[:16] of rf_kernels.hip + rf_internal.h: `%s`" % kernel_source_hash(),
           "", "## `kernel_stats.csv` (all dispatches, as written by rocprofv3)", "",
           "| kernel | calls | total us | average us | min us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for r in st:
        out.append("| %s | %s | %.1f | %.2f | %.2f | %.2f | %.2f |" % (
            short_name(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e3,
            float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    by = {}
    for r in tr:
        by.setdefault(short_name(r["Kernel_Name"]), []).append(
            (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out += ["", "## Dispatches that did work (from `kernel_trace.csv`)", "",
            "Launches the step driver enqueues past the end of a PCG solve or of the Picard loop "
            "return at once; a dispatch counts as working when it lasts longer than 30 % of the "
            "kernel's 90th-percentile duration and 4.5 us.", "",
            "| kernel | working dispatches | average us | median us | short dispatches |",
            "|---|---|---|---|---|"]
    for name, ds in by.items():
        ds = sorted(ds)
        p90 = ds[min(len(ds) - 1, int(0.9 * len(ds)))]
        work = [d for d in ds if d > max(0.3 * p90, 4.5)]
        avg = sum(work) / len(work) if work else 0.0
        med = work[len(work) // 2] if work else 0.0
        out.append("| %s | %d | %.2f | %.2f | %d |" % (name, len(work), avg, med,
                                                       len(ds) - len(work)))
    path = os.path.join(ROOT, "profiles", "kernel_stats_%s%s.md" % (args.workload, tag(args.precision)))
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")
    print(path)


def counters(d, counter):
    rows = read_csv(find_csv(d, "counter_collection.csv"))
    per = {}
    for r in rows:
        if r["Counter_Name"] != counter:
            continue
        key = (r["Dispatch_Id"], short_name(r["Kernel_Name"]))
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    out = {}
    for (did, name), v in per.items():
        out.setdefault(name, []).append((int(did), v))
    for v in out.values():
        v.sort()
    return out


def pmc(args):
    fetch = counters(args.fetch_dir, "FETCH_SIZE")
    write = counters(args.write_dir, "WRITE_SIZE")
    copy_kib = args.copy_mib * 1024.0
    copies_f = [v for _, v in fetch.get("__amd_rocclr_copyBuffer", [])]
    copies_w = [v for _, v in write.get("__amd_rocclr_copyBuffer", [])]
    if not copies_f or not copies_w:
        raise SystemExit("no copy kernel in the counter runs (bench.py --calibrate-copy-mib)")
    fscale = copy_kib / max(copies_f)
    wscale = copy_kib / max(copies_w)
    sha = kernel_source_hash()
    out = ["# rocprofv3 hardware counters -- " + title(args.workload, args.precision), "",
           "Two counter runs (one counter each) of:", "", "```", args.command_fetch,
           args.command_write, "```", "",
           "Calibration: the %d MiB device copy (`__amd_rocclr_copyBuffer`) reads FETCH_SIZE = "
           "%.0f KiB and WRITE_SIZE = %.0f KiB, so FETCH_SIZE is scaled by %.3f and WRITE_SIZE "
           "by %.3f to get bytes (KiB x 1024 x scale)." % (args.copy_mib, max(copies_f),
                                                        max(copies_w), fscale, wscale), "",
           "Kernel source sha256[:16]: `%s`" % sha, "",
           "A dispatch counts as working when its FETCH_SIZE is at least 10 % of the kernel's "
           "largest; the per-dispatch figures average the working dispatches.", "",
           "| kernel | dispatches (working) | HBM read MB / dispatch | HBM write MB / dispatch "
           "| total MB / dispatch |", "|---|---|---|---|---|"]
    groups = {}
    for name, fs in fetch.items():
        key = kernel_key(name)
        if key is None:
            continue
        ws = dict(write.get(name, []))
        big = max(v for _, v in fs)
        work = [(did, v) for did, v in fs if v >= 0.1 * big]
        # the two runs enqueue the same dispatches in the same order
        wvals = sorted(ws.values(), reverse=True)[:len(work)]
        rd = sum(v for _, v in work) / len(work) * 1024.0 * fscale
        wr = (sum(wvals) / len(wvals) if wvals else 0.0) * 1024.0 * wscale
        out.append("| %s | %d | %.1f | %.1f | %.1f |" % (name, len(work), rd / 1e6, wr / 1e6,
                                                       (rd + wr) / 1e6))
        g = groups.setdefault(key, [0.0, 0.0, 0])
        g[0] += rd * len(work)
        g[1] += wr * len(work)
        g[2] += len(work)
    md = "pmc_%s%s.md" % (args.workload, tag(args.precision))
    with open(os.path.join(ROOT, "profiles", md), "w") as f:
        f.write("\n".join(out) + "\n")
    print(os.path.join("profiles", md))
    for key, (rd, wr, n) in groups.items():
        rec = {"workload": args.workload, "precision": args.precision, "kernel": key,
               "kernel_source_sha": sha, "bytes_per_launch": (rd + wr) / n,
               "read_bytes": rd / n, "write_bytes": wr / n, "fetch_scale": fscale,
               "write_scale": wscale, "source": "profiles/" + md}
        path = os.path.join(ROOT, "profiles", "pmc_%s_%s%s.json" % (key, args.workload,
                                                                  tag(args.precision)))
        with open(path, "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    sub = ap.add_subparsers(dest="mode", required=True)
    for mode in ("stats", "pmc"):
        p = sub.add_parser(mode)
        p.add_argument("--workload", required=True)
        p.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    s = sub.choices["stats"]
    s.add_argument("--dir", required=True, help="rocprofv3 output folder of the run")
    s.add_argument("--command", required=True, help="the profiled command, as run")
    p = sub.choices["pmc"]
    p.add_argument("--fetch-dir", required=True)
    p.add_argument("--write-dir", required=True)
    p.add_argument("--copy-mib", type=int, default=1024)
    p.add_argument("--command-fetch", required=True)
    p.add_argument("--command-write", required=True)
    args = ap.parse_args()
    stats(args) if args.mode == "stats" else pmc(args)


if __name__ == "__main__":
    main()
