"""Builds the CPU emulation of the library (tests/simt): the HIP sources of
the 3-D solver and of the column ensemble compiled as host C++ on the SIMT
emulator, with AddressSanitizer and UndefinedBehaviorSanitizer and, where the
host has them, fused multiply-adds contracted as on the GPU, linked into the
case driver.  Test infrastructure only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1809_10895_amd", "csrc")
EXE = os.path.join(HERE, "driver_simt")
SOURCES = ["rf_kernels.hip", "rf_host.cpp", "rf_noalloc.hip", "rf_ensemble.hip", "rf_ensemble_host.cpp"]


def host_has_fma():
    try:
        with open("/proc/cpuinfo") as f:
            return any(line.startswith("flags") and " fma " in line + " " for line in f)
    except OSError:
        return False


def build(sanitize=True, fma=None):
    """fma: contract a*b + c into fused multiply-adds, as the device compiler
    does for the GPU (default: when the host CPU has FMA instructions)."""
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I", HERE, "-I",
             os.path.join(ROOT, "include"), "-DRF_ENS_RUN_ENABLED=1", "-Wno-unused-variable",
             "-Wno-unused-but-set-variable"]
    if fma if fma is not None else host_has_fma():
        flags += ["-O2", "-mfma", "-ffp-contract=fast"]   # g++ contracts from -O2 on
    if sanitize:
        flags += ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    srcs = [os.path.join(CSRC, f) for f in SOURCES]
    cmd = (["g++"] + flags + ["-x", "c++"] + srcs + ["-x", "none", os.path.join(HERE, "simt.cpp"),
                                                     os.path.join(HERE, "driver.cpp"), "-o", EXE + ".tmp"])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("emulation build failed:\n" + r.stderr[-6000:])
    os.replace(EXE + ".tmp", EXE)
    return EXE


if __name__ == "__main__":
    print(build())
