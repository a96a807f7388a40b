"""Builds the CPU emulation of the library (tests/simt): the HIP sources of
the 3-D solver and of the column ensemble compiled as host C++ on the SIMT
emulator, with AddressSanitizer and UndefinedBehaviorSanitizer, linked into
the case driver.  Test infrastructure only."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1809_10895_amd", "csrc")
EXE = os.path.join(HERE, "driver_simt")
SOURCES = ["rf_kernels.hip", "rf_host.cpp", "rf_noalloc.hip", "rf_ensemble.hip", "rf_ensemble_host.cpp"]


def build(sanitize=True):
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I", HERE, "-I",
             os.path.join(ROOT, "include"), "-DRF_ENS_RUN_ENABLED=1", "-Wno-unused-variable",
             "-Wno-unused-but-set-variable"]
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
