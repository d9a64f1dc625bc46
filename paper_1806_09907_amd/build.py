"""Build the airhip HIP library (libairhip.so) for gfx950 with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libairhip.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 arithmetic is disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]
# the roctx ranges of the entry points and stages
LINK_FLAGS = ["-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


LIB_DEBUG = os.path.join(HERE, "libairhip_debug.so")


def _compile(out: str, extra, verbose: bool) -> subprocess.Popen:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(HERE, "..", "include"), "-o",
           out + ".tmp", *sources(), *LINK_FLAGS]
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.Popen(cmd)


def build(verbose: bool = False, debug: bool = True) -> str:
    """Build libairhip.so and, with `debug`, the bounds-checked
    libairhip_debug.so (-DAIR_DEBUG_BOUNDS) beside it, in parallel."""
    jobs = [(LIB, _compile(LIB, [], verbose))]
    if debug:
        jobs.append((LIB_DEBUG, _compile(LIB_DEBUG, ["-DAIR_DEBUG_BOUNDS"], verbose)))
    for out, proc in jobs:
        if proc.wait() != 0:
            raise subprocess.CalledProcessError(proc.returncode, f"hipcc -> {out}")
    for out, _ in jobs:
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
