"""Build the HIP C-ABI libraries for gfx950 with hipcc, in-tree:
liblbm.so (the phase-field LBM step, include/lbm.h), libsurr.so (the
learned surrogate's kernels, include/surrogate.h), libdrops.so (the
drop-size diagnostic, include/drops.h) and libprobe.so (the HBM bandwidth
probe of the measurements, include/probe.h)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "liblbm.so")
SURR_LIB = os.path.join(LIBDIR, "libsurr.so")
DROPS_LIB = os.path.join(LIBDIR, "libdrops.so")
PROBE_LIB = os.path.join(LIBDIR, "libprobe.so")
TARGETS = [(LIB, ["lbm.hip"]), (SURR_LIB, ["nn.hip"]), (DROPS_LIB, ["ccl.hip"]), (PROBE_LIB, ["probe.hip"])]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # keep hipcc from forming packed FP32 instructions on its own
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def _compile(out: str, sources, verbose: bool):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *[os.path.join(CSRC, s) for s in sources], "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    return subprocess.Popen(cmd), out


def build(verbose: bool = False) -> str:
    """Compile the libraries (in parallel); returns the LBM library path."""
    os.makedirs(LIBDIR, exist_ok=True)
    procs = [_compile(out, srcs, verbose) for out, srcs in TARGETS]
    failed = [out for p, out in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, f"hipcc ({', '.join(failed)})")
    for _, out in procs:
        os.replace(out + ".tmp", out)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
