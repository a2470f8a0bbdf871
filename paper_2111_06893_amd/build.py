"""Builds libdgtn.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdgtn.so")
SOURCES = ["host.cpp", "kernels.hip", "fields.hip", "capi.hip", "solver.hip", "mg.hip", "adjoint.hip", "residual.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=fast",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    raise RuntimeError("hipcc not found")


# Host code built with AddressSanitizer and UndefinedBehaviorSanitizer (device
# code unchanged): for checking the host-side calls (mesh, geometry, hierarchy
# and smoother planning) on the CPU.  Load the result with the ASan runtime
# preloaded.
SANITIZE_FLAGS = [
    "-O1", "-g",
    "-Xarch_host", "-fsanitize=address",
    "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer",
]


def build(verbose: bool = False, sanitize: bool = False, out: str | None = None) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    target = out or LIB
    tmp = target + ".tmp"
    flags = [f for f in HIPCC_FLAGS if not (sanitize and f == "-O3")] + (SANITIZE_FLAGS if sanitize else [])
    cmd = [hipcc(), *flags, "-I", os.path.join(HERE, "..", "include"), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose and r.stderr:
        sys.stderr.write(r.stderr)
    os.replace(tmp, target)
    return target


if __name__ == "__main__":
    print(build(verbose=True))
