"""Build libfrmi.so (HIP kernels for gfx950 + C++ host setup) and libfrprobe.so (the
benchmark's HBM streaming probe) in the package directory.

Usage: python -m paper_2408_16509_amd.build  (or call build()).  Always recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfrmi.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are avoided (kept out of the generated code)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
]


def hipcc():
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


PROBE_LIB = os.path.join(HERE, "libfrprobe.so")


def _hipcc(srcs, out, verbose):
    tmp = out + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(HERE, "..", "include")] + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """libfrmi.so (the FR library) and libfrprobe.so (the benchmark's streaming probe)."""
    _hipcc([os.path.join(CSRC, "frmi.hip"), os.path.join(CSRC, "setup.cpp")], LIB, verbose)
    _hipcc([os.path.join(CSRC, "stream_probe.hip")], PROBE_LIB, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
