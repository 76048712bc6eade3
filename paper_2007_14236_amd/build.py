"""Build libsnn.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2007_14236_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsnn.so")
SOURCES = ["kernels_build.hip", "kernels_step.hip", "kernels_rec.hip", "kernels_stdp.hip", "snn_api.cpp", "snn_server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("SNN_OFFLOAD_ARCH", "gfx950")

DEVICE_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
    # every float operation rounds as written unless an fma is spelled out
    "-ffp-contract=off",
    # no packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src: str, obj: str) -> None:
    cmd = [HIPCC] + DEVICE_FLAGS + ["-c", src, "-o", obj]
    if src.endswith(".hip"):
        cmd[1:1] = ["-x", "hip"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    for line in (r.stdout + r.stderr).splitlines():
        if "warning" in line and "packed-fp32-ops" not in line and "target-feature" not in line:
            sys.stderr.write(line + "\n")


def build(verbose: bool = True) -> str:
    """Compile every source and link libsnn.so (always rebuilds)."""
    t0 = time.time()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = []
    for s in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(s)[0] + ".o")
        _compile(os.path.join(CSRC, s), obj)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s")
    return LIB


if __name__ == "__main__":
    build()
