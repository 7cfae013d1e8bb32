"""Build the HIP library libclbm.so for gfx950, in-tree.

Usage: ``python -m paper_1705_11092_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libclbm.so")
SOURCES = ["clbm_kernels.hip", "clbm_api.hip"]
HEADERS = ["clbm_device.h", "clbm_internal.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # Contract a*b+c into FMA only inside one source expression, so the same
    # node arithmetic inlined into different kernels rounds the same way.
    "-ffp-contract=on",
    # Keep the compiler from emitting packed FP32 arithmetic.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(extra_flags=None, out=LIB, verbose=False) -> str:
    """Compile every HIP source into one shared library; always rebuilds."""
    cmd = [HIPCC, *FLAGS, *(extra_flags or []), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", out + ".tmp", *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass does not know the packed-fp32 feature and says so.
    lines = [ln for ln in (res.stdout + res.stderr).splitlines()
             if "packed-fp32-ops" not in ln and "is not a recognized feature" not in ln
             and ln.strip() and not ln.startswith("1 warning")]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(lines))
    if verbose and lines:
        print("\n".join(lines))
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
