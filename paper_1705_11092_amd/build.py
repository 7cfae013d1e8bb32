"""Build the HIP library libclbm.so for gfx950, in-tree.

Usage: ``python -m paper_1705_11092_amd.build`` (or ``build()`` from Python).
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libclbm.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # Contract a*b+c into FMA only inside one source expression, so the same
    # node arithmetic inlined into different kernels rounds the same way.
    "-ffp-contract=on",
    # Keep the compiler from emitting packed FP32 arithmetic.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
]


def sources():
    """Every translation unit: the C-ABI layer, the helper kernels and one
    unit of step kernels per storage type."""
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _filter(text: str):
    # hipcc's host pass does not know the packed-fp32 feature and says so.
    return [ln for ln in text.splitlines()
            if "packed-fp32-ops" not in ln and "is not a recognized feature" not in ln
            and ln.strip() and not ln.startswith("1 warning")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    lines = _filter(res.stdout + res.stderr)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(lines))
    if verbose and lines:
        print("\n".join(lines), flush=True)


def build(extra_flags=None, out=LIB, verbose=False, jobs=None) -> str:
    """Compile every HIP source (in parallel, one object each) and link them
    into one shared library; always rebuilds."""
    objdir = os.path.join(os.path.dirname(out), "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = jobs or min(len(sources()), os.cpu_count() or 4)
    objs, cmds = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src)[:-4] + ".o")
        objs.append(obj)
        cmds.append([HIPCC, *FLAGS, *(extra_flags or []), *inc, "-c", "-o", obj, src])
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as pool:
        for f in [pool.submit(_run, c, verbose) for c in cmds]:
            f.result()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out + ".tmp", *objs], verbose)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
