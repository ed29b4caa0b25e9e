"""Build libnbx.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_1510_04068_amd.build

The library lands next to this file as ``libnbx.so``; object files go to ``_build/``.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libnbx.so")
SOURCES = ["nbx_kernels.hip", "nbx_blockstep.hip", "nbx_runtime.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 (v_pk_*_f32) generation is switched off: every FP32 op is a plain VALU op.
FLAGS = [
    "-O3",
    "--offload-arch=gfx950",
    "-fPIC",
    "-std=c++17",
    "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-I", CSRC,
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(line for line in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in line)
    if res.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), out))
    if out.strip():
        print(out)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = [os.path.join(BUILD, src.replace(".hip", ".o")) for src in SOURCES]
    if verbose:
        print("hipcc", " ".join(SOURCES), flush=True)
    # the translation units compile independently: one hipcc per file, side by side
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        jobs = [pool.submit(_run, [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
                for src, obj in zip(SOURCES, objs)]
        for j in jobs:
            j.result()
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB, flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
