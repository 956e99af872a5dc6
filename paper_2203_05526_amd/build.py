"""Build the HIP library libhgf.so for gfx950 in-tree with hipcc.

Run ``python -m paper_2203_05526_amd.build`` (or call ``build()``).  Every
source is compiled to an object, then linked into one shared library next to
this file.  Packed FP32 vector instructions are disabled for device code.
"""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhgf.so")
ARCH = os.environ.get("HGF_OFFLOAD_ARCH", "gfx950")

SOURCES = ["hgf_kernels.hip", "hgf_full_tiled.hip", "hgf_tiled_c64.hip", "hgf_tiled_c128.hip", "hgf_tiled_r32.hip",
           "hgf_tiled_r64.hip", "hgf_scratch.hip", "hgf_stream.hip", "hgf_separated.hip", "hgf_api.cpp", "hgf_functions.cpp", "hgf_network.cpp",
           "hgf_step.cpp", "hgf_autotune.cpp", "hgf_readout.cpp", "hgf_grad.cpp", "hgf_separated_host.cpp",
           "hgf_tables.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", f"-I{CSRC}"]
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), "-c"] + COMMON
    if src.endswith(".hip"):
        cmd += DEVICE
    cmd += [os.path.join(CSRC, src), "-o", obj]
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
