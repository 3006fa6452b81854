"""Build liblbm.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2503_07898_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
OBJ_DIR = os.path.join(HERE, "_build")

# (source, extra flags): the stepping and utility kernels are compiled once
# per lattice; the D3Q27 objects carry their symbols in namespace lbm::k27
SOURCES = [("api.cpp", []), ("builder.cpp", []), ("multires_builder.cpp", []), ("step_kernels.hip", []),
           ("util_kernels.hip", []), ("mlp_kernels.hip", []),
           ("step_kernels.hip", ["-DLBM_Q27"]), ("util_kernels.hip", ["-DLBM_Q27"])]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-ffp-contract=off",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
# packed FP32 instructions are kept out of every kernel
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(job) -> str:
    src, extra = job
    obj = os.path.join(OBJ_DIR, src + ("".join(f.replace("-D", ".") for f in extra)).lower() + ".o")
    cmd = [HIPCC, *COMMON, *DEVICE_ONLY, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of liblbm.so failed")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
