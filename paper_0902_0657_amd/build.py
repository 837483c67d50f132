"""Builds liblpdec.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_0902_0657_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblpdec.so")
ARCH = os.environ.get("LPDEC_ARCH", "gfx950")

SOURCES = ["lpdec_inst_f64_lds.hip", "lpdec_inst_f64_glb.hip", "lpdec_inst_f32_lds.hip",
           "lpdec_inst_f32_glb.hip", "lpdec_kernels.hip", "lpdec_api.cpp"]
HEADERS = ["lpdec_common.hpp", "lpdec_device.hpp", "lpdec_launch.hpp", "lpdec_kernels.hpp"]

# Packed FP32 instructions are disabled for every HIP translation unit; the host pass of
# hipcc prints a harmless warning about the unknown feature.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compiles every source (in parallel, one hipcc per file) and links liblpdec.so."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    jobs = jobs or min(len(SOURCES), max(1, min(16, os.cpu_count() or 1)))

    def compile_one(src):
        obj = os.path.join(CSRC, src + ".o")
        cmd = [hipcc, *FLAGS, "-I", os.path.join(HERE, "..", "include"), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, r

    objs = []
    with ThreadPoolExecutor(jobs) as ex:
        for src, obj, r in ex.map(compile_one, SOURCES):
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of liblpdec.so failed")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
