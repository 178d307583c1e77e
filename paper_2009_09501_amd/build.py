"""Build step of the HIP library: hipcc for gfx950 into libpstereo.so (in-tree).

Each source compiles to an object in parallel, then one link step.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD_DIR = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(HERE, "libpstereo.so")
SOURCES = ["kernels_depth.hip", "kernels_render.hip", "kernels_batch.hip", "pstereo_api.hip",
           "pstereo_batch_api.hip", "pstereo_server.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMPILE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
                 # no packed-FP32 instructions anywhere in the device code
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                 "-Wall", "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def sources():
    return [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build_library(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link ``libpstereo.so``."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    jobs = []
    for s in sources():
        obj = os.path.join(BUILD_DIR, os.path.splitext(s)[0] + ".o")
        jobs.append((obj, [HIPCC, *COMPILE_FLAGS, "-c", os.path.join(CSRC, s), "-o", obj]))

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(max_workers=min(len(jobs), 8)) as ex:
        list(ex.map(run, [c for _, c in jobs]))
    tmp = LIB_PATH + ".tmp"
    run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in jobs])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build_library(verbose=True))
