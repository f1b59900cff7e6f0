"""Builds libqcw.so (HIP, gfx950) in-tree with hipcc.

Every HIP source under csrc/ is compiled for gfx950 into one shared library
next to this file; the request server's load generator (loadgen/) is built
beside it against that library.  Packed FP32 instruction selection is disabled for all
device code.  Usage: python -m paper_1101_1785_amd.build
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libqcw.so")
OBJ_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "lib")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core results in ordinary VGPRs: keeps the batch kernel at 4 waves/SIMD
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    # no wave-level combining of atomics: the channel kernels' ticket draws
    # (one lane) are used a tile later, and the combining waits for them at once
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
    f"-I{INCLUDE}", f"-I{CSRC}",
    # the run-time compiler (hipRTC) of the ROCm installation that builds the library
    f'-DQCW_ROCM_LIB="{ROCM_LIB}"',
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def _compile(src: str) -> str:
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}")
    if out.strip():
        sys.stderr.write(out + "\n")
    return obj


def build(jobs: int = 8) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           "-ldl", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_loadgen()
    return LIB


LOADGEN_SRC = os.path.join(HERE, "loadgen", "serve_load.cpp")
LOADGEN = os.path.join(HERE, "serve_load")


def build_loadgen() -> str:
    """The open-loop load generator for the request server (host code only,
    linked against libqcw.so next to it)."""
    tmp = LOADGEN + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-Wall", f"-I{INCLUDE}", LOADGEN_SRC, "-o", tmp,
           f"-L{HERE}", "-lqcw", "-Wl,-rpath,$ORIGIN", "-lpthread"]
    subprocess.check_call(cmd)
    os.replace(tmp, LOADGEN)
    return LOADGEN


if __name__ == "__main__":
    print(build())
