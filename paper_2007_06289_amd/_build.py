"""Builds libfhtfbp.so (HIP for gfx950) in-tree, next to this file.

    python -m paper_2007_06289_amd._build

Sources are compiled in parallel into ``_build/`` and linked into ``libfhtfbp.so``.  Every HIP
source is compiled with packed-FP32 instruction selection disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfhtfbp.so")

HIP_SOURCES = ["fht_pass_l4.hip", "fht_pass_l8.hip", "fht_pass_l16.hip", "fht_pass_l32.hip",
               "fht_pass_l64.hip", "fht_cols.hip", "coef_grad.hip", "conv_net.hip", "direct_fbp.hip", "resample.hip",
               "fhtfbp_api.hip"]
CPP_SOURCES = ["fit_iir.cpp"]
HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]
# Per-source additions.  The network's matrix-core results go straight to vector registers
# (by default the compiler puts them in accumulation registers and copies each one out
# before the bias, conversion and store: 8 extra vector instructions per pair of 16-pixel
# groups in the first layer alone).
EXTRA_FLAGS = {"conv_net.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libfhtfbp)")


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hipcc = _hipcc()
    jobs = []
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append([hipcc, *HIP_FLAGS, *EXTRA_FLAGS.get(src, []), "-I", INCLUDE, "-c",
                     os.path.join(CSRC, src), "-o", obj])
    for src in CPP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append(["g++", "-O2", "-fPIC", "-std=c++17", "-I", INCLUDE, "-c",
                     os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr)
    objs = [os.path.join(BUILD, s + ".o") for s in HIP_SOURCES + CPP_SOURCES]
    tmp = LIB + ".tmp"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
