"""Builds libslf.so (HIP, gfx950) in-tree: paper_1812_06856_amd/_build/libslf.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "libslf.so")
SOURCES = ["slf_api.hip", "slf_kernels.hip", "slf_pool.hip", "slf_fusion.hip", "slf_slic.hip"]
# the fusion's FP64 projection and the segmentation's FP32 distances are fixed
# sequences of correctly rounded operations
EXTRA_FLAGS = {"slf_fusion.hip": ["-ffp-contract=off"], "slf_slic.hip": ["-ffp-contract=off"]}
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def build(verbose: bool = False, jobs: int = 4) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        cmd = [hipcc, *HIPCC_FLAGS, *EXTRA_FLAGS.get(src, []), "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-x", "hip", "-c",
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for pr in procs:
        if pr.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # the VALU issue-rate probe (bench.py --issue-rates), a separate executable
    probe = os.path.join(OUT_DIR, "issue_rates")
    cmd = [hipcc, *HIPCC_FLAGS, "-x", "hip", os.path.join(CSRC, "issue_rates.hip"), "-o", probe + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(probe + ".tmp", probe)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
