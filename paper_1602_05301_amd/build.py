"""Build the gfx950 shared library ``libqbxfmm.so`` in-tree.

Host planning (C++17) is compiled with g++, the kernels and the device part
of the C ABI with hipcc for gfx950, and everything is linked by hipcc.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libqbxfmm.so")
BUILD = os.path.join(HERE, "_build")

HOST_SRC = ["planner.cpp", "abi_plan.cpp"]
HIP_SRC = ["kernels.hip", "areaquery.hip", "krylov.hip", "abi_device.cpp"]

ARCH = os.environ.get("QBX_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions stay disabled for every HIP translation unit.
# No automatic FMA contraction: the kernels write their fused multiply-adds
# explicitly, so a result does not depend on how a template instance (the
# number of densities per launch, say) happens to be scheduled.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=off", "-Wno-unused-result"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
              "-I/opt/rocm/include"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    jobs = []
    for s in HOST_SRC:
        o = os.path.join(BUILD, s + ".o")
        jobs.append(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    for s in HIP_SRC:
        o = os.path.join(BUILD, s + ".o")
        jobs.append([HIPCC, *HIP_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    procs = [(cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
             for cmd in jobs]
    failed = []
    for cmd, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            failed.append((cmd, out + err))
        elif verbose and (out or err):
            sys.stderr.write(out + err)
    if failed:
        for cmd, msg in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + msg + "\n")
        raise RuntimeError("compilation failed")
    tmp = OUT + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lm"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
