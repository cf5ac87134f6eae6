"""Build libtchol.so in-tree with hipcc for gfx950.

    python -m paper_1402_6601_amd.build

hipcc cross-compiles without a GPU, so this runs on any machine with ROCm.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtchol.so")
ARCH = os.environ.get("TCHOL_OFFLOAD_ARCH", "gfx950")

SOURCES = ["tchol_device.hip", "tchol_refine.hip", "tchol_batched32.hip", "tchol_api.cpp",
           "plan.cpp", "tchol_noalloc.hip"]

# Packed FP32 instructions are disabled for all device code.  Matrix-core
# accumulators are allocated in ordinary vector registers: with the default
# (accumulation registers) the compiler copies every loop-carried
# accumulator between the two register files on each K chunk.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-mllvm", "-amdgpu-mfma-vgpr-form"]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cand = os.path.join(rocm, "bin", "hipcc")
    return cand if os.path.exists(cand) else "hipcc"


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall", "-fvisibility=hidden",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] + DEVICE_FLAGS
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    cmd += ["-o", tmp]
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out.strip():
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
