"""Build the HIP library (gfx950) in-tree: paper_2106_13281_amd/libbraxmi.so."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbraxmi.so")
SOURCES = ["bx_api.cpp", "bx_parse.cpp", "bx_kernels.hip", "bx_vjp.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed-FP32 instructions (v_pk_*_f32) anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-fno-math-errno",
    # FP32 divide and sqrt without the correctly-rounded sequences (about
    # 2.5 ulp); the parity budget against the FP64 checker is 1e-4
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    # FP32 denormals flushed to zero (no range scaling around reciprocals)
    "-fgpu-flush-denormals-to-zero",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def build(verbose=False):
    tmp = LIB + f".tmp{os.getpid()}"
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [HIPCC, *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print("built", LIB)
