"""Build libchamfer.so for gfx950 with hipcc (in-tree)."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libchamfer.so")

SOURCES = ["api.hip", "hash.hip", "sample.hip", "nnmin.hip", "nnmin_mfma.hip", "nnmin_lowp.hip", "serve.hip",
           "retrieve.hip", "reduce.hip"]

# -ffp-contract=off: no implicit fused multiply-adds (the canonical float32
# operations are spelled out, fmaf where an fma is meant).  Packed FP32
# instructions are disabled.  Denormals are kept (IEEE, like the host).
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = SO + ".tmp"
    cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
