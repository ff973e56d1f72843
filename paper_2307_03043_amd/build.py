"""Build libchamfer.so for gfx950 with hipcc (in-tree).

Every source is compiled to an object in parallel (no device code crosses
files: kernels call only device functions of their own file or of the
headers), then the objects are linked into the shared library.
"""

import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libchamfer.so")

SOURCES = ["api.hip", "hash.hip", "sample.hip", "nnmin.hip", "nnmin_lowp.hip", "nnmin_split.hip",
           "serve.hip", "retrieve.hip", "reduce.hip"]

# -ffp-contract=off: no implicit fused multiply-adds (the canonical float32
# operations are spelled out, fmaf where an fma is meant).  Packed FP32
# instructions are disabled.  Denormals are kept (IEEE, like the host).
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 1)), 16)
    with tempfile.TemporaryDirectory(prefix="chamfer_build_") as tmpdir:
        def compile_one(src):
            obj = os.path.join(tmpdir, os.path.splitext(src)[0] + ".o")
            cmd = [hipcc, *FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            return obj

        with ThreadPoolExecutor(max_workers=jobs) as pool:
            objs = list(pool.map(compile_one, SOURCES))
        tmp = SO + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
