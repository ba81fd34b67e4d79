"""Build the HIP library in-tree with hipcc for gfx950.

lsp_api.hip (the C ABI) and one spec_<name>.hip per spline type are compiled
in parallel into objects under a temporary folder, then linked into
lib/liblsp.so.
"""

import glob
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "lib", "liblsp.so")
CSRC = os.path.join(PKG, "csrc")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    "--offload-arch=gfx950",
    # no packed FP32 instructions (some of their forms are unreliable on the target)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # hardware float atomics for the given-order adjoint scatter-add
    "-munsafe-fp-atomics",
    "-ffp-contract=fast",
]


def sources():
    return [os.path.join(CSRC, "lsp_api.hip")] + sorted(glob.glob(os.path.join(CSRC, "spec_*.hip")))


def build_library(verbose=False, jobs=None):
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include")]
    tmpdir = tempfile.mkdtemp(prefix="lsp_build_")
    try:
        def compile_one(src):
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            cmd = [hipcc, *HIPCC_FLAGS, *inc, "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.run(cmd, check=True)
            return obj

        srcs = sources()
        jobs = jobs or min(len(srcs), max(1, min(os.cpu_count() or 1, 16)))
        with ThreadPoolExecutor(max_workers=jobs) as pool:
            objs = list(pool.map(compile_one, srcs))
        tmp = LIB + ".tmp"
        cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
