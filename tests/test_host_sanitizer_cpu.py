"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's translation units are compiled host-only (no device code, so
nothing can be launched) with ASan + UBSan, linked into a separate shared
library, and the host-side ABI tests (plan matching for every shipped spline,
Voronoi plans, argument validation, dims and dtype checks, workspace sizes
and schedule bookkeeping) run against it in a subprocess with the sanitizer
runtime preloaded.  Any report aborts that subprocess.
"""

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2102_08514_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "hostsan")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
COMPILE = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "--cuda-host-only",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def _build():
    os.makedirs(OUT, exist_ok=True)
    srcs = [os.path.join(CSRC, "lsp_api.hip")] + sorted(glob.glob(os.path.join(CSRC, "spec_*.hip")))

    def one(src):
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        subprocess.run([HIPCC, *COMPILE, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj],
                       check=True, capture_output=True)
        return obj

    with ThreadPoolExecutor(max_workers=8) as pool:
        objs = list(pool.map(one, srcs))
    # Host-only objects still reference their translation unit's device
    # binary, which the HIP module constructor registers.  Define each as a
    # clang offload bundle with only an empty host entry: no device code.
    names = set()
    for obj in objs:
        nm = subprocess.run(["nm", "-u", obj], check=True, capture_output=True, text=True).stdout
        names.update(ln.split()[-1] for ln in nm.splitlines() if ln.split()[-1].startswith("__hip_fatbin_"))
    triple = b"host-x86_64-unknown-linux-gnu-"
    bundle = (b"__CLANG_OFFLOAD_BUNDLE__" + (1).to_bytes(8, "little") +
              (32 + 24 + len(triple)).to_bytes(8, "little") + (0).to_bytes(8, "little") +
              len(triple).to_bytes(8, "little") + triple)
    body = ", ".join(str(b) for b in bundle)
    stub = os.path.join(OUT, "fatbin_stubs.c")
    with open(stub, "w") as fh:
        for n in sorted(names):
            fh.write(f"const unsigned char {n}[{len(bundle)}] __attribute__((aligned(4096))) = {{{body}}};\n")
    subprocess.run(["gcc", "-c", "-fPIC", stub, "-o", stub + ".o"], check=True, capture_output=True)
    objs.append(stub + ".o")
    lib = os.path.join(OUT, "liblsp_hostsan.so")
    link = [CLANGXX, "-shared", "-shared-libsan", "-fsanitize=address,undefined", *objs,
            "-L/opt/rocm/lib", "-lamdhip64", "-o", lib]
    subprocess.run(link, check=True, capture_output=True)
    return lib


@pytest.mark.skipif(not os.path.exists(HIPCC) or _runtime() is None, reason="hipcc or the ASan runtime missing")
def test_abi_host_code_is_sanitizer_clean():
    lib = _build()
    env = dict(os.environ)
    env.update({
        "LSP_LIBRARY": lib,
        "LD_PRELOAD": _runtime(),
        # Python itself is not instrumented and keeps objects alive at exit
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    })
    # the ctypes-level ABI tests (the ones that need torch tensors are left to the plain run)
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", os.path.join(ROOT, "tests", "test_abi_cpu.py"),
           "-k", "not api_argument_validation and not no_fallback and not host_tensors"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
