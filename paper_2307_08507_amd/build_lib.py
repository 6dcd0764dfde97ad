"""Build libmdot.so (HIP, gfx950) in-tree with hipcc.

Every HIP source is compiled with `-Xclang -target-feature -Xclang -packed-fp32-ops`
so the compiler does not form packed FP32 instructions; the hot loops are written with
scalar FP32/FP64 arithmetic.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libmdot.so")
SOURCES = ["mdot_kernels.hip", "mdot_api.cpp"]
ARCH = os.environ.get("MDOT_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", f"-I{os.path.join(ROOT, 'include')}", "-Wall",
              "-Wno-unused-function"]
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OUT_DIR, src + ".o")
        cmd = [hipcc(), *common, "-c", path, "-o", obj]
        if src.endswith(".hip"):
            # kernel arguments (a few pointers and ints) are preloaded into SGPRs at dispatch, so a
            # kernel's first dependent load does not wait for a kernarg-segment fetch
            cmd += [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-munsafe-fp-atomics", "-mllvm", "-amdgpu-kernarg-preload-count=16"]
        else:
            pass
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
