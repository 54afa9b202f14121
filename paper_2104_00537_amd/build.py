"""Builds libsph.so (the gfx950 HIP kernels and the C ABI of include/sph.h)
in-tree with hipcc.  Run ``python -m paper_2104_00537_amd.build``."""
from __future__ import annotations

import glob
import hashlib
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libsph.so")
ARCH = os.environ.get("SPH_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
]
# No packed FP32 instructions (v_pk_*_f32) anywhere in the device code.  The
# feature exists only for the GPU target, so it goes to the device pass
# alone: each source is compiled twice, the device code to a code-object
# bundle and the host code with that bundle embedded, both under one
# compilation-unit id so that the host side's registrations of kernels and
# __device__ variables name the device side's symbols.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links them."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    tag = f".{os.getpid()}"

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    def compile_one(src):
        base = os.path.join(objdir, os.path.basename(src) + tag)
        cuid = "sph_" + hashlib.sha1(os.path.basename(src).encode()).hexdigest()[:16]
        common = [hipcc, *HIPCC_FLAGS, f"-cuid={cuid}", *inc, "-c", src]
        run([*common, "--offload-device-only", *DEVICE_FLAGS, "-o", base + ".hipfb"])
        run([*common, "--offload-host-only", "-Xclang", "-fcuda-include-gpubinary",
             "-Xclang", base + ".hipfb", "-o", base + ".o"])
        os.remove(base + ".hipfb")
        return base + ".o"

    jobs = max(1, min(len(sources()), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, sources()))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    for o in objs:
        os.remove(o)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
