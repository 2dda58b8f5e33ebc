"""Build the HIP library libmcaad.so for gfx950 (in-tree, next to this file).

hipcc cross-compiles without a GPU.  Packed FP32 instructions are disabled
(-packed-fp32-ops): the kernels use scalar FP32/FP64 VALU arithmetic only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIBDIR, "libmcaad.so")

SOURCES = ["mc_kernels.hip", "lv_kernels.hip", "slv_kernels.hip", "bse_kernels.hip", "capi.hip", "mlp.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def flags(extra=()):
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-Wall", *extra]


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    objs, procs = [], []
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    for src in SOURCES:   # one hipcc per source, all at once
        obj = os.path.join(LIBDIR, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *flags(extra), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [src for src, p in procs if p.wait() != 0]
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(failed))
    tmp = LIB + ".tmp"
    subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, resource_usage="--usage" in sys.argv))
