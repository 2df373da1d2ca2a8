"""Build libpond.so (the HIP kernels and the C ABI) in-tree for gfx950.

    python -m paper_1806_05089_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libpond.so")
SOURCES = ["pond_api.hip", "pond_forward.hip", "pond_step.hip", "pond_adjoint.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions stay off: ordinary scalar code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


# Checking build: the same library with every LDS window filled with NaN
# before it is staged (a kernel that read a window value it had not staged
# would return NaN there); the tests compare it with libpond.so.
POISON_LIB = os.path.join(PKG, "libpond_ldspoison.so")


def build(verbose: bool = False, extra_flags=(), out: str = LIB) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *extra_flags, "-I", INCLUDE, "-I", CSRC, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_poison(verbose: bool = False) -> str:
    return build(verbose, ("-DPOND_LDS_POISON",), POISON_LIB)


if __name__ == "__main__":
    build(verbose=True)
    build_poison(verbose=True)
    sys.exit(0)
