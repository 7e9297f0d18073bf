"""Build step: compile the HIP sources of the library for gfx950 (hipcc)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "fdtd.hip")
LIB = os.path.join(HERE, "libfdtd.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed FP32 arithmetic: some of its forms have given silently wrong results on gfx950
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


ROOT = os.path.dirname(HERE)
C_CHECK_SRC = os.path.join(ROOT, "tests", "c_abi", "fdtd_abi_check.c")
C_CHECK_BIN = os.path.join(ROOT, "tests", "c_abi", "fdtd_abi_check")


def c_check_cmd(out: str) -> list[str]:
    """gcc command that builds the plain-C program of tests/c_abi against the
    library and the HIP runtime's C API (C11, warnings as errors)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
            "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"), C_CHECK_SRC, "-o", out,
            "-L" + HERE, "-lfdtd", "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
            "-Wl,-rpath,$ORIGIN/../../paper_2011_14043_amd", "-Wl,-rpath," + os.path.join(rocm, "lib")]


def build(verbose: bool = False) -> str:
    """Compile libfdtd.so in-tree, then the plain-C check program that links
    it; returns the library's path.  Raises on failure."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-o", tmp, SRC]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, LIB)
    cmd = c_check_cmd(C_CHECK_BIN)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
