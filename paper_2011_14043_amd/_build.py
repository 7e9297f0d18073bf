"""Build step: compile the HIP sources of the library for gfx950 (hipcc).

csrc/fdtd.hip (the C ABI, host code and the small kernels) and the parts of
csrc/kern_inst.hip (the line-pass kernel instantiations, -DFDTD_PART=n) are
compiled to objects in parallel and linked into libfdtd.so.

Debug configuration: csrc/fdtd.hip is compiled a second time with its host
code under AddressSanitizer and UndefinedBehaviorSanitizer (device code as in
the product build) and linked with the same kernel objects into
libfdtd_san.so, which only the test program tests/c_abi/fdtd_abi_exercise
loads; that program is built with the same sanitizers and carries their
runtime."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "fdtd.hip")
KERN_SRC = os.path.join(HERE, "csrc", "kern_inst.hip")
KERN_PARTS = 17   # kern_inst.hip: FDTD_PART = 0 .. 16
LIB = os.path.join(HERE, "libfdtd.so")
OBJ_DIR = os.path.join(HERE, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # no packed FP32 arithmetic: some of its forms have given silently wrong results on gfx950
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


# host code only: each sanitizer option goes to the host compilation
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-g"]
SAN_LIB = os.path.join(HERE, "libfdtd_san.so")

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


EXERCISE_SRC = os.path.join(ROOT, "tests", "c_abi", "fdtd_abi_exercise.c")
EXERCISE_BIN = os.path.join(ROOT, "tests", "c_abi", "fdtd_abi_exercise")
# the C program of the debug configuration (clang, the sanitizers' runtime linked in)
EXERCISE_SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def exercise_cmds(out: str) -> list[list[str]]:
    """clang commands that build tests/c_abi/fdtd_abi_exercise.c against the
    host-sanitized library (compile as C11 with warnings as errors, link with
    the C++ driver so that the sanitizers' C++ runtime parts come along)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    llvm = os.path.join(rocm, "llvm", "bin")
    obj = out + ".o"
    return [[os.path.join(llvm, "clang"), "-std=c11", "-O1", "-g", *EXERCISE_SANITIZE, "-Wall", "-Wextra", "-Werror",
             "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(rocm, "include"), "-I" + os.path.join(ROOT, "include"),
             "-c", EXERCISE_SRC, "-o", obj],
            [os.path.join(llvm, "clang++"), *EXERCISE_SANITIZE, obj, "-o", out, "-L" + HERE, "-lfdtd_san",
             "-L" + os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
             "-Wl,-rpath,$ORIGIN/../../paper_2011_14043_amd", "-Wl,-rpath," + os.path.join(rocm, "lib")]]


def _jobs() -> int:
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(16, n if n > 0 else (os.cpu_count() or 4)))


def build(verbose: bool = False, extra_flags: list[str] | None = None) -> str:
    """Compile libfdtd.so in-tree, then the plain-C check program that links
    it; returns the library's path.  Raises on failure."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    flags = HIPCC_FLAGS + list(extra_flags or [])
    jobs = [(SRC, os.path.join(OBJ_DIR, "fdtd.o"), [])]
    for part in range(KERN_PARTS):
        jobs.append((KERN_SRC, os.path.join(OBJ_DIR, f"kern_{part}.o"), [f"-DFDTD_PART={part}"]))

    san_obj = os.path.join(OBJ_DIR, "fdtd_san.o")

    def compile_one(job):
        src, obj, defs = job
        cmd = [hipcc, *flags, *defs, "-c", "-o", obj, src]
        res = subprocess.run(cmd, capture_output=True, text=True)
        return cmd, res

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(compile_one, jobs + [(SRC, san_obj, HOST_SANITIZE)]))
    for cmd, res in results:
        if res.returncode != 0:
            raise RuntimeError("hipcc failed: " + " ".join(cmd) + "\n" + res.stdout + res.stderr)
        if verbose:
            print(" ".join(cmd))
    tmp = LIB + ".tmp"
    cmd = [hipcc, *flags, "-shared", "-o", tmp, *[j[1] for j in jobs]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, LIB)
    tmp = SAN_LIB + ".tmp"
    cmd = [hipcc, *flags, "-shared", "-o", tmp, san_obj, *[j[1] for j in jobs[1:]]]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc link (sanitized host) failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, SAN_LIB)
    for cmd in [c_check_cmd(C_CHECK_BIN), *exercise_cmds(EXERCISE_BIN)]:
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(os.path.basename(cmd[0]) + " failed:\n" + res.stdout + res.stderr)
        if verbose:
            print(" ".join(cmd))
    if os.path.exists(EXERCISE_BIN + ".o"):
        os.remove(EXERCISE_BIN + ".o")
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
