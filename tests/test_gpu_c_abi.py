"""The library driven from plain C (tests/c_abi/fdtd_abi_check.c, built by
__graft_entry__.build() with gcc against include/fdtd.h and the HIP
runtime's C API): fundamental ADI conserves its energy invariant and equals
conventional ADI, through the C ABI alone."""
import json
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "fdtd_abi_check")


def test_plain_c_program():
    if not os.path.exists(BIN):
        pytest.fail(f"{BIN} not built (run __graft_entry__.build())")
    print("[case] plain-C ABI program, 24x20x22 FP64 ADI", flush=True)
    res = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    print(res.stdout, res.stderr, flush=True)
    assert res.returncode == 0, res.stderr
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["energy_drift"] < 1e-12 and out["fundamental_vs_conventional"] < 1e-12


def test_sanitized_exercise_program():
    """Every entry point and its error paths from plain C, through the library
    built with its host code under AddressSanitizer and UndefinedBehaviorSanitizer
    (tests/c_abi/fdtd_abi_exercise): no sanitizer report, leaks included, and
    every status code as documented."""
    from paper_2011_14043_amd import _build
    from .test_abi_cpu import sanitizer_env
    if not (os.path.exists(_build.EXERCISE_BIN) and os.path.exists(_build.SAN_LIB)):
        pytest.fail("sanitized build missing (run __graft_entry__.build())")
    print("[case] sanitized exercise program (host ASan/UBSan)", flush=True)
    res = subprocess.run([_build.EXERCISE_BIN], capture_output=True, text=True, timeout=300, env=sanitizer_env())
    print(res.stdout[-4000:], res.stderr[-8000:], flush=True)
    assert res.returncode == 0, res.stderr[-8000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    assert out["failures"] == 0 and out["checks"] > 500, out
