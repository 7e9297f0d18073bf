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
