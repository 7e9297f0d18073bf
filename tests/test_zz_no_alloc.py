"""fdtd_diff_norm_noalloc (the entry point that allocates nothing) against
fdtd_diff_norm: bit-for-bit equal results, through the C ABI, on two calls in
a row whose second one has the smaller grid (fewer first-stage partial sums
than the first call left in the shared static work area), in FP32 and FP64,
and a non-finite input reported the same way.  Collected last (test_zz_), so
that a failure here hides no other test."""
import ctypes

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _fields(nx, ny, nz, seed, dtype):
    u = W.random_fields(nx, ny, nz, seed=seed)
    return ([torch.tensor(a, dtype=dtype, device=DEV) for a in u[:3]],
            [torch.tensor(a, dtype=dtype, device=DEV) for a in u[3:]])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_noalloc_equals_diff_norm_large_then_small(dtype):
    from paper_2011_14043_amd import Plan
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    # the first grid uses all 1024 partial sums, the second 3 of them
    for (nx, ny, nz), seed in (((96, 80, 72), 1), ((8, 9, 7), 2)):
        print(f"[case] diff_norm_noalloc {nx}x{ny}x{nz} {dtype}", flush=True)
        eps = W.random_box_eps(nx, ny, nz, seed=seed, nboxes=8)
        plan = Plan(nx, ny, nz, dt, h, h, h, dtype=dtype, eps_r=torch.tensor(eps))
        Ea, Ha = _fields(nx, ny, nz, 10 + seed, dtype)
        Eb, Hb = _fields(nx, ny, nz, 20 + seed, dtype)
        got = plan.diff_norm_noalloc(Ea, Ha, Eb, Hb)
        want = plan.diff_norm(Ea, Ha, Eb, Hb)
        assert got == want, (got, want)
        # the same call again returns the same value (nothing left from the last call)
        assert plan.diff_norm_noalloc(Ea, Ha, Eb, Hb) == want
        assert np.isfinite(got[0]) and got[1] > 0
        plan.close()


def test_noalloc_reports_nonfinite_and_invalid():
    from paper_2011_14043_amd import FdtdError, Plan, _lib
    h = 1e-3
    dt = W.yee_dt(h, h, h, 2.0)
    plan = Plan(6, 7, 8, dt, h, h, h, dtype=torch.float32)
    Ea, Ha = _fields(6, 7, 8, 3, torch.float32)
    Eb, Hb = _fields(6, 7, 8, 4, torch.float32)
    Ea[1][2, 3, 4] = float("nan")
    with pytest.raises(FdtdError) as exc:
        plan.diff_norm_noalloc(Ea, Ha, Eb, Hb)
    assert exc.value.status == -5
    L = _lib.lib()
    out = (ctypes.c_double * 2)()
    assert L.fdtd_diff_norm_noalloc(None, None, None, None, None, out) == -1
    plan.close()
