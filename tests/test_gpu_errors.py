"""Paths that need a plan on the device: non-finite fields are reported after
stepping (FDTD_ENONFINITE) and the plan stays usable afterwards; sampled
per-launch timing."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_nonfinite_fields_reported(dtype):
    from paper_2011_14043_amd import FdtdError, Plan
    nx, ny, nz, h = 8, 9, 10, 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    u0 = W.random_fields(nx, ny, nz, seed=1)
    E = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[:3]]
    H = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[3:]]
    E[2][4, 4, 4] = float("nan")             # a dynamic Ez sample
    plan = Plan(nx, ny, nz, dt, h, h, h, dtype=dtype)
    with pytest.raises(FdtdError, match="ENONFINITE"):
        plan.run(E, H, 2, energy_every=1)
    # the plan keeps working on finite input
    E = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[:3]]
    H = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[3:]]
    tr = plan.run(E, H, 2, energy_every=1)
    plan.close()
    assert np.all(np.isfinite(tr))


@pytest.mark.parametrize("every,steps", [(1, 5), (4, 9), (8, 3)])
def test_sampled_launch_timing(every, steps):
    """fdtd_set_timing(p, k) brackets the line passes of main-iteration steps
    0, k, 2k, ...: ADI has 4 y/z and 2 x passes per step; a timed run does not
    change the fields; k < 0 is rejected."""
    from paper_2011_14043_amd import FdtdError, Plan
    nx, ny, nz, h = 20, 18, 16, 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    u0 = W.random_fields(nx, ny, nz, seed=2)
    fields = lambda: ([torch.tensor(a, dtype=torch.float32, device=DEV) for a in u0[:3]],
                      [torch.tensor(a, dtype=torch.float32, device=DEV) for a in u0[3:]])
    plan = Plan(nx, ny, nz, dt, h, h, h)
    E0, H0 = fields()
    plan.run(E0, H0, steps)
    plan.set_timing(every)
    E, H = fields()
    plan.run(E, H, steps)
    tm = plan.last_timing()
    timed = len(range(0, steps, every))
    assert tm["yz_launches"] == 4 * timed and tm["x_launches"] == 2 * timed
    assert tm["yz_ms_avg"] > 0 and tm["x_ms_avg"] > 0 and tm["main_ms"] > 0
    for a, b in zip(E + H, E0 + H0):
        assert torch.equal(a, b)
    plan.set_timing(0)
    plan.run(E, H, 1)
    assert plan.last_timing()["yz_launches"] == 0
    with pytest.raises(FdtdError):
        plan.set_timing(-1)
    plan.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_diff_norm_matches_host_sum(dtype):
    """fdtd_diff_norm against the energy-weighted sums formed on the host from
    the same values (eps of the owning cell, in-extent samples only)."""
    import numpy as np
    import torch
    import oracle
    import workloads as W
    from paper_2011_14043_amd import Plan
    nx, ny, nz, h = 37, 21, 30, 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    tdt = torch.float64 if dtype == "f64" else torch.float32
    eps = W.random_box_eps(nx, ny, nz, seed=90, nboxes=6)
    a, b = W.random_fields(nx, ny, nz, seed=91), W.random_fields(nx, ny, nz, seed=92)
    plan = Plan(nx, ny, nz, dt, h, h, h, dtype=tdt, eps_r=torch.tensor(eps))
    dev = [torch.tensor(x, dtype=tdt, device="cuda") for x in a + b]
    num, den = plan.diff_norm(dev[0:3], dev[3:6], dev[6:9], dev[9:12])
    plan.close()
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    av = [x.double().cpu().numpy() for x in dev[0:6]]
    bv = [x.double().cpu().numpy() for x in dev[6:12]]
    ref_num = oracle.energy([x - y for x, y in zip(av, bv)], g)
    ref_den = oracle.energy(bv, g)
    assert abs(num / ref_num - 1) < 1e-12 and abs(den / ref_den - 1) < 1e-12
    p2 = Plan(nx, ny, nz, dt, h, h, h, dtype=tdt)
    same = p2.diff_norm(dev[0:3], dev[3:6], dev[0:3], dev[3:6])
    p2.close()
    assert same[0] == 0.0 and same[1] > 0.0
