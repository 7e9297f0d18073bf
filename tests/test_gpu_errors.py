"""Error paths that need a plan on the device: non-finite fields are reported
after stepping (FDTD_ENONFINITE), and the plan stays usable afterwards."""
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
