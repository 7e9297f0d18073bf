"""The output path of fdtd_run.  Without an energy trace the last line passes
of a run store the output straight into the caller's arrays and a wall kernel
writes the samples no pass writes; with an energy trace the state takes the
output and a copy kernel moves it to the caller.  Both give the same fields bit
for bit, for every line-pass scheme and form, every precision, with a source,
from fields that are random everywhere (wall-tangential E and normal H on the
walls included, and the entries outside each component's extent, which
neither path writes)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PREC = {"f32": (torch.float32, torch.float32, None), "f32p": (torch.float32, torch.float32, False),
        "f64": (torch.float64, torch.float64, None), "f32s64": (torch.float32, torch.float64, None)}


@pytest.fixture(scope="module")
def case():
    nx, ny, nz = 23, 19, 27
    dx, dy, dz = 1.0e-3, 1.3e-3, 0.8e-3
    rng = np.random.default_rng(31)
    u0 = [rng.standard_normal((nz + 1, ny + 1, nx + 1)) for _ in range(6)]
    return dict(nx=nx, ny=ny, nz=nz, dx=dx, dy=dy, dz=dz, dt=W.yee_dt(dx, dy, dz, 6.0),
                eps=W.random_box_eps(nx, ny, nz, seed=32, nboxes=6), u0=u0)


def _plan(c, scheme, form, prec, mu=None):
    from paper_2011_14043_amd import Plan
    dtype, solve, refine = PREC[prec]
    return Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["dx"], c["dy"], c["dz"], scheme=scheme, form=form,
                dtype=dtype, solve_dtype=solve, eps_r=torch.tensor(c["eps"]), refine=refine,
                mu_r=None if mu is None else torch.tensor(mu))


def _fields(c, dtype):
    return ([torch.tensor(a, dtype=dtype, device=DEV) for a in c["u0"][:3]],
            [torch.tensor(a, dtype=dtype, device=DEV) for a in c["u0"][3:]])


@pytest.mark.parametrize("scheme,form", [("adi", "fundamental"), ("adi", "conventional"), ("lod1", "fundamental"),
                                         ("lod1", "conventional"), ("ss2", "fundamental"), ("ss2", "conventional"),
                                         ("lod2", "fundamental"), ("lod2", "conventional"),
                                         ("douglas_gunn", "fundamental")])
@pytest.mark.parametrize("prec", ["f32", "f32p", "f64", "f32s64"])
@pytest.mark.parametrize("steps", [1, 13])
def test_direct_output_equals_copied_output(case, scheme, form, prec, steps):
    from paper_2011_14043_amd import Source
    print(f"[case] output path {scheme}/{form} {prec} steps={steps}", flush=True)
    dtype = PREC[prec][0]
    dt = case["dt"]
    src = Source(11, 7, 13, f0=1 / (12 * dt), tau=3 * dt, t0=2 * dt, amp=1e10)
    plan = _plan(case, scheme, form, prec)
    Ed, Hd = _fields(case, dtype)
    Ec, Hc = _fields(case, dtype)
    plan.run(Ed, Hd, steps, source=src)
    plan.set_step(0)
    energy = plan.run(Ec, Hc, steps, source=src, energy_every=1)
    plan.close()
    assert np.all(np.isfinite(energy))
    for a, b in zip(Ed + Hd, Ec + Hc):
        assert torch.equal(a, b)


@pytest.mark.parametrize("form", ["fundamental", "conventional"])
def test_output_with_permeability_map(case, form):
    """Fundamental forms with a permeability map write the output directly,
    conventional ones through the copy; both equal their energy-trace runs."""
    from paper_2011_14043_amd import Source
    rng = np.random.default_rng(33)
    mu = rng.uniform(1, 3, (case["nz"], case["ny"], case["nx"])).astype(np.float32)
    dt = case["dt"]
    src = Source(11, 7, 13, f0=1 / (12 * dt), tau=3 * dt, t0=2 * dt, amp=1e10)
    plan = _plan(case, "adi", form, "f64", mu=mu)
    Ed, Hd = _fields(case, torch.float64)
    Ec, Hc = _fields(case, torch.float64)
    plan.run(Ed, Hd, 7, source=src)
    plan.set_step(0)
    plan.run(Ec, Hc, 7, source=src, energy_every=7)
    plan.close()
    for a, b in zip(Ed + Hd, Ec + Hc):
        assert torch.equal(a, b)
