"""Precision sweep: 128^3 cells, random-box eps_r (32 boxes), N(0,1) fields,
CFL number 10, 1000 steps, every fundamental scheme, FP64 / FP32-storage with
FP64 solves / FP32 (the library's choice) / FP32 with refined solves / plain
FP32 solves on the GPU against the FP64 oracle (fixtures written by
tests/golden/make_precision_sweep.py, which calls only the oracle).

Reported and checked at steps 100, 500 and 1000: the energy-weighted relative
L2 error over 4096 seeded samples per component, and the relative error of the
field's energy norm.  Bars: FP64 1e-10; every FP32-field mode the library
chooses by default (FP64 solves, FDTD_F32, refined FP32) 1e-4, the accuracy
target for FP32 fields after 1000 steps.  FDTD_F32 refines its solves (the
fundamental forms refine wherever refined passes are built); plain FP32 solves
(FDTD_F32_PLAIN) are swept too, as the comparison: their fixed rounding of the
diagonal 2 + sigma (a relative perturbation up to 1.2e-7 / sigma of the medium,
sigma = eps mu dw^2 / theta^2) and of the medium-only factors, the same at
every step, makes their error grow linearly with the step count, to 3e-4 at
CFL 10 (bar 1e-3), 4e-5 to 9e-5 at CFL 5 (bar 2e-4) and 4e-5 to 6e-5 at
CFL 1 (bar 1e-4).  Every scheme is also swept at CFL 5, the CFL number of
the 512^3 workload, and at CFL 1, the other end of its CFL range (fixtures
precision_sweep_<scheme>_cfl5.npz, _cfl1.npz)."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import yee

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
DEV = "cuda:0"
# precision key -> (field dtype, solve dtype, refine: None = the library's choice)
PREC = {"f64": (torch.float64, torch.float64, None), "f32s64": (torch.float32, torch.float64, None),
        "f32": (torch.float32, torch.float32, None), "f32r": (torch.float32, torch.float32, True),
        "f32p": (torch.float32, torch.float32, False)}
BAR = {"f64": 1e-10, "f32s64": 1e-4, "f32": 1e-4, "f32r": 1e-4, "f32p": 1e-3}
BAR_CFL5 = {"f32s64": 1e-4, "f32": 1e-4, "f32r": 1e-4, "f32p": 2e-4}


def _golden(scheme):
    path = os.path.join(GOLDEN, f"precision_sweep_{scheme}.npz")
    if not os.path.exists(path):
        pytest.fail(f"missing fixture {path}: run tests/golden/make_precision_sweep.py {scheme}")
    return np.load(path)


@pytest.fixture(scope="module")
def setup():
    n, h = 128, 1e-3
    dt = W.yee_dt(h, h, h, 10.0)
    eps = W.random_box_eps(n, n, n, seed=2, nboxes=32)
    u0 = W.random_fields(n, n, n, seed=3)
    g = oracle.Grid(n, n, n, h, h, h, dt, eps)
    return dict(n=n, h=h, dt=dt, eps=eps, u0=u0, g=g)


def _sweep(c, ref, scheme, prec, expect_refined=None):
    from paper_2011_14043_amd import Plan
    n = c["n"]
    assert int(ref["n"]) == n
    dtype, solve, refine = PREC[prec]
    E = [torch.tensor(a, dtype=dtype, device=DEV) for a in c["u0"][:3]]
    H = [torch.tensor(a, dtype=dtype, device=DEV) for a in c["u0"][3:]]
    plan = Plan(n, n, n, c["dt"], c["h"], c["h"], c["h"], scheme=scheme, dtype=dtype, solve_dtype=solve,
                eps_r=torch.tensor(c["eps"]), refine=refine)
    # FDTD_F32 refines the fundamental forms' solves (at every CFL number)
    if expect_refined is None:
        expect_refined = prec in ("f32", "f32r")
    assert plan.refined == expect_refined
    done = 0
    errs, nerrs = [], []
    for m, step in enumerate(ref["steps"]):
        plan.run(E, H, int(step) - done)
        done = int(step)
        torch.cuda.synchronize()
        fields = [t.double().cpu().numpy() for t in E + H]
        num = den = 0.0
        for k, comp in enumerate(yee.COMPONENTS):
            idx = ref[f"idx_{comp}"]
            got = fields[k].ravel()[idx]
            want = ref[f"val_{comp}"][m]
            wt = c["g"].material(comp).ravel()[idx]
            num += float(np.sum(wt * (got - want) ** 2))
            den += float(np.sum(wt * want ** 2))
        err = (num / den) ** 0.5
        nerr = abs(yee.energy(fields, c["g"]) - ref["norm2"][m]) / ref["norm2"][m]
        errs.append(err)
        nerrs.append(nerr)
        print(f"  step {int(step):5d}: sampled rel-L2 {err:.3e}  energy-norm rel {nerr:.3e}", flush=True)
    plan.close()
    return errs, nerrs


@pytest.mark.parametrize("prec", ["f64", "f32s64", "f32", "f32r", "f32p"])
@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_precision_sweep(setup, scheme, prec):
    ref = _golden(scheme)
    print(f"[case] precision sweep 128^3 CFL10 {scheme}/{prec}", flush=True)
    errs, nerrs = _sweep(setup, ref, scheme, prec)
    assert max(errs) <= BAR[prec], errs       # steps 100, 500 and 1000
    assert max(nerrs) <= BAR[prec], nerrs


@pytest.fixture(scope="module")
def setup_cfl5(setup):
    c = dict(setup)
    c["dt"] = W.yee_dt(c["h"], c["h"], c["h"], 5.0)
    c["g"] = oracle.Grid(c["n"], c["n"], c["n"], c["h"], c["h"], c["h"], c["dt"], c["eps"])
    return c


@pytest.mark.parametrize("prec", ["f32s64", "f32", "f32r", "f32p"])
@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_precision_cfl5(setup_cfl5, scheme, prec):
    """The same sweep at CFL 5, the CFL number of the 512^3 workload."""
    ref = _golden(f"{scheme}_cfl5")
    assert float(ref["cfl"]) == 5.0
    print(f"[case] precision sweep 128^3 CFL5 {scheme}/{prec}", flush=True)
    errs, nerrs = _sweep(setup_cfl5, ref, scheme, prec)
    assert max(errs) <= BAR_CFL5[prec], errs
    assert max(nerrs) <= BAR_CFL5[prec], nerrs


@pytest.fixture(scope="module")
def setup_cfl1(setup):
    c = dict(setup)
    c["dt"] = W.yee_dt(c["h"], c["h"], c["h"], 1.0)
    c["g"] = oracle.Grid(c["n"], c["n"], c["n"], c["h"], c["h"], c["h"], c["dt"], c["eps"])
    return c


@pytest.mark.parametrize("prec", ["f32s64", "f32", "f32r", "f32p"])
@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_precision_cfl1(setup_cfl1, scheme, prec):
    """The same sweep at CFL 1 (smallest sigma 12)."""
    ref = _golden(f"{scheme}_cfl1")
    assert float(ref["cfl"]) == 1.0
    print(f"[case] precision sweep 128^3 CFL1 {scheme}/{prec}", flush=True)
    errs, nerrs = _sweep(setup_cfl1, ref, scheme, prec)
    assert max(errs) <= 1e-4, errs
    assert max(nerrs) <= 1e-4, nerrs
