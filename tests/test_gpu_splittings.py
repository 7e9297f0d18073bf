"""GPU parity of the D'Yakonov and Douglas-Gunn scheme ids (Sec. II-E)
against the oracle's own forms of those splittings, which the CPU pins tie to
the original formulae (orgDY), the delta formulation and Peaceman-Rachford;
with a source, the ADI convention."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.source import Source as OSource

from .test_gpu_parity import PREC, TOL, gpu_run

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def case():
    """37 x 45 x 70 cells (ragged tiles), CFL 10, random boxes and fields."""
    nx, ny, nz, h = 37, 45, 70, 1e-3
    dt = W.yee_dt(h, h, h, 10.0)
    eps = W.random_box_eps(nx, ny, nz, seed=12, nboxes=8)
    u0 = W.random_fields(nx, ny, nz, seed=13)
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    refs = {s: oracle.run(s, "fundamental", g, u0, 12, None, 3) for s in oracle.SPLITTINGS}
    return dict(nx=nx, ny=ny, nz=nz, h=h, dt=dt, eps=eps, u0=u0, g=g, refs=refs)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s64", "f32r"])
@pytest.mark.parametrize("scheme", ["dyakonov", "douglas_gunn"])
def test_splitting_parity(case, scheme, dtype):
    c = case
    key = "dy" if scheme == "dyakonov" else "dg"
    print(f"[case] 37x45x70 {scheme}/{dtype}", flush=True)
    got, tr = gpu_run(scheme, "fundamental", dtype, c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["eps"],
                      c["u0"], 12, None, 3)
    ref, tr_ref = c["refs"][key]
    err = oracle.yee.weighted_rel_l2(got, ref, c["g"])
    terr = np.max(np.abs(np.array(tr) - np.array(tr_ref)) / np.abs(np.array(tr_ref)))
    print(f"  rel-L2 {err:.3e}  energy {terr:.3e}")
    assert err < TOL[dtype]
    assert terr < 10 * TOL[dtype]


@pytest.mark.parametrize("scheme", ["dyakonov", "douglas_gunn"])
def test_splitting_runs_the_adi_passes(case, scheme):
    """Same kernels, input and output processing as fundamental ADI: the
    fields agree bit for bit."""
    c = case
    args = (c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["eps"], c["u0"], 7)
    a, _ = gpu_run("adi", "fundamental", "f32", *args)
    b, _ = gpu_run(scheme, "fundamental", "f32", *args)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("scheme", ["dyakonov", "douglas_gunn"])
def test_splitting_rejects_conventional_form(scheme):
    from paper_2011_14043_amd import Plan
    n, h = 16, 1e-3
    dt = W.yee_dt(h, h, h, 4.0)
    with pytest.raises(RuntimeError, match="EUNSUPPORTED"):
        Plan(n, n, n, dt, h, h, h, scheme=scheme, form="conventional")


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scheme", ["dyakonov", "douglas_gunn"])
def test_splitting_with_source(case, scheme, dtype):
    """With a point source: against the oracle's fundamental form with the ADI
    convention, and bit for bit against an ADI plan."""
    c = case
    key = "dy" if scheme == "dyakonov" else "dg"
    ci = W.interior_cell(c["nx"], c["ny"], c["nz"], seed=14)
    src = OSource(*ci, amp=1e12, t0=3 * c["dt"], tau=3 * c["dt"], f0=1 / (12 * c["dt"]))
    print(f"[case] 37x45x70 {scheme}/{dtype} with source", flush=True)
    ref, _ = oracle.run(key, "fundamental", c["g"], c["u0"], 12, src)
    args = (c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["eps"], c["u0"], 12, src)
    got, _ = gpu_run(scheme, "fundamental", dtype, *args)
    err = oracle.yee.weighted_rel_l2(got, ref, c["g"])
    print(f"  rel-L2 {err:.3e}")
    assert err < TOL[dtype]
    adi, _ = gpu_run("adi", "fundamental", dtype, *args)
    for x, y in zip(adi, got):
        assert np.array_equal(x, y)


def test_dyakonov_batch_equals_adi_batch():
    from paper_2011_14043_amd import BatchPlan
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    shapes = [(16, 18, 17), (21, 16, 25), (17, 23, 16)]
    grids, fields0 = [], []
    for g, (nx, ny, nz) in enumerate(shapes):
        grids.append((nx, ny, nz, torch.tensor(W.random_box_eps(nx, ny, nz, seed=50 + g, nboxes=4))))
        fields0.append(W.random_fields(nx, ny, nz, seed=60 + g))
    out = {}
    for scheme in ("adi", "dyakonov"):
        print(f"[case] batch of 3 grids {scheme}", flush=True)
        plan = BatchPlan(grids, dt, h, h, h, scheme=scheme, dtype=torch.float32)
        f = [([torch.tensor(a, dtype=torch.float32, device=DEV) for a in u0[:3]],
              [torch.tensor(a, dtype=torch.float32, device=DEV) for a in u0[3:]]) for u0 in fields0]
        plan.run(f, 10)
        torch.cuda.synchronize()
        plan.close()
        out[scheme] = [t.cpu() for E, H in f for t in E + H]
    for x, y in zip(out["adi"], out["dyakonov"]):
        assert torch.equal(x, y)


@pytest.mark.parametrize("scheme", ["dyakonov", "douglas_gunn"])
def test_splitting_gradient_equals_adi(scheme):
    """The adjoint gradient of a splitting plan is ADI's, bit for bit, with
    and without a source."""
    from paper_2011_14043_amd import Plan, Source
    nx, ny, nz, h = 24, 20, 18, 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    eps = torch.tensor(W.random_box_eps(nx, ny, nz, seed=80, nboxes=6))
    u0 = W.random_fields(nx, ny, nz, seed=81)
    E = [torch.tensor(a, dtype=torch.float64, device=DEV) for a in u0[:3]]
    H = [torch.tensor(a, dtype=torch.float64, device=DEV) for a in u0[3:]]
    box = (6, 14, 5, 12, 6, 10)
    out = {}
    src = Source(5, 6, 4, f0=1 / (10 * dt), tau=3 * dt, t0=4 * dt, amp=1e12)
    for s in ("adi", scheme):
        print(f"[case] gradient 24x20x18 {s}", flush=True)
        plan = Plan(nx, ny, nz, dt, h, h, h, scheme=s, dtype=torch.float64, eps_r=eps)
        out[s] = [plan.grad_eps(E, H, 30, (12, 10, 12), design_box=box, ckpt_every=7),
                  plan.grad_eps(E, H, 30, (12, 10, 12), src, design_box=box, ckpt_every=7)]
        torch.cuda.synchronize()
        plan.close()
    for a, b in zip(out["adi"], out[scheme]):
        assert a[0] == b[0]
        assert torch.equal(a[1], b[1])
