"""Every kernel configuration the autotuner may pick computes the same result
(to rounding) as the oracle: all FP32 y/z variants and x variants, on a
ragged grid and on a grid whose lines fill their chunks exactly."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.source import Source as OSource

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
YZ_F32 = [(16, 32, 1024), (16, 16, 512), (8, 16, 1024), (32, 16, 512), (8, 32, 512)]
X_CFG = [(8, 256), (8, 64), (16, 128)]


@pytest.fixture(scope="module", params=[(37, 45, 70), (64, 64, 64)], ids=["ragged", "full"])
def case(request):
    nx, ny, nz = request.param
    h = 1e-3
    dt = W.yee_dt(h, h, h, 10.0)
    eps = W.random_box_eps(nx, ny, nz, seed=5, nboxes=8)
    u0 = W.random_fields(nx, ny, nz, seed=6)
    src = OSource(*W.interior_cell(nx, ny, nz, seed=7), amp=1e12, t0=3 * dt, tau=3 * dt, f0=1 / (12 * dt))
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    refs = {(s, f): oracle.run(s, f, g, u0, 6, src)[0] for s, f in [("adi", "fundamental"), ("lod1", "conventional")]}
    return dict(nx=nx, ny=ny, nz=nz, h=h, dt=dt, eps=eps, u0=u0, src=src, g=g, refs=refs)


def _run(c, scheme, form, cfg_yz, cfg_x, refine=False):
    from paper_2011_14043_amd import FdtdError, Plan, Source
    E = [torch.tensor(a, dtype=torch.float32, device=DEV) for a in c["u0"][:3]]
    H = [torch.tensor(a, dtype=torch.float32, device=DEV) for a in c["u0"][3:]]
    plan = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["h"], c["h"], scheme=scheme, form=form,
                dtype=torch.float32, eps_r=torch.tensor(c["eps"]), refine=refine)
    try:
        M, TX, NT = cfg_yz
        for ax in (1, 2):
            plan.set_kernel_config(ax, chunk=M, tile_x=TX, block_threads=NT, remap=1)
        plan.set_kernel_config(0, chunk=cfg_x[0], block_threads=cfg_x[1], remap=1)
    except FdtdError:
        plan.close()
        return None
    s = c["src"]
    plan.run(E, H, 6, source=Source(s.i, s.j, s.k, f0=s.f0, tau=s.tau, t0=s.t0, amp=s.amp))
    torch.cuda.synchronize()
    plan.close()
    return [t.double().cpu().numpy() for t in E + H]


@pytest.mark.parametrize("scheme,form", [("adi", "fundamental"), ("lod1", "conventional")])
@pytest.mark.parametrize("cfg_yz", YZ_F32, ids=lambda v: "yz%d-%d-%d" % v)
def test_yz_variants(case, scheme, form, cfg_yz):
    print(f"[case] configs {case['nx']}x{case['ny']}x{case['nz']} {scheme}/{form} yz={cfg_yz}", flush=True)
    got = _run(case, scheme, form, cfg_yz, (8, 256))
    if got is None:
        pytest.skip("variant does not fit this grid")
    err = oracle.yee.weighted_rel_l2(got, case["refs"][(scheme, form)], case["g"])
    assert err <= 2e-5, err


@pytest.mark.parametrize("cfg_x", X_CFG, ids=lambda v: "x%d-%d" % v)
def test_x_variants(case, cfg_x):
    got = _run(case, "adi", "fundamental", (16, 16, 512), cfg_x)
    assert got is not None
    err = oracle.yee.weighted_rel_l2(got, case["refs"][("adi", "fundamental")], case["g"])
    assert err <= 2e-5, err


@pytest.mark.parametrize("scheme", ["adi", "ss2"])
@pytest.mark.parametrize("cfg_yz", [(8, 16, 1024), (8, 32, 512), (16, 32, 1024), (16, 16, 512)],
                         ids=lambda v: "yz%d-%d-%d" % v)
@pytest.mark.parametrize("wpb", [4, 1])
def test_refined_variants(case, scheme, cfg_yz, wpb):
    """Refined FP32 solves in every launch shape built for them (x lines:
    8-slot chunks; y/z lines: 8 or 16); other chunk lengths are rejected."""
    from paper_2011_14043_amd import FdtdError, Plan
    print(f"[case] refined {case['nx']}x{case['ny']}x{case['nz']} {scheme} yz={cfg_yz} wpb={wpb}", flush=True)
    got = _run(case, scheme, "fundamental", cfg_yz, (8, 64 * wpb), refine=True)
    if got is None:
        pytest.skip("variant does not fit this grid")
    ref = case["refs"][(scheme, "fundamental")] if scheme == "adi" else \
        oracle.run(scheme, "fundamental", case["g"], case["u0"], 6, case["src"])[0]
    err = oracle.yee.weighted_rel_l2(got, ref, case["g"])
    print(f"  rel-L2 {err:.3e}", flush=True)
    assert err <= 1e-5, err
    plan = Plan(case["nx"], case["ny"], case["nz"], case["dt"], case["h"], case["h"], case["h"], refine=True)
    try:
        with pytest.raises(FdtdError):
            plan.set_kernel_config(1, chunk=32, tile_x=16, block_threads=512, remap=1)
        with pytest.raises(FdtdError):
            plan.set_kernel_config(0, chunk=16, block_threads=256, remap=1)
    finally:
        plan.close()
