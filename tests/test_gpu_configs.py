"""Every kernel configuration the autotuner may pick computes the same result
(to rounding) as the oracle: every y/z variant built for the solve precision
(FP32 solves: 5, FP64 solves: 3) and every x variant, in FP32, FP64 and FP32
fields with FP64 solves, for fundamental ADI, conventional ADI (the cross-term
passes), conventional LOD1 and fundamental SS2, on a ragged grid and on a grid
whose lines fill their chunks exactly.  The refined FP32 passes have their own
sweep (every launch shape built for them)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle.source import Source as OSource

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
YZ_F32 = [(16, 32, 1024), (16, 16, 512), (8, 16, 1024), (32, 16, 512), (8, 32, 512)]
YZ_F64 = [(16, 16, 512), (8, 8, 512), (8, 16, 1024)]
X_CFG = [(8, 256), (8, 64), (16, 128)]
# precision key -> (field dtype, solve dtype, refine, y/z variants, bar after 6 steps)
PREC = {"f32p": (torch.float32, torch.float32, False, YZ_F32, 2e-5),
        "f64": (torch.float64, torch.float64, None, YZ_F64, 1e-11),
        "f32s64": (torch.float32, torch.float64, None, YZ_F64, 2e-6)}
SCHEME_FORMS = [("adi", "fundamental"), ("adi", "conventional"), ("lod1", "conventional"), ("ss2", "fundamental")]


@pytest.fixture(scope="module", params=[(37, 45, 70), (64, 64, 64)], ids=["ragged", "full"])
def case(request):
    nx, ny, nz = request.param
    h = 1e-3
    dt = W.yee_dt(h, h, h, 10.0)
    eps = W.random_box_eps(nx, ny, nz, seed=5, nboxes=8)
    u0 = W.random_fields(nx, ny, nz, seed=6)
    src = OSource(*W.interior_cell(nx, ny, nz, seed=7), amp=1e12, t0=3 * dt, tau=3 * dt, f0=1 / (12 * dt))
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    # both forms of a scheme give the same fields: one oracle run per scheme
    refs = {s: oracle.run(s, "fundamental", g, u0, 6, src)[0] for s in ("adi", "lod1", "ss2")}
    return dict(nx=nx, ny=ny, nz=nz, h=h, dt=dt, eps=eps, u0=u0, src=src, g=g, refs=refs)


def _run(c, scheme, form, cfg_yz, cfg_x, prec):
    from paper_2011_14043_amd import FdtdError, Plan, Source
    dtype, solve, refine = PREC[prec][:3] if prec in PREC else (torch.float32, torch.float32, True)
    E = [torch.tensor(a, dtype=dtype, device=DEV) for a in c["u0"][:3]]
    H = [torch.tensor(a, dtype=dtype, device=DEV) for a in c["u0"][3:]]
    plan = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["h"], c["h"], scheme=scheme, form=form,
                dtype=dtype, solve_dtype=solve, eps_r=torch.tensor(c["eps"]), refine=refine)
    try:
        M, TX, NT = cfg_yz
        for ax in (1, 2):
            plan.set_kernel_config(ax, chunk=M, tile_x=TX, block_threads=NT, remap=1)
        plan.set_kernel_config(0, chunk=cfg_x[0], block_threads=cfg_x[1], remap=1)
        for ax in (1, 2):
            assert plan.kernel_config(ax) == {"chunk": M, "tile_x": TX, "block_threads": NT, "remap": 1}
    except FdtdError:
        plan.close()
        return None
    s = c["src"]
    plan.run(E, H, 6, source=Source(s.i, s.j, s.k, f0=s.f0, tau=s.tau, t0=s.t0, amp=s.amp))
    torch.cuda.synchronize()
    plan.close()
    return [t.double().cpu().numpy() for t in E + H]


def _yz_params():
    out = []
    for prec, (_, _, _, yz, _) in PREC.items():
        for cfg in yz:
            out.append(pytest.param(prec, cfg, id=f"{prec}-yz%d-%d-%d" % cfg))
    return out


@pytest.mark.parametrize("scheme,form", SCHEME_FORMS, ids=[f"{s}-{f[:4]}" for s, f in SCHEME_FORMS])
@pytest.mark.parametrize("prec,cfg_yz", _yz_params())
def test_yz_variants(case, prec, scheme, form, cfg_yz):
    print(f"[case] configs {case['nx']}x{case['ny']}x{case['nz']} {scheme}/{form} {prec} yz={cfg_yz}", flush=True)
    got = _run(case, scheme, form, cfg_yz, (8, 256), prec)
    if got is None:
        # the only variants left out: those whose P chunks of M slots exceed a
        # block (long lines) and FP64 conventional ADI in 1024-thread blocks
        n_max = max(case["nx"], case["ny"], case["nz"])
        M, TX, NT = cfg_yz
        P = 1 << max(0, ((n_max + M - 1) // M - 1).bit_length())
        assert TX * P > NT or P > 64 or (prec == "f64" and scheme == "adi" and form == "conventional" and NT == 1024)
        pytest.skip("variant not built for this grid")
    err = oracle.yee.weighted_rel_l2(got, case["refs"][scheme], case["g"])
    print(f"  rel-L2 {err:.3e}", flush=True)
    assert err <= PREC[prec][4], err


@pytest.mark.parametrize("scheme,form", SCHEME_FORMS, ids=[f"{s}-{f[:4]}" for s, f in SCHEME_FORMS])
@pytest.mark.parametrize("prec", list(PREC))
@pytest.mark.parametrize("cfg_x", X_CFG, ids=lambda v: "x%d-%d" % v)
def test_x_variants(case, prec, scheme, form, cfg_x):
    print(f"[case] configs {case['nx']}x{case['ny']}x{case['nz']} {scheme}/{form} {prec} x={cfg_x}", flush=True)
    got = _run(case, scheme, form, (16, 16, 512), cfg_x, prec)
    assert got is not None
    err = oracle.yee.weighted_rel_l2(got, case["refs"][scheme], case["g"])
    print(f"  rel-L2 {err:.3e}", flush=True)
    assert err <= PREC[prec][4], err


@pytest.mark.parametrize("scheme", ["adi", "ss2"])
@pytest.mark.parametrize("cfg_yz", [(8, 16, 1024), (8, 32, 512), (16, 32, 1024), (16, 16, 512)],
                         ids=lambda v: "yz%d-%d-%d" % v)
@pytest.mark.parametrize("wpb", [4, 1])
def test_refined_variants(case, scheme, cfg_yz, wpb):
    """Refined FP32 solves in every launch shape built for them (x lines:
    8-slot chunks; y/z lines: 8 or 16); other chunk lengths are rejected."""
    from paper_2011_14043_amd import FdtdError, Plan
    print(f"[case] refined {case['nx']}x{case['ny']}x{case['nz']} {scheme} yz={cfg_yz} wpb={wpb}", flush=True)
    got = _run(case, scheme, "fundamental", cfg_yz, (8, 64 * wpb), "f32r")
    if got is None:
        pytest.skip("variant does not fit this grid")
    err = oracle.yee.weighted_rel_l2(got, case["refs"][scheme], case["g"])
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
