"""Permeability maps (mu_r per cell, eq. (AMat) with the 1/mu entries and
eq. (bd), d = dt/(2 mu)): the HIP library against the FP64 oracle, whose
schemes with random eps and mu are pinned to the dense matrix formulas on the
CPU.

With mu varying along a line the scaled line systems have per-row
off-diagonals, which the permeability-map kernel variants solve.  Checked on a
ragged grid with mu_r ~ U[1, 3] independently per cell (every H sample of a
line differs from its neighbours), random eps_r boxes, a point source and
CFL 10: every scheme in both forms at every precision, the energy trace, the
input and output processing, every kernel configuration the autotuner may
pick, the adjoint gradient, the energy-weighted distance, and the argument
checks.  Bars as for unit permeability: FP64 1e-11, FP32 fields with FP64
solves 2e-6, FP32 2e-5 after a dozen steps (energy trace 10x)."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import adjoint
from oracle.source import Source as OSource

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PREC = {"f64": (torch.float64, torch.float64), "f32": (torch.float32, torch.float32),
        "f32s64": (torch.float32, torch.float64)}
TOL = {"f64": 1e-11, "f32": 2e-5, "f32s64": 2e-6}
STEPS, EVERY = 12, 3


def _run(c, scheme, form, prec, steps=STEPS, every=EVERY, mu=True, cfg=None, src=True):
    from paper_2011_14043_amd import Plan, Source
    dtype, solve = PREC[prec]
    E = [torch.tensor(a, dtype=dtype, device=DEV) for a in c["u0"][:3]]
    H = [torch.tensor(a, dtype=dtype, device=DEV) for a in c["u0"][3:]]
    plan = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["h"], c["h"], scheme=scheme, form=form, dtype=dtype,
                solve_dtype=solve, eps_r=torch.tensor(c["eps"]), mu_r=torch.tensor(c["mu"]) if mu else None)
    if cfg is not None:
        for ax, kc in cfg.items():
            plan.set_kernel_config(ax, **kc)
    s = c["src"]
    source = Source(s.i, s.j, s.k, f0=s.f0, tau=s.tau, t0=s.t0, amp=s.amp) if src else None
    tr = plan.run(E, H, steps, source=source, energy_every=every)
    torch.cuda.synchronize()
    refined = plan.refined
    plan.close()
    return [t.double().cpu().numpy() for t in E + H], tr, refined


@pytest.fixture(scope="module")
def case():
    nx, ny, nz, h = 37, 30, 45, 1e-3
    dt = W.yee_dt(h, h, h, 10.0)
    eps = W.random_box_eps(nx, ny, nz, seed=31, nboxes=8)
    mu = W.random_mu(nx, ny, nz, seed=32)
    u0 = W.random_fields(nx, ny, nz, seed=33)
    ci = W.interior_cell(nx, ny, nz, seed=34)
    src = OSource(*ci, amp=1e12, t0=3 * dt, tau=3 * dt, f0=1 / (12 * dt))
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps, mu)
    refs = {s: oracle.run(s, "fundamental", g, u0, STEPS, src, EVERY) for s in oracle.SCHEMES}
    refs["dy"] = oracle.run("dy", "fundamental", g, u0, STEPS, src, EVERY)
    refs["dg"] = oracle.run("dg", "fundamental", g, u0, STEPS, src, EVERY)
    return dict(nx=nx, ny=ny, nz=nz, h=h, dt=dt, eps=eps, mu=mu, u0=u0, src=src, g=g, refs=refs)


def _check(c, got, tr, ref, tr_ref, tol, tag):
    err = oracle.yee.weighted_rel_l2(got, ref, c["g"])
    terr = float(np.max(np.abs(np.array(tr) - np.array(tr_ref)) / np.abs(np.array(tr_ref))))
    print(f"  {tag}: rel-L2 {err:.3e}  energy {terr:.3e}", flush=True)
    assert err < tol, err
    assert terr < 10 * tol, terr
    # outside-the-box entries untouched, wall-tangential E exactly 0
    for n, comp in enumerate(W.COMPONENTS):
        if comp[0] == "E":
            wall = W.wall_tangential_mask(comp, c["nx"], c["ny"], c["nz"]) & \
                W.extent_mask(comp, c["nx"], c["ny"], c["nz"])
            assert np.all(got[n][wall] == 0.0)
        out = ~W.extent_mask(comp, c["nx"], c["ny"], c["nz"])
        assert np.array_equal(got[n][out], c["u0"][n][out].astype(got[n].dtype))


@pytest.mark.parametrize("prec", ["f64", "f32", "f32s64"])
@pytest.mark.parametrize("form", ["fundamental", "conventional"])
@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_mu_parity(case, scheme, form, prec):
    print(f"[case] mu map 37x30x45 {scheme}/{form}/{prec}", flush=True)
    got, tr, refined = _run(case, scheme, form, prec)
    assert not refined   # permeability maps solve without refinement
    ref, tr_ref = case["refs"][scheme]
    _check(case, got, tr, ref, tr_ref, TOL[prec], f"{scheme}/{form}/{prec}")


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("scheme,key", [("dyakonov", "dy"), ("douglas_gunn", "dg")])
def test_mu_splittings(case, scheme, key, prec):
    """D'Yakonov and Douglas-Gunn (the fundamental ADI passes) against the
    oracle's own forms of these splittings."""
    print(f"[case] mu map {scheme}/{prec}", flush=True)
    got, tr, _ = _run(case, scheme, "fundamental", prec)
    ref, tr_ref = case["refs"][key]
    _check(case, got, tr, ref, tr_ref, TOL[prec], f"{scheme}/{prec}")


def _cfg_params():
    out = []
    for prec, yz in (("f32", [(16, 16, 512), (8, 16, 512), (8, 8, 512)]), ("f64", [(8, 16, 512), (8, 8, 512)]),
                     ("f32s64", [(8, 16, 512), (8, 8, 512)])):
        for M, TX, NT in yz:
            for wpb in (1, 4):
                out.append(pytest.param(prec, (M, TX, NT), wpb, id=f"{prec}-yz{M}-{TX}-{NT}-x{wpb}"))
    return out


@pytest.mark.parametrize("scheme,form", [("adi", "fundamental"), ("adi", "conventional"),
                                         ("lod1", "conventional")])
@pytest.mark.parametrize("prec,yz,wpb", _cfg_params())
def test_mu_kernel_configs(case, scheme, form, prec, yz, wpb):
    """Every permeability-map kernel variant the autotuner may pick."""
    M, TX, NT = yz
    print(f"[case] mu configs {scheme}/{form}/{prec} yz={yz} x wpb={wpb}", flush=True)
    cfg = {0: dict(chunk=8, block_threads=64 * wpb, remap=1)}
    for ax in (1, 2):
        cfg[ax] = dict(chunk=M, tile_x=TX, block_threads=NT, remap=1)
    got, tr, _ = _run(case, scheme, form, prec, cfg=cfg)
    ref, tr_ref = case["refs"][scheme]
    _check(case, got, tr, ref, tr_ref, TOL[prec], "config")


def test_mu_unsupported_configs(case):
    """Variants not built for permeability maps are rejected."""
    from paper_2011_14043_amd import FdtdError, Plan
    c = case
    p = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["h"], c["h"], eps_r=torch.tensor(c["eps"]),
             mu_r=torch.tensor(c["mu"]))
    try:
        with pytest.raises(FdtdError):
            p.set_kernel_config(0, chunk=16, block_threads=256, remap=1)
        with pytest.raises(FdtdError):
            p.set_kernel_config(1, chunk=16, tile_x=32, block_threads=1024, remap=1)
    finally:
        p.close()


def test_mu_autotuned(case):
    """The autotuner's choice for a permeability-map plan, against the oracle."""
    from paper_2011_14043_amd import Plan, Source
    c = case
    E = [torch.tensor(a, dtype=torch.float32, device=DEV) for a in c["u0"][:3]]
    H = [torch.tensor(a, dtype=torch.float32, device=DEV) for a in c["u0"][3:]]
    p = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["h"], c["h"], eps_r=torch.tensor(c["eps"]),
             mu_r=torch.tensor(c["mu"]))
    p.autotune(2)
    cfg = [p.kernel_config(ax) for ax in range(3)]
    print(f"[case] mu autotuned {cfg}", flush=True)
    assert cfg[0]["chunk"] == 8
    s = c["src"]
    tr = p.run(E, H, STEPS, source=Source(s.i, s.j, s.k, f0=s.f0, tau=s.tau, t0=s.t0, amp=s.amp),
               energy_every=EVERY)
    torch.cuda.synchronize()
    p.close()
    ref, tr_ref = c["refs"]["adi"]
    _check(c, [t.double().cpu().numpy() for t in E + H], tr, ref, tr_ref, TOL["f32"], "autotuned")


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mu_of_ones_is_unit_permeability(case, prec):
    """A map of ones runs the unit-permeability passes: bit for bit the plan
    without a map."""
    c = dict(case)
    c["mu"] = np.ones_like(case["mu"])
    a, tra, ra = _run(c, "adi", "fundamental", prec)
    b, trb, rb = _run(c, "adi", "fundamental", prec, mu=False)
    assert ra == rb
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    assert np.array_equal(np.array(tra), np.array(trb))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mu_long_lines_and_full_chunks(prec):
    """Lines of 512 cells (the longest a permeability map allows: 64 chunks of
    8 slots), lines that fill their chunks exactly, anisotropic cells and
    mu_r up to 5, both forms, against the oracle."""
    nx, ny, nz = 512, 8, 16
    hx, hy, hz = 0.5e-3, 1e-3, 0.8e-3
    dt = W.yee_dt(hx, hy, hz, 6.0)
    eps = W.random_box_eps(nx, ny, nz, seed=41, nboxes=6)
    mu = W.random_mu(nx, ny, nz, seed=42, vmin=1.0, vmax=5.0)
    u0 = W.random_fields(nx, ny, nz, seed=43)
    g = oracle.Grid(nx, ny, nz, hx, hy, hz, dt, eps, mu)
    ref, _ = oracle.run("adi", "fundamental", g, u0, 4)
    from paper_2011_14043_amd import Plan
    dtype, solve = PREC[prec]
    print(f"[case] mu long lines 512x8x16 {prec}", flush=True)
    for form in ("fundamental", "conventional"):
        E = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[:3]]
        H = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[3:]]
        p = Plan(nx, ny, nz, dt, hx, hy, hz, form=form, dtype=dtype, solve_dtype=solve, eps_r=torch.tensor(eps),
                 mu_r=torch.tensor(mu))
        p.run(E, H, 4)
        torch.cuda.synchronize()
        p.close()
        err = oracle.yee.weighted_rel_l2([t.double().cpu().numpy() for t in E + H], ref, g)
        print(f"  {form}: rel-L2 {err:.3e}", flush=True)
        assert err < TOL[prec], err


@pytest.mark.parametrize("form", ["fundamental", "conventional"])
@pytest.mark.parametrize("cfl", [2.0, 8.0])
def test_mu_crank_nicolson(cfl, form):
    """Crank-Nicolson without factorization with a permeability map (1/mu of
    every H sample in the curls, the preconditioner diagonal and the H
    updates) against the oracle's sparse direct solve, FP64."""
    from paper_2011_14043_amd import Plan
    nx, ny, nz, h = 14, 12, 13, 1e-3
    dt = W.yee_dt(h, h, h, cfl)
    eps = W.random_box_eps(nx, ny, nz, seed=70, nboxes=6)
    mu = W.random_mu(nx, ny, nz, seed=73)
    u0 = W.random_fields(nx, ny, nz, seed=71)
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps, mu)
    print(f"[case] mu CN 14x12x13 CFL {cfl} {form}", flush=True)
    ref, tr_ref = oracle.run("cn", form, g, u0, 6, None, 1)
    p = Plan(nx, ny, nz, dt, h, h, h, scheme="crank_nicolson", form=form, dtype=torch.float64,
             eps_r=torch.tensor(eps), mu_r=torch.tensor(mu))
    p.set_cg(1e-13, 2000)
    E = [torch.tensor(a, dtype=torch.float64, device=DEV) for a in u0[:3]]
    H = [torch.tensor(a, dtype=torch.float64, device=DEV) for a in u0[3:]]
    tr = p.run(E, H, 6, energy_every=1)
    torch.cuda.synchronize()
    st = p.last_cg()
    p.close()
    err = oracle.yee.weighted_rel_l2([t.cpu().numpy() for t in E + H], ref, g)
    print(f"  rel-L2 {err:.3e}  iterations {st['iterations']}", flush=True)
    assert err < 1e-10, err
    assert np.allclose(tr, tr_ref, rtol=1e-10)


def test_mu_diff_norm(case):
    """fdtd_diff_norm weights H by mu0 mu_r of its cell (energy-weighted
    distance, as the oracle's)."""
    from paper_2011_14043_amd import Plan
    c = case
    a = W.random_fields(c["nx"], c["ny"], c["nz"], seed=35)
    b = W.random_fields(c["nx"], c["ny"], c["nz"], seed=36)
    p = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["h"], c["h"], dtype=torch.float64,
             eps_r=torch.tensor(c["eps"]), mu_r=torch.tensor(c["mu"]))
    ta = [torch.tensor(x, dtype=torch.float64, device=DEV) for x in a]
    tb = [torch.tensor(x, dtype=torch.float64, device=DEV) for x in b]
    num, den = p.diff_norm(ta[:3], ta[3:], tb[:3], tb[3:])
    p.close()
    got = float(np.sqrt(num / den))
    ref = oracle.yee.weighted_rel_l2(a, b, c["g"])
    print(f"[case] mu diff_norm {got:.15e} vs {ref:.15e}", flush=True)
    assert abs(got - ref) <= 1e-12 * ref


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_mu_adjoint_gradient(prec):
    """dJ/d eps_r with a permeability map against the oracle's reverse-mode
    gradient (tiny grid)."""
    from paper_2011_14043_amd import Plan, Source
    nx, ny, nz, h = 5, 4, 6, 1e-3
    dt = W.yee_dt(h, h, h, 3.0)
    eps = W.random_box_eps(nx, ny, nz, seed=51, nboxes=3)
    mu = W.random_mu(nx, ny, nz, seed=52)
    u0 = W.random_fields(nx, ny, nz, seed=53)
    src = OSource(2, 2, 2, amp=1e11, t0=3 * dt, tau=2 * dt, f0=1 / (10 * dt))
    probe = (3, 2, 3)
    steps = 10
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps, mu)
    J_ref, grad_ref = adjoint.gradient(g, u0, steps, src, probe)
    dtype, solve = PREC[prec]
    E = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[:3]]
    H = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[3:]]
    p = Plan(nx, ny, nz, dt, h, h, h, dtype=dtype, solve_dtype=solve, eps_r=torch.tensor(eps),
             mu_r=torch.tensor(mu))
    J, grad = p.grad_eps(E, H, steps, probe, Source(src.i, src.j, src.k, f0=src.f0, tau=src.tau, t0=src.t0,
                                                    amp=src.amp), (0, nx, 0, ny, 0, nz), 4)
    p.close()
    grad = grad.cpu().numpy()
    scale = np.max(np.abs(grad_ref))
    gerr = np.max(np.abs(grad - grad_ref)) / scale
    jerr = abs(J - J_ref) / abs(J_ref)
    print(f"[case] mu adjoint {prec}: J {jerr:.3e}  grad {gerr:.3e}", flush=True)
    tol = 1e-9 if prec == "f64" else 2e-4
    assert jerr < tol and gerr < tol


def test_mu_arguments(case):
    """Non-positive or non-finite mu_r, refinement and axes above 512 cells with
    a permeability map are rejected."""
    from paper_2011_14043_amd import FdtdError, Plan
    c = case
    args = (c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["h"], c["h"])
    for bad in (0.0, -1.0, np.inf, np.nan):
        m = c["mu"].copy()
        m[3, 4, 5] = bad
        with pytest.raises(FdtdError, match="EINVAL"):
            Plan(*args, mu_r=torch.tensor(m))
    mu = torch.tensor(c["mu"])
    with pytest.raises(FdtdError, match="EUNSUPPORTED"):
        Plan(*args, mu_r=mu, refine=True)
    with pytest.raises(ValueError):
        Plan(*args, mu_r=torch.ones(3, 3, 3))
    n = 520
    with pytest.raises(FdtdError, match="EUNSUPPORTED"):
        Plan(n, 2, 2, c["dt"], c["h"], c["h"], c["h"], mu_r=torch.full((2, 2, n), 2.0))
    # the same plan without the map is accepted (FP32 allows 1024 cells per axis)
    Plan(n, 2, 2, c["dt"], c["h"], c["h"], c["h"]).close()
