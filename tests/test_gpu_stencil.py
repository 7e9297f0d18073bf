"""Parameter-optimized 4-point differences on the GPU (fdtd_set_stencil on an
order-4 plan) against the FP64 oracle with the same outer weight, whose
operators and schemes are pinned on the CPU (tests/test_oracle_stencil.py).

Checked: every fundamental scheme at every precision on a ragged grid with
random eps_r boxes, a point source and CFL 10 (fields and energy trace), with
the least-squares weight for four samples per wavelength; a cavity mode at
48^3 against the exact 6x6 evolution with K(k) dw = 2 (1 - 3b) sin(k dw/2)
+ 2 b sin(3 k dw/2); energy conservation at CFL 20; the fourth-order weight
set back gives the fourth-order run bit for bit; the argument checks.  Bars as
for the fourth-order passes: FP64 1e-11, FP32 fields with FP64 solves 2e-6,
FP32 2e-5."""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.source import Source as OSource

from . import _analytic as an

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
# precision key -> (field dtype, solve dtype, refine): "f32" plain FP32 solves
PREC = {"f64": (torch.float64, torch.float64, None), "f32": (torch.float32, torch.float32, False),
        "f32s64": (torch.float32, torch.float64, None)}
TOL = {"f64": 1e-11, "f32": 2e-5, "f32s64": 2e-6}
STEPS, EVERY = 8, 2


def _b_opt():
    from paper_2011_14043_amd import optimized_stencil
    return optimized_stencil(math.pi / 2)


def _fields(u0, dtype):
    return ([torch.tensor(a, dtype=dtype, device=DEV) for a in u0[:3]],
            [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[3:]])


def _plan(c, scheme, prec, outer):
    from paper_2011_14043_amd import Plan
    dtype, solve, refine = PREC[prec]
    p = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["hx"], c["hy"], c["hz"], scheme=scheme, dtype=dtype,
             solve_dtype=solve, eps_r=None if c.get("eps") is None else torch.tensor(c["eps"]), refine=refine)
    p.set_order(4)
    p.set_stencil(outer)
    return p


def _gsrc(s):
    from paper_2011_14043_amd import Source
    return Source(s.i, s.j, s.k, f0=s.f0, tau=s.tau, t0=s.t0, amp=s.amp)


@pytest.fixture(scope="module")
def case():
    nx, ny, nz = 23, 19, 27
    hx, hy, hz = 1e-3, 1.2e-3, 0.9e-3
    dt = W.yee_dt(hx, hy, hz, 10.0)
    eps = W.random_box_eps(nx, ny, nz, seed=91, nboxes=8)
    u0 = W.random_fields(nx, ny, nz, seed=92)
    ci = W.interior_cell(nx, ny, nz, seed=93, margin=4)
    src = OSource(*ci, amp=1e12, t0=3 * dt, tau=3 * dt, f0=1 / (12 * dt))
    b = oracle.yee.optimized_outer(math.pi / 2)
    g = oracle.Grid(nx, ny, nz, hx, hy, hz, dt, eps, order=4, outer=b)
    refs = {s: oracle.run(s, "fundamental", g, u0, STEPS, src, EVERY) for s in oracle.SCHEMES}
    return dict(nx=nx, ny=ny, nz=nz, hx=hx, hy=hy, hz=hz, dt=dt, eps=eps, u0=u0, src=src, g=g, refs=refs, b=b)


def test_weight_from_library_equals_oracle(case):
    assert abs(_b_opt() - case["b"]) <= 1e-10 * abs(case["b"])


@pytest.mark.parametrize("prec", ["f64", "f32", "f32s64"])
@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_optimized_stencil_parity(case, scheme, prec):
    c = case
    print(f"[case] optimized stencil 23x19x27 {scheme}/{prec} b={c['b']:.6f}", flush=True)
    p = _plan(c, scheme, prec, c["b"])
    E, H = _fields(c["u0"], PREC[prec][0])
    tr = p.run(E, H, STEPS, source=_gsrc(c["src"]), energy_every=EVERY)
    torch.cuda.synchronize()
    p.close()
    got = [t.double().cpu().numpy() for t in E + H]
    ref, tr_ref = c["refs"][scheme]
    err = oracle.yee.weighted_rel_l2(got, ref, c["g"])
    terr = float(np.max(np.abs(np.array(tr) - np.array(tr_ref)) / np.abs(np.array(tr_ref))))
    print(f"  rel-L2 {err:.3e}  energy {terr:.3e}", flush=True)
    assert err < TOL[prec], err
    assert terr < 10 * TOL[prec], terr


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_optimized_stencil_cavity_mode(prec):
    n, h = 48, 1e-3
    dt = W.yee_dt(h, h, h, 6.0)
    mnp = (5, 3, 7)
    b = _b_opt()
    a = np.random.default_rng(9).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(n, n, n, h, h, h, *mnp, order=4, outer=b)
    N = 25
    ref = an.mode_fields(n, n, n, h, h, h, *mnp, np.linalg.matrix_power(an.scheme_matrix("adi", A6, B6, dt), N) @ a)
    u0 = an.mode_fields(n, n, n, h, h, h, *mnp, a)
    c = dict(nx=n, ny=n, nz=n, hx=h, hy=h, hz=h, dt=dt, eps=None)
    print(f"[case] optimized stencil cavity mode 48^3 {prec}", flush=True)
    p = _plan(c, "adi", prec, b)
    E, H = _fields(u0, PREC[prec][0])
    p.run(E, H, N)
    torch.cuda.synchronize()
    p.close()
    g = oracle.Grid(n, n, n, h, h, h, dt)
    err = oracle.yee.weighted_rel_l2([t.double().cpu().numpy() for t in E + H], ref, g)
    print(f"  rel-L2 {err:.3e}", flush=True)
    assert err < TOL[prec], err


def test_optimized_stencil_energy_conserved():
    nx, ny, nz, h = 20, 17, 15, 1e-3
    dt = W.yee_dt(h, h, h, 20.0)
    c = dict(nx=nx, ny=ny, nz=nz, hx=h, hy=h, hz=h, dt=dt, eps=W.random_box_eps(nx, ny, nz, seed=95, nboxes=6))
    p = _plan(c, "adi", "f64", _b_opt())
    E, H = _fields(W.random_fields(nx, ny, nz, seed=96), torch.float64)
    tr = np.array(p.run(E, H, 60, energy_every=10))
    p.close()
    drift = float(np.abs(tr - tr[0]).max() / tr[0])
    print(f"[case] optimized stencil energy drift {drift:.3e}", flush=True)
    assert drift < 1e-12


def test_fourth_order_weight_restores_fourth_order(case):
    """Setting b back to -1/24 gives the default fourth-order run bit for bit."""
    c = case
    pa = _plan(c, "adi", "f64", c["b"])
    pa.set_stencil(-1.0 / 24.0)
    from paper_2011_14043_amd import Plan
    pb = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["hx"], c["hy"], c["hz"], scheme="adi", dtype=torch.float64,
              eps_r=torch.tensor(c["eps"]))
    pb.set_order(4)
    fa, fb = _fields(c["u0"], torch.float64), _fields(c["u0"], torch.float64)
    pa.run(*fa, 6, source=_gsrc(c["src"]))
    pb.run(*fb, 6, source=_gsrc(c["src"]))
    torch.cuda.synchronize()
    pa.close()
    pb.close()
    for x, y in zip(fa[0] + fa[1], fb[0] + fb[1]):
        assert torch.equal(x, y)


def test_set_stencil_arguments(case):
    from paper_2011_14043_amd import FdtdError, Plan
    c = case
    p = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["hx"], c["hy"], c["hz"], scheme="adi", dtype=torch.float64)
    with pytest.raises(FdtdError) as e:
        p.set_stencil(-0.05)                 # second-order plan
    assert e.value.status == -4
    p.set_order(4)
    for bad in (0.3, -0.26, float("nan")):
        with pytest.raises(FdtdError) as e:
            p.set_stencil(bad)
        assert e.value.status == -1
    p.set_stencil(-0.05)
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_optimized_stencil_adjoint_gradient(prec):
    """The adjoint sweep with the optimized weight (its transposed sub-steps
    are the same passes with theta -> -theta) against the oracle's reverse
    mode on the same operator."""
    from oracle import adjoint
    nx, ny, nz, h = 5, 4, 6, 1e-3
    dt = W.yee_dt(h, h, h, 3.0)
    eps = W.random_box_eps(nx, ny, nz, seed=97, nboxes=3)
    u0 = W.random_fields(nx, ny, nz, seed=98)
    src = OSource(2, 2, 2, amp=1e11, t0=3 * dt, tau=2 * dt, f0=1 / (10 * dt))
    probe, steps = (3, 2, 3), 10
    b = _b_opt()
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps, order=4, outer=b)
    J_ref, grad_ref = adjoint.gradient(g, u0, steps, src, probe)
    c = dict(nx=nx, ny=ny, nz=nz, hx=h, hy=h, hz=h, dt=dt, eps=eps)
    p = _plan(c, "adi", prec, b)
    E, H = _fields(u0, PREC[prec][0])
    J, grad = p.grad_eps(E, H, steps, probe, _gsrc(src), (0, nx, 0, ny, 0, nz), 4)
    p.close()
    grad = grad.cpu().numpy()
    gerr = np.max(np.abs(grad - grad_ref)) / np.max(np.abs(grad_ref))
    jerr = abs(J - J_ref) / abs(J_ref)
    print(f"[case] optimized stencil adjoint {prec}: J {jerr:.3e}  grad {gerr:.3e}", flush=True)
    tol = 1e-9 if prec == "f64" else 2e-4
    assert jerr < tol and gerr < tol
