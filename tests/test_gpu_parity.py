"""GPU parity: the HIP library (through the C ABI) against the FP64 CPU oracle.

Tolerances (energy-weighted relative L2 over all six components): FP64 path
1e-11 (rounding order only); FP32 path 2e-6 per 10 steps of growth allowance
on these short runs (1e-4 is the bar after 1000 steps).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle.source import Source as OSource

from . import _analytic as an
from ._sampled import lod1_xline, lod1_yline, lod1_zline

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _lib():
    from paper_2011_14043_amd import Plan, Source
    return Plan, Source


PREC = {"f64": (torch.float64, torch.float64), "f32": (torch.float32, torch.float32),
        "f32s64": (torch.float32, torch.float64), "f32r": (torch.float32, torch.float32)}
REFINED = {"f32r"}   # FP32 solves refined once (fundamental forms only)


def gpu_run(scheme, form, dtype, nx, ny, nz, dt, h, eps, u0, steps, src=None, every=0):
    """dtype: a key of PREC or a torch dtype."""
    Plan, Source = _lib()
    refine = isinstance(dtype, str) and dtype in REFINED
    dtype, solve = PREC[dtype] if isinstance(dtype, str) else (dtype, dtype)
    dev = torch.device(DEV)
    hx, hy, hz = h if isinstance(h, tuple) else (h, h, h)
    E = [torch.tensor(a, dtype=dtype, device=dev) for a in u0[:3]]
    H = [torch.tensor(a, dtype=dtype, device=dev) for a in u0[3:]]
    plan = Plan(nx, ny, nz, dt, hx, hy, hz, scheme=scheme, form=form, dtype=dtype, solve_dtype=solve,
                eps_r=None if eps is None else torch.tensor(eps), refine=refine)
    s = None
    if src is not None:
        s = Source(src.i, src.j, src.k, f0=src.f0, tau=src.tau, t0=src.t0, amp=src.amp)
    tr = plan.run(E, H, steps, source=s, energy_every=every)
    torch.cuda.synchronize()
    plan.close()
    return [t.double().cpu().numpy() for t in E + H], tr


TOL = {"f64": 1e-11, "f32": 2e-5, "f32s64": 2e-6, "f32r": 1e-5}


@pytest.fixture(scope="module")
def ragged_case():
    """37 x 45 x 70 cells: ragged x tiles, several chunks per line, CFL 10,
    random boxes, random fields, a point source; oracle per scheme."""
    nx, ny, nz, h = 37, 45, 70, 1e-3
    dt = W.yee_dt(h, h, h, 10.0)
    eps = W.random_box_eps(nx, ny, nz, seed=2, nboxes=8)
    u0 = W.random_fields(nx, ny, nz, seed=3)
    ci = W.interior_cell(nx, ny, nz, seed=4)
    src = OSource(*ci, amp=1e12, t0=3 * dt, tau=3 * dt, f0=1 / (12 * dt))
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    refs = {s: oracle.run(s, "fundamental", g, u0, 12, src, 3) for s in oracle.SCHEMES}
    return dict(nx=nx, ny=ny, nz=nz, h=h, dt=dt, eps=eps, u0=u0, src=src, g=g, refs=refs)


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s64", "f32r"])
@pytest.mark.parametrize("form", ["fundamental", "conventional"])
@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_ragged_parity(ragged_case, scheme, form, dtype):
    if dtype in REFINED and form == "conventional":
        pytest.skip("refined solves are built for the fundamental forms")
    c = ragged_case
    print(f"[case] ragged 37x45x70 {scheme}/{form}/{dtype}", flush=True)
    got, tr = gpu_run(scheme, form, dtype, c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["eps"], c["u0"], 12,
                      c["src"], 3)
    ref, tr_ref = c["refs"][scheme]
    err = oracle.yee.weighted_rel_l2(got, ref, c["g"])
    terr = np.max(np.abs(np.array(tr) - np.array(tr_ref)) / np.abs(np.array(tr_ref)))
    print(f"  rel-L2 {err:.3e}  energy {terr:.3e}")
    assert err < TOL[dtype]
    assert terr < 10 * TOL[dtype]
    # outside-the-box entries untouched, wall-tangential E exactly 0
    for n, comp in enumerate(W.COMPONENTS):
        if comp[0] == "E":
            wall = W.wall_tangential_mask(comp, c["nx"], c["ny"], c["nz"]) & \
                W.extent_mask(comp, c["nx"], c["ny"], c["nz"])
            assert np.all(got[n][wall] == 0.0)
        out = ~W.extent_mask(comp, c["nx"], c["ny"], c["nz"])
        assert np.array_equal(got[n][out], c["u0"][n][out].astype(got[n].dtype))


@pytest.mark.parametrize("dtype", ["f64", "f32", "f32s64", "f32r"])
@pytest.mark.parametrize("form", ["fundamental", "conventional"])
def test_cavity_24cube_200_steps(dtype, form):
    if dtype in REFINED and form == "conventional":
        pytest.skip("refined solves are built for the fundamental forms")
    """24^3 vacuum PEC cavity, 1 mm, CFL 4, N(0,1) fields, 200 steps, energy
    trace every step (the small configuration)."""
    n, h = 24, 1e-3
    dt = W.yee_dt(h, h, h, 4.0)
    u0 = W.random_fields(n, n, n, seed=1)
    g = oracle.Grid(n, n, n, h, h, h, dt)
    ref, tr_ref = oracle.run("adi", "fundamental", g, u0, 200, None, 1)
    got, tr = gpu_run("adi", form, dtype, n, n, n, dt, h, None, u0, 200, None, 1)
    err = oracle.yee.weighted_rel_l2(got, ref, g)
    tr, tr_ref = np.array(tr), np.array(tr_ref)
    drift = np.max(np.abs(tr - tr[0])) / tr[0]
    print(f"[case] 24^3 cavity, CFL 4, 200 steps {form}/{dtype}: rel-L2 {err:.3e}, drift {drift:.3e}")
    # pure FP32 solves: the pivots 2 + sigma - g are rounded the same way at
    # every node of a uniform region, a coherent error of ~eps (1 + sqrt(sigma))
    # / sigma in sigma, so drift and field error grow ~linearly (~5e-8 / step here)
    # (one refinement step removes that bias: what is left grows like a random walk)
    tol = {"f64": 1e-11, "f32": 3e-5, "f32s64": 2e-6, "f32r": 1e-5}[dtype]
    assert err < tol
    assert np.max(np.abs(tr - tr_ref) / tr_ref) < tol
    assert drift < {"f64": 1e-12, "f32": 3e-5, "f32s64": 1e-6, "f32r": 1e-5}[dtype]


@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
@pytest.mark.parametrize("form", ["fundamental", "conventional"])
def test_anisotropic_long_lines(scheme, form):
    """Unequal cell sizes and a 600-cell axis (larger chunks) in FP32 and FP64."""
    nx, ny, nz = 600, 9, 7
    hs = (0.9e-3, 1.3e-3, 1.1e-3)
    dt = W.yee_dt(*hs, 6.0)
    eps = W.random_box_eps(nx, ny, nz, seed=5, nboxes=10)
    u0 = W.random_fields(nx, ny, nz, seed=6)
    g = oracle.Grid(nx, ny, nz, *hs, dt, eps)
    ref, _ = oracle.run(scheme, "fundamental", g, u0, 6)
    got, _ = gpu_run(scheme, form, "f32", nx, ny, nz, dt, hs, eps, u0, 6)
    assert oracle.yee.weighted_rel_l2(got, ref, g) < 1e-5
    g2 = oracle.Grid(7, 9, 300, *hs, dt)  # z-long lines in FP64 (<= 512 cells)
    u1 = W.random_fields(7, 9, 300, seed=7)
    ref2, _ = oracle.run(scheme, "fundamental", g2, u1, 4)
    got2, _ = gpu_run(scheme, form, "f64", 7, 9, 300, dt, hs, None, u1, 4)
    assert oracle.yee.weighted_rel_l2(got2, ref2, g2) < 1e-11


@pytest.fixture(scope="module")
def max_line_refs():
    """Lines of the longest length a plan accepts along each axis: 1024 cells
    for FP32 fields, 512 for FP64; CFL 8, random boxes, a source."""
    out = {}
    for prec, nmax in (("f32", 1024), ("f64", 512)):
        for axis in range(3):
            dims = [11, 9, 10]
            dims[axis] = nmax
            nx, ny, nz = dims
            h = 1e-3
            dt = W.yee_dt(h, h, h, 8.0)
            eps = W.random_box_eps(nx, ny, nz, seed=20 + axis, nboxes=8)
            u0 = W.random_fields(nx, ny, nz, seed=30 + axis)
            src = OSource(*W.interior_cell(nx, ny, nz, seed=40 + axis, margin=2), amp=1e12, t0=2 * dt, tau=2 * dt,
                          f0=1 / (10 * dt))
            g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
            out[(prec, axis)] = (dims, dt, h, eps, u0, src, g, oracle.run("adi", "fundamental", g, u0, 5, src)[0])
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_maximum_line_length(max_line_refs, prec, axis):
    (nx, ny, nz), dt, h, eps, u0, src, g, ref = max_line_refs[(prec, axis)]
    print(f"[case] max line length {prec} {nx}x{ny}x{nz}", flush=True)
    got, _ = gpu_run("adi", "fundamental", prec, nx, ny, nz, dt, h, eps, u0, 5, src)
    err = oracle.yee.weighted_rel_l2(got, ref, g)
    assert err < (2e-5 if prec == "f32" else 1e-11), err


@pytest.mark.parametrize("dims", [(2, 2, 2), (2, 3, 4), (5, 2, 3), (64, 2, 2)])
def test_degenerate_small_grids(dims):
    nx, ny, nz = dims
    h = 1e-3
    dt = W.yee_dt(h, h, h, 3.0)
    u0 = W.random_fields(nx, ny, nz, seed=8)
    g = oracle.Grid(nx, ny, nz, h, h, h, dt)
    for scheme in ("adi", "lod2"):
        ref, _ = oracle.run(scheme, "fundamental", g, u0, 5)
        for form in ("fundamental", "conventional"):
            got, _ = gpu_run(scheme, form, "f64", nx, ny, nz, dt, h, None, u0, 5)
            assert oracle.yee.weighted_rel_l2(got, ref, g) < 1e-11


def test_zero_steps_leaves_fields():
    n, h = 8, 1e-3
    dt = W.yee_dt(h, h, h, 2.0)
    u0 = W.random_fields(n, n, n, seed=9)
    got, tr = gpu_run("adi", "fundamental", "f64", n, n, n, dt, h, None, u0, 0, None, 1)
    for a, b in zip(got, u0):
        assert np.array_equal(a, b)
    g = oracle.Grid(n, n, n, h, h, h, dt)
    assert abs(tr[0] - oracle.conventional.invariant("adi", oracle.yee.clean(u0, g), g)) < 1e-12 * tr[0]


def _mode_on_gpu(nx, ny, nz, h, mnp, amps, dtype):
    """Cavity mode (m, n, p) sampled on the GPU (test-side helper)."""
    (kx, ky, kz), _ = an.wavenumbers(nx, ny, nz, h, h, h, *mnp)
    dev = torch.device(DEV)
    f64 = torch.float64

    def ax(n_, k_, half):
        x = (torch.arange(n_ + 1, device=dev, dtype=f64) + half) * h * k_
        return x

    xi, xh = ax(nx, kx, 0.0), ax(nx, kx, 0.5)
    yi, yh = ax(ny, ky, 0.0), ax(ny, ky, 0.5)
    zi, zh = ax(nz, kz, 0.0), ax(nz, kz, 0.5)
    s, c = torch.sin, torch.cos
    prof = [
        (s(zi), s(yi), c(xh)), (s(zi), c(yh), s(xi)), (c(zh), s(yi), s(xi)),
        (c(zh), c(yh), s(xi)), (c(zh), s(yi), c(xh)), (s(zi), c(yh), c(xh)),
    ]
    out = []
    for n_, (pz, py, px) in enumerate(prof):
        a = amps[n_] * pz[:, None, None] * py[None, :, None] * px[None, None, :]
        comp = W.COMPONENTS[n_]
        # extent, wall-tangential E
        if comp in ("Ex", "Hy", "Hz"):
            a[:, :, nx] = 0
        if comp in ("Ey", "Hx", "Hz"):
            a[:, ny, :] = 0
        if comp in ("Ez", "Hx", "Hy"):
            a[nz, :, :] = 0
        if comp == "Ex":
            a[:, [0, ny], :] = 0
            a[[0, nz], :, :] = 0
        if comp == "Ey":
            a[:, :, [0, nx]] = 0
            a[[0, nz], :, :] = 0
        if comp == "Ez":
            a[:, :, [0, nx]] = 0
            a[:, [0, ny], :] = 0
        out.append(a.to(dtype).contiguous())
    return out


@pytest.mark.parametrize("n,prec,steps,form", [(128, "f64", 20, "fundamental"), (512, "f32", 10, "fundamental"),
                                               (512, "f32s64", 10, "fundamental"), (512, "f32r", 10, "fundamental"),
                                               (512, "f32", 10, "conventional"), (512, "f64", 10, "conventional"),
                                               (512, "f32s64", 10, "conventional")],
                         ids=["128-f64", "512-f32", "512-f32s64", "512-f32r", "512-f32-conv", "512-f64-conv",
                              "512-f32s64-conv"])
def test_cavity_mode_at_full_size(n, prec, steps, form):
    """A PEC cavity mode evolves by the exact 6x6 ADI amplification matrix at
    any grid size (eq. (clsADI); the fundamental form equals it): property pin
    at the benchmark size, 512^3.  Fundamental FP32 in the kernel
    configuration of the benchmark's FP32 plans (x lines 8-slot chunks in
    128-thread blocks, y/z lines 16-slot chunks, 32-wide tiles, 1024-thread
    variant, XCD-aware order); conventional ADI (the baseline of the
    fundamental-versus-conventional comparison, its cross-term passes) in
    whatever configuration the autotuner picks, as in the benchmark."""
    Plan, _ = _lib()
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    mnp = (3, 2, 5)
    a = np.random.default_rng(11).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(n, n, n, h, h, h, *mnp)
    M = an.scheme_matrix("adi", A6, B6, dt)
    amp = np.linalg.matrix_power(M, steps) @ a
    dtype, solve = PREC[prec]
    fields = _mode_on_gpu(n, n, n, h, mnp, a, dtype)
    plan = Plan(n, n, n, dt, h, h, h, scheme="adi", form=form, dtype=dtype, solve_dtype=solve,
                refine=True if prec in REFINED else (False if prec == "f32" else None))
    if form == "conventional":
        plan.autotune(3)
        print(f"  autotuned: {[plan.kernel_config(ax) for ax in range(3)]}", flush=True)
    elif n == 512 and prec in ("f32", "f32r"):
        plan.set_kernel_config(0, chunk=8, block_threads=128, remap=0)
        for ax in (1, 2):
            plan.set_kernel_config(ax, chunk=16, tile_x=32, block_threads=1024, remap=1)
    plan.run(fields[:3], fields[3:], steps)
    torch.cuda.synchronize()
    plan.close()
    ref = _mode_on_gpu(n, n, n, h, mnp, amp, torch.float64)
    w = [8.8541878128e-12] * 3 + [1.25663706212e-6] * 3
    num = sum(wi * float(torch.sum((f.double() - r) ** 2)) for wi, f, r in zip(w, fields, ref))
    den = sum(wi * float(torch.sum(r ** 2)) for wi, r in zip(w, ref))
    err = math.sqrt(num / den)
    print(f"[case] cavity mode {n}^3 {prec} {form}: rel-L2 {err:.3e}")
    assert err < {"f64": 1e-11, "f32": 2e-5, "f32s64": 2e-6, "f32r": 1e-5}[prec]


@pytest.fixture(scope="module")
def full_size_case():
    """512^3, the benchmark's medium (32 random eps_r boxes, seed 2), CFL 5,
    N(0,1) fields (seed 3)."""
    n, h = 512, 1e-3
    return n, h, W.yee_dt(h, h, h, 5.0), W.random_box_eps(n, n, n, seed=2, nboxes=32), W.random_fields(n, n, n, seed=3)


@pytest.mark.parametrize("form", ["fundamental", "conventional"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_lod1_sampled_lines_full_size(full_size_case, prec, form):
    """One LOD1 step, fundamental and conventional form, at 512^3 (FP32 in the
    benchmark's kernel configuration, and FP64): Ex and Hy on sampled z lines,
    Ey and Hz on x lines, Ez and Hx on y lines, next to the walls and inside,
    element by element against the oracle's sub-steps on the thin slabs those
    lines depend on (``_sampled.lod1_zline``, ``_xline``, ``_yline``, pinned against
    whole-grid oracle steps).  Bars as for a few steps: 2e-5 (FP32), 1e-11
    (FP64), energy-weighted relative L2 over the sampled lines."""
    Plan, _ = _lib()
    n, h, dt, eps, u0 = full_size_case
    dtype = torch.float32 if prec == "f32" else torch.float64
    print(f"[case] LOD1 {form} sampled lines 512^3 {prec}", flush=True)
    E = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[:3]]
    H = [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[3:]]
    plan = Plan(n, n, n, dt, h, h, h, scheme="lod1", form=form, dtype=dtype, eps_r=torch.from_numpy(eps))
    if prec == "f32":
        plan.set_kernel_config(0, chunk=8, block_threads=128, remap=0)
        for ax in (1, 2):
            plan.set_kernel_config(ax, chunk=16, tile_x=32, block_threads=1024, remap=1)
    plan.run(E, H, 1)
    torch.cuda.synchronize()
    plan.close()
    eps64 = eps.astype(np.float64)
    num = den = 0.0
    for i0, j0 in [(0, 1), (257, 300), (n - 1, n - 1), (100, 2)]:
        ref_ex, ref_hy = lod1_zline(eps64, u0[0][:, :, i0], u0[5][:, :, i0], u0[2][:, j0, :], u0[4][:, j0, :],
                                    i0, j0, h, dt, form)
        got_ex = E[0][:, j0, i0].double().cpu().numpy()
        got_hy = H[1][:, j0, i0].double().cpu().numpy()
        num += 8.8541878128e-12 * np.sum((got_ex - ref_ex) ** 2) + 1.25663706212e-6 * np.sum((got_hy - ref_hy) ** 2)
        den += 8.8541878128e-12 * np.sum(ref_ex ** 2) + 1.25663706212e-6 * np.sum(ref_hy ** 2)
    for j0, k0 in [(0, 1), (300, 257), (n - 1, n - 1), (2, 100)]:
        ref_ey, ref_hz = lod1_xline(eps64, u0[1][:, j0, :], u0[3][:, j0, :], u0[0][k0, :, :], u0[5][k0, :, :],
                                    j0, k0, h, dt, form)
        got_ey = E[1][k0, j0, :].double().cpu().numpy()
        got_hz = H[2][k0, j0, :].double().cpu().numpy()
        num += 8.8541878128e-12 * np.sum((got_ey - ref_ey) ** 2) + 1.25663706212e-6 * np.sum((got_hz - ref_hz) ** 2)
        den += 8.8541878128e-12 * np.sum(ref_ey ** 2) + 1.25663706212e-6 * np.sum(ref_hz ** 2)
    for k0, i0 in [(0, 1), (257, 300), (n - 1, n - 1), (100, 2)]:
        ref_ez, ref_hx = lod1_yline(eps64, u0[2][k0, :, :], u0[4][k0, :, :], u0[1][:, :, i0], u0[3][:, :, i0],
                                    k0, i0, h, dt, form)
        got_ez = E[2][k0, :, i0].double().cpu().numpy()
        got_hx = H[0][k0, :, i0].double().cpu().numpy()
        num += 8.8541878128e-12 * np.sum((got_ez - ref_ez) ** 2) + 1.25663706212e-6 * np.sum((got_hx - ref_hx) ** 2)
        den += 8.8541878128e-12 * np.sum(ref_ez ** 2) + 1.25663706212e-6 * np.sum(ref_hx ** 2)
    del E, H
    err = math.sqrt(num / den)
    print(f"[case] LOD1 {form} sampled lines 512^3 {prec}: rel-L2 {err:.3e}", flush=True)
    assert err < {"f32": 2e-5, "f64": 1e-11}[prec]


@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_energy_conserved_full_size(scheme):
    """The scheme's energy invariant at the benchmark's size and medium (512^3,
    32 random eps_r boxes, CFL 5), FP32 in the benchmark's kernel
    configuration, from a cavity mode (a PEC-compatible field; in the random
    medium it is no eigenmode, so every line solve does work).  Bar: FP32
    storage and solve rounding, a few units of 6e-8 per step of relative
    energy, 10 steps -> 2e-5."""
    Plan, _ = _lib()
    n, h = 512, 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    eps = torch.from_numpy(W.random_box_eps(n, n, n, seed=2, nboxes=32))
    a = np.random.default_rng(12).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    fields = _mode_on_gpu(n, n, n, h, (3, 2, 5), a, torch.float32)
    plan = Plan(n, n, n, dt, h, h, h, scheme=scheme, form="fundamental", dtype=torch.float32, eps_r=eps)
    plan.set_kernel_config(0, chunk=8, block_threads=128, remap=0)
    for ax in (1, 2):
        plan.set_kernel_config(ax, chunk=16, tile_x=32, block_threads=1024, remap=1)
    tr = np.array(plan.run(fields[:3], fields[3:], 10, energy_every=1))
    torch.cuda.synchronize()
    plan.close()
    drift = np.max(np.abs(tr - tr[0])) / tr[0]
    print(f"[case] energy 512^3 {scheme} f32: drift {drift:.3e} over {len(tr) - 1} steps")
    assert len(tr) == 11 and np.all(np.isfinite(tr))
    assert drift < 2e-5


@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_energy_conserved_cfl20(scheme):
    n, h = 40, 1e-3
    dt = W.yee_dt(h, h, h, 20.0)
    eps = W.random_box_eps(n, n, n, seed=12, nboxes=8)
    u0 = W.random_fields(n, n, n, seed=13)
    # pure FP32 solves drift by ~2e-7 per step at CFL 20 (coherent rounding of
    # the pivots 2 + sigma - g when sigma = 1/(2 beta) << 1); FP64 solves on
    # FP32 fields drift only by random storage rounding
    for dtype, tol in (("f64", 1e-12), ("f32", 1e-4), ("f32s64", 2e-6)):
        _, tr = gpu_run(scheme, "fundamental", dtype, n, n, n, dt, h, eps, u0, 100, None, 10)
        tr = np.array(tr)
        drift = np.max(np.abs(tr - tr[0])) / tr[0]
        print(f"[case] energy {scheme} {dtype} drift {drift:.3e}")
        assert drift < tol


@pytest.mark.parametrize("scheme", ["adi", "ss2"])
def test_per_cell_eps_float_path(scheme):
    """More than 256 distinct eps_r values: the passes read eps_r as FP32 per
    node instead of a material index (both layouts must agree with the oracle)."""
    nx, ny, nz, h = 30, 31, 33, 1e-3
    dt = W.yee_dt(h, h, h, 7.0)
    eps = np.random.default_rng(21).uniform(1.0, 12.0, (nz, ny, nx)).astype(np.float32)
    u0 = W.random_fields(nx, ny, nz, seed=22)
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    ref, _ = oracle.run(scheme, "fundamental", g, u0, 8)
    for form in ("fundamental", "conventional"):
        got, _ = gpu_run(scheme, form, "f64", nx, ny, nz, dt, h, eps, u0, 8)
        assert oracle.yee.weighted_rel_l2(got, ref, g) < 1e-11
        got, _ = gpu_run(scheme, form, "f32", nx, ny, nz, dt, h, eps, u0, 8)
        assert oracle.yee.weighted_rel_l2(got, ref, g) < 2e-5
