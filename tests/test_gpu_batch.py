"""Batched grids (fdtd_plan_batch / fdtd_run_batch): one launch per line pass
over all grids, one captured HIP graph per time step.  Checked against the
FP64 oracle per grid on small uneven grids and against the single-grid GPU
path on the 64-cavity workload (sizes U[16, 96], 500 steps, CFL 5)."""
import os

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PREC = {"f64": (torch.float64, torch.float64), "f32": (torch.float32, torch.float32),
        "f32s64": (torch.float32, torch.float64), "f32r": (torch.float32, torch.float32)}
TOL = {"f64": 1e-11, "f32": 2e-5, "f32s64": 2e-6, "f32r": 1e-5}


def _fields(u0, dtype):
    return ([torch.tensor(a, dtype=dtype, device=DEV) for a in u0[:3]],
            [torch.tensor(a, dtype=dtype, device=DEV) for a in u0[3:]])


def _grids(sizes, seed):
    out = []
    for g, (nx, ny, nz) in enumerate(sizes):
        eps = W.random_box_eps(nx, ny, nz, seed=seed + g, nboxes=32)
        u0 = W.random_fields(nx, ny, nz, seed=seed + 100 + g)
        out.append((nx, ny, nz, eps, u0))
    return out


SMALL = [(16, 18, 17), (21, 16, 25), (17, 23, 16), (30, 19, 22), (16, 16, 16)]


@pytest.fixture(scope="module")
def small_refs():
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    grids = _grids(SMALL, seed=40)
    refs = {}
    for scheme in oracle.SCHEMES:
        refs[scheme] = [oracle.run(scheme, "fundamental", oracle.Grid(nx, ny, nz, h, h, h, dt, eps), u0, 10)[0]
                        for (nx, ny, nz, eps, u0) in grids]
    return dict(h=h, dt=dt, grids=grids, refs=refs)


@pytest.mark.parametrize("prec", ["f64", "f32s64", "f32", "f32r"])
@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
def test_batch_vs_oracle_small(small_refs, scheme, prec):
    from paper_2011_14043_amd import BatchPlan
    c = small_refs
    dtype, solve = PREC[prec]
    print(f"[case] batch 5 grids {scheme}/{prec}", flush=True)
    plan = BatchPlan([(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in c["grids"]], c["dt"], c["h"],
                     c["h"], c["h"], scheme=scheme, dtype=dtype, solve_dtype=solve, refine=prec == "f32r")
    fields = [_fields(u0, dtype) for (*_, u0) in c["grids"]]
    plan.run(fields, 10)
    torch.cuda.synchronize()
    plan.close()
    for g, ((nx, ny, nz, eps, _), (E, H)) in enumerate(zip(c["grids"], fields)):
        got = [t.double().cpu().numpy() for t in E + H]
        gr = oracle.Grid(nx, ny, nz, c["h"], c["h"], c["h"], c["dt"], eps)
        err = oracle.yee.weighted_rel_l2(got, c["refs"][scheme][g], gr)
        assert err <= TOL[prec], (g, err)


@pytest.mark.parametrize("launch", ["fused", "yz-one-launch"])
@pytest.mark.parametrize("scheme", ["adi", "ss2"])
def test_batch_refined_16slot_vs_oracle(small_refs, scheme, launch):
    """Refined batched passes with 16-slot y/z chunks (512-thread blocks),
    the x lines fused into the same launch or a launch of their own."""
    from paper_2011_14043_amd import BatchPlan
    c = small_refs
    print(f"[case] batch 5 grids refined 16-slot {scheme} {launch}", flush=True)
    plan = BatchPlan([(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in c["grids"]], c["dt"], c["h"],
                     c["h"], c["h"], scheme=scheme, dtype=torch.float32, refine=True)
    plan.set_kernel_config(0, chunk=8, block_threads=0 if launch == "fused" else 256, remap=1)
    for ax in (1, 2):
        plan.set_kernel_config(ax, chunk=16, tile_x=16, block_threads=512, remap=1)
    fields = [_fields(u0, torch.float32) for (*_, u0) in c["grids"]]
    plan.run(fields, 10)
    torch.cuda.synchronize()
    plan.close()
    for g, ((nx, ny, nz, eps, _), (E, H)) in enumerate(zip(c["grids"], fields)):
        got = [t.double().cpu().numpy() for t in E + H]
        gr = oracle.Grid(nx, ny, nz, c["h"], c["h"], c["h"], c["dt"], eps)
        err = oracle.yee.weighted_rel_l2(got, c["refs"][scheme][g], gr)
        assert err <= TOL["f32r"], (g, err)


def test_batch_split_runs_and_configs_agree(small_refs):
    """12 steps in one call == 7 + 5 steps (input/output processing between
    calls is exact for ADI); every kernel configuration gives the same
    result to rounding; the graph is rebuilt after a configuration change."""
    from paper_2011_14043_amd import BatchPlan
    c = small_refs
    grids = [(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in c["grids"]]
    plan = BatchPlan(grids, c["dt"], c["h"], c["h"], c["h"], scheme="adi", dtype=torch.float64)
    f1 = [_fields(u0, torch.float64) for (*_, u0) in c["grids"]]
    f2 = [_fields(u0, torch.float64) for (*_, u0) in c["grids"]]
    plan.run(f1, 12)
    plan.run(f2, 7)
    plan.run(f2, 5)
    torch.cuda.synchronize()
    for (E1, H1), (E2, H2) in zip(f1, f2):
        for a, b in zip(E1 + H1, E2 + H2):
            torch.testing.assert_close(a, b, rtol=0, atol=1e-12 * float(a.abs().max()) + 1e-300)
    plan.set_kernel_config(0, chunk=16, block_threads=128)
    plan.set_kernel_config(1, chunk=8, tile_x=8, block_threads=512)
    f3 = [_fields(u0, torch.float64) for (*_, u0) in c["grids"]]
    plan.run(f3, 12)
    torch.cuda.synchronize()
    plan.close()
    for (E1, H1), (E3, H3) in zip(f1, f3):
        for a, b in zip(E1 + H1, E3 + H3):
            torch.testing.assert_close(a, b, rtol=0, atol=1e-12 * float(a.abs().max()) + 1e-300)


def test_batch_invalid():
    from paper_2011_14043_amd import BatchPlan, FdtdError, _lib
    import ctypes
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    L = _lib.lib()
    d = (_lib.FdtdDesc * 2)(_lib.FdtdDesc(16, 16, 16, dt, h, h, h, 0, 1, 0, None, None, 0),
                            _lib.FdtdDesc(16, 16, 16, dt, h, h, h, 0, 1, 0, None, None, 0))
    hnd = ctypes.c_void_p()
    assert L.fdtd_plan_batch(d, 2, None, ctypes.byref(hnd)) == -4       # conventional form
    d[1].form = 0
    assert L.fdtd_plan_batch(d, 2, None, ctypes.byref(hnd)) == -1       # mixed forms
    d[0].form = 0
    d[1].scheme = 1
    assert L.fdtd_plan_batch(d, 2, None, ctypes.byref(hnd)) == -1       # mixed schemes
    d[1].scheme = 0
    d[1].dtype = 3
    assert L.fdtd_plan_batch(d, 2, None, ctypes.byref(hnd)) == -1       # mixed precisions
    d[1].dtype = 0
    d[1].nx = 1
    assert L.fdtd_plan_batch(d, 2, None, ctypes.byref(hnd)) == -1       # invalid grid
    assert L.fdtd_plan_batch(d, 0, None, ctypes.byref(hnd)) == -1
    plan = BatchPlan([(16, 17, 18, None)], dt, h, h, h)
    E = [torch.zeros((19, 18, 17), device=DEV) for _ in range(3)]
    pe = (ctypes.c_void_p * 3)(*[t.data_ptr() for t in E])
    # single-grid entry points reject a batch plan
    assert L.fdtd_run(plan._h, pe, pe, 1, None, None, 1) == -1
    with pytest.raises(FdtdError, match="EINVAL"):
        plan.set_kernel_config(1, chunk=16, tile_x=24, block_threads=512)
    # x lines fused into the y/z launch: the batch default; single grids have no such launch
    assert plan.kernel_config(0)["block_threads"] == 0
    plan.close()
    from paper_2011_14043_amd import Plan
    sp = Plan(16, 16, 16, dt, h, h, h, eps_r=torch.ones(16, 16, 16))
    with pytest.raises(FdtdError, match="EINVAL"):
        sp.set_kernel_config(0, chunk=8, block_threads=0)
    sp.close()


# ---------------------------------------------------------------------------
# the 64-cavity workload
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def cavities():
    sizes = W.cavity_batch(64, seed=4)
    return _grids(sizes, seed=1000)


@pytest.fixture(scope="module")
def cavities_single_f64(cavities):
    """Each cavity alone through the single-grid FP64 path, 500 steps."""
    from paper_2011_14043_amd import Plan
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    out = []
    for (nx, ny, nz, eps, u0) in cavities:
        E, H = _fields(u0, torch.float64)
        p = Plan(nx, ny, nz, dt, h, h, h, scheme="adi", dtype=torch.float64, eps_r=torch.tensor(eps))
        p.run(E, H, 500)
        p.close()
        out.append([t.cpu().numpy() for t in E + H])
    return out


@pytest.mark.parametrize("prec,tol", [("f64", 1e-10), ("f32s64", 2e-5), ("f32", 1e-4), ("f32r", 2e-5)])
def test_64_cavities_vs_single_grid(cavities, cavities_single_f64, prec, tol):
    from paper_2011_14043_amd import BatchPlan
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    dtype, solve = PREC[prec]
    print(f"[case] 64 cavities U[16,96], 500 steps, {prec}", flush=True)
    plan = BatchPlan([(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in cavities], dt, h, h, h,
                     scheme="adi", dtype=dtype, solve_dtype=solve, refine=prec == "f32r")
    plan.autotune(2)
    fields = [_fields(u0, dtype) for (*_, u0) in cavities]
    plan.run(fields, 500)
    torch.cuda.synchronize()
    plan.close()
    worst = 0.0
    for g, ((nx, ny, nz, eps, _), (E, H)) in enumerate(zip(cavities, fields)):
        got = [t.double().cpu().numpy() for t in E + H]
        gr = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
        err = oracle.yee.weighted_rel_l2(got, cavities_single_f64[g], gr)
        worst = max(worst, err)
    print(f"  worst cavity rel-L2 vs single-grid FP64: {worst:.2e}", flush=True)
    assert worst <= tol


def _cavity_golden():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cavities_64.npz")
    if not os.path.exists(path):
        pytest.fail(f"missing fixture {path}: run tests/golden/make_cavities.py")
    return np.load(path)


def _sampled_err(fields, ref, g, tag, gr):
    """Energy-weighted relative L2 over the fixture's samples of cavity g
    (oracle grid gr for the weights)."""
    num = den = 0.0
    got = [t.double().cpu().numpy().ravel() for t in fields[0] + fields[1]]
    for k, c in enumerate(oracle.yee.COMPONENTS):
        idx = ref[f"idx_{c}_{g}"]
        want = ref[f"{tag}val_{c}_{g}"]
        wt = gr.material(c).ravel()[idx]
        num += float(np.sum(wt * (got[k][idx] - want) ** 2))
        den += float(np.sum(wt * want ** 2))
    return (num / den) ** 0.5


@pytest.mark.parametrize("prec,tol", [("f64", 1e-11), ("f32", 2e-5)])
def test_64_cavities_vs_oracle_50_steps(cavities, prec, tol):
    """Every cavity of the 64-cavity batch (one launch per sub-step, captured
    graphs, autotuned) after 50 steps against the oracle, on 512 seeded samples
    per component (fixture written by tests/golden/make_cavities.py from the
    oracle only); FP64, and FP32 as the library runs it at CFL 5 (refined
    solves).  Plus the whole-field energy against the oracle's."""
    from paper_2011_14043_amd import BatchPlan
    ref = _cavity_golden()
    assert int(ref["steps_all"]) == 50
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    dtype, solve = PREC[prec]
    sizes = [tuple(int(v) for v in sz) for sz in ref["sizes"]]
    assert sizes == [tuple(c[:3]) for c in cavities]
    print(f"[case] 64 cavities vs oracle, 50 steps, {prec}", flush=True)
    plan = BatchPlan([(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in cavities], dt, h, h, h,
                     scheme="adi", dtype=dtype, solve_dtype=solve)
    if prec == "f32":
        assert plan.refined
    plan.autotune(2)
    fields = [_fields(u0, dtype) for (*_, u0) in cavities]
    plan.run(fields, 50)
    torch.cuda.synchronize()
    plan.close()
    worst, worst_n = 0.0, 0.0
    for g, (nx, ny, nz, eps, _) in enumerate(cavities):
        gr = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
        err = _sampled_err(fields[g], ref, g, "", gr)
        got = [t.double().cpu().numpy() for t in fields[g][0] + fields[g][1]]
        nerr = abs(oracle.yee.energy(got, gr) - float(ref[f"norm2_{g}"])) / float(ref[f"norm2_{g}"])
        worst, worst_n = max(worst, err), max(worst_n, nerr)
        assert err <= tol, (g, err)
        assert nerr <= tol, (g, nerr)
    print(f"  worst cavity sampled rel-L2 {worst:.2e}, energy {worst_n:.2e}", flush=True)


def test_64_cavities_smallest_vs_oracle(cavities):
    """The four smallest cavities of the batch after 500 steps (FP64 batch)
    against the oracle (fixture samples)."""
    from paper_2011_14043_amd import BatchPlan
    ref = _cavity_golden()
    assert int(ref["steps_small"]) == 500
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    order = sorted(range(len(cavities)), key=lambda g: np.prod(cavities[g][:3]))[:4]
    assert sorted(order) == sorted(int(v) for v in ref["small"])
    plan = BatchPlan([(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in cavities], dt, h, h, h,
                     scheme="adi", dtype=torch.float64)
    fields = [_fields(u0, torch.float64) for (*_, u0) in cavities]
    plan.run(fields, 500)
    torch.cuda.synchronize()
    plan.close()
    for g in order:
        nx, ny, nz, eps, u0 = cavities[g]
        err = _sampled_err(fields[g], ref, g, "s", oracle.Grid(nx, ny, nz, h, h, h, dt, eps))
        print(f"  cavity {g} {nx}x{ny}x{nz}: sampled rel-L2 vs oracle {err:.2e}", flush=True)
        assert err <= 1e-10


@pytest.mark.parametrize("scheme", ["lod1", "adi"])
def test_graph_replays_match_eager_single_grids(small_refs, scheme):
    """A batch run replays the captured eight-step graph floor(steps / 8) times
    (ADI: of steps - 1, the last step being special) and launches the rest
    directly.  Calls of 9 steps (LOD1: one replay and one direct step; ADI:
    one replay and the last step), with eager input/output kernels and a
    synchronization between them: after each call the batch equals the
    single-grid plans stepped eagerly."""
    from paper_2011_14043_amd import BatchPlan, Plan
    c = small_refs
    grids = [(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in c["grids"]]
    bp = BatchPlan(grids, c["dt"], c["h"], c["h"], c["h"], scheme=scheme, dtype=torch.float64)
    fb = [_fields(u0, torch.float64) for (*_, u0) in c["grids"]]
    singles = [Plan(nx, ny, nz, c["dt"], c["h"], c["h"], c["h"], scheme=scheme, dtype=torch.float64, eps_r=e)
               for (nx, ny, nz, e) in grids]
    fs = [_fields(u0, torch.float64) for (*_, u0) in c["grids"]]
    for call in range(4):
        bp.run(fb, 9)
        for p, (E, H) in zip(singles, fs):
            p.run(E, H, 9)
        torch.cuda.synchronize()
        for (E1, H1), (E2, H2) in zip(fb, fs):
            for a, b in zip(E1 + H1, E2 + H2):
                torch.testing.assert_close(a, b, rtol=0, atol=1e-12 * float(b.abs().max()) + 1e-300)
    bp.close()
    for p in singles:
        p.close()


@pytest.mark.parametrize("launch", ["fused", "yz-one-launch", "yz-separate"])
@pytest.mark.parametrize("refine", [False, True], ids=["f32", "f32r"])
@pytest.mark.parametrize("scheme", ["adi", "lod1"])
def test_batch_bitwise_equals_single_grids(scheme, refine, launch):
    """Grids whose chunk counts are the same powers of two in both paths run
    the same arithmetic: the batch (graph replays; a sub-step as one launch
    with the x lines fused, or the x pass alone and the y and z passes in one
    launch, or one launch each) equals the single-grid plans (eager) bit for
    bit, over 17 steps (two replays of the eight-step graph)."""
    from paper_2011_14043_amd import BatchPlan, Plan
    split = launch == "yz-separate"
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    grids = _grids([(32, 64, 32), (64, 32, 64)], seed=300)

    def configure(p, batch=False):
        p.set_kernel_config(0, chunk=8, block_threads=0 if (batch and launch == "fused") else 256, remap=1)
        p.set_kernel_config(1, chunk=8, tile_x=16, block_threads=1024, remap=1)
        if split:
            p.set_kernel_config(2, chunk=16, tile_x=16, block_threads=512, remap=1)
        else:
            p.set_kernel_config(2, chunk=8, tile_x=16, block_threads=1024, remap=1)

    bp = BatchPlan([(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in grids], dt, h, h, h,
                   scheme=scheme, dtype=torch.float32, refine=refine)
    configure(bp, batch=True)
    assert bp.kernel_config(0)["block_threads"] == (0 if launch == "fused" else 256)
    fb = [_fields(u0, torch.float32) for (*_, u0) in grids]
    bp.run(fb, 17)
    torch.cuda.synchronize()
    bp.close()
    for (nx, ny, nz, eps, u0), (Eb, Hb) in zip(grids, fb):
        p = Plan(nx, ny, nz, dt, h, h, h, scheme=scheme, dtype=torch.float32, eps_r=torch.tensor(eps), refine=refine)
        configure(p)
        E, H = _fields(u0, torch.float32)
        p.run(E, H, 17)
        torch.cuda.synchronize()
        p.close()
        for a, b in zip(E + H, Eb + Hb):
            assert torch.equal(a, b)


@pytest.mark.parametrize("prec,yz", [("f32", (8, 16, 1024)), ("f32", (8, 32, 512)), ("f32", (16, 32, 1024)),
                                     ("f32", (16, 16, 512)), ("f32r", (8, 16, 1024)), ("f64", (8, 8, 512)),
                                     ("f64", (8, 16, 1024)), ("f64", (16, 16, 512))])
def test_batch_fused_bitwise_equals_separate(prec, yz):
    """One launch per sub-step (x-line blocks inside the y/z launch, in blocks
    of its size) against the x pass as a launch of its own: the same line
    solves in other blocks, so bit-for-bit equal, over 12 uneven cavities and
    17 steps, for every y/z configuration the fused launch is built for."""
    from paper_2011_14043_amd import BatchPlan
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    dtype = torch.float64 if prec == "f64" else torch.float32
    grids = _grids(W.cavity_batch(12, seed=7), seed=500)
    print(f"[case] fused vs separate {prec} yz={yz}", flush=True)
    out = []
    for fused in (False, True):
        bp = BatchPlan([(nx, ny, nz, torch.tensor(eps)) for (nx, ny, nz, eps, _) in grids], dt, h, h, h,
                       dtype=dtype, refine=prec == "f32r")
        bp.set_kernel_config(0, chunk=8, block_threads=0 if fused else 256, remap=1)
        for ax in (1, 2):
            bp.set_kernel_config(ax, chunk=yz[0], tile_x=yz[1], block_threads=yz[2], remap=1)
        f = [_fields(u0, dtype) for (*_, u0) in grids]
        bp.run(f, 17)
        torch.cuda.synchronize()
        bp.close()
        out.append(f)
    for (Ea, Ha), (Eb, Hb) in zip(*out):
        for a, b in zip(Ea + Ha, Eb + Hb):
            assert torch.equal(a, b)
