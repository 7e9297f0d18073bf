"""Captured step graphs of single-grid runs (fdtd_set_graph): replays give the
fields of direct launches bit for bit, over several calls in a row with eager
work and synchronizations between them, across a change of the source cell
and of a kernel configuration (both re-capture the graph), for every scheme
in both forms and every precision; and the argument checks."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PREC = {"f32": (torch.float32, torch.float32, None), "f32p": (torch.float32, torch.float32, False),
        "f64": (torch.float64, torch.float64, None), "f32s64": (torch.float32, torch.float64, None)}


def _plan(c, scheme, form, prec, graph):
    from paper_2011_14043_amd import Plan
    dtype, solve, refine = PREC[prec]
    p = Plan(c["nx"], c["ny"], c["nz"], c["dt"], c["h"], c["h"], c["h"], scheme=scheme, form=form, dtype=dtype,
             solve_dtype=solve, eps_r=torch.tensor(c["eps"]), refine=refine)
    p.set_graph(graph)
    return p


@pytest.fixture(scope="module")
def case():
    nx, ny, nz, h = 37, 30, 45, 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    return dict(nx=nx, ny=ny, nz=nz, h=h, dt=dt, eps=W.random_box_eps(nx, ny, nz, seed=21, nboxes=8),
                u0=W.random_fields(nx, ny, nz, seed=22))


@pytest.mark.parametrize("scheme,form", [("adi", "fundamental"), ("adi", "conventional"), ("lod1", "fundamental"),
                                         ("ss2", "fundamental"), ("lod2", "fundamental"), ("lod2", "conventional"),
                                         ("dyakonov", "fundamental")])
@pytest.mark.parametrize("prec,graph", [("f32", 8), ("f32p", 3), ("f64", 8), ("f32s64", 5)])
def test_graph_replays_equal_direct_launches(case, scheme, form, prec, graph):
    from paper_2011_14043_amd import Source
    print(f"[case] graphs {scheme}/{form} {prec} steps per graph {graph}", flush=True)
    dtype = PREC[prec][0]
    pg = _plan(case, scheme, form, prec, graph)
    pe = _plan(case, scheme, form, prec, 0)
    fields = []
    for _ in range(2):
        fields.append(([torch.tensor(a, dtype=dtype, device=DEV) for a in case["u0"][:3]],
                       [torch.tensor(a, dtype=dtype, device=DEV) for a in case["u0"][3:]]))
    dt = case["dt"]
    src_a = Source(12, 9, 20, f0=1 / (14 * dt), tau=4 * dt, t0=6 * dt, amp=1e11)
    src_b = Source(25, 17, 30, f0=1 / (10 * dt), tau=3 * dt, t0=20 * dt, amp=5e10)
    calls = [(17, src_a), (1, src_a), (9, src_a), (24, src_b), (8, None), ("cfg", None), (33, src_b)]
    for m, (n, src) in enumerate(calls):
        if n == "cfg":
            # a kernel configuration change between calls re-captures the graph
            for p in (pg, pe):
                p.set_kernel_config(0, chunk=8, block_threads=64, remap=0)
            continue
        for p, (E, H) in zip((pg, pe), fields):
            p.run(E, H, n, source=src)
        # eager work and a synchronization between the calls
        junk = torch.ones(1000, device=DEV).cumsum(0)
        torch.cuda.synchronize()
        assert float(junk[-1]) == 1000.0
        (Eg, Hg), (Ee, He) = fields
        for a, b in zip(Eg + Hg, Ee + He):
            assert torch.equal(a, b), f"call {m} ({n} steps) differs"
        assert all(bool(torch.isfinite(t).all()) for t in Eg + Hg)
    pg.close()
    pe.close()


def test_set_graph_arguments():
    from paper_2011_14043_amd import BatchPlan, FdtdError, Plan
    h = 1e-3
    dt = W.yee_dt(h, h, h, 2.0)
    p = Plan(8, 9, 10, dt, h, h, h)
    for bad in (-1, 65):
        with pytest.raises(FdtdError, match="EINVAL"):
            p.set_graph(bad)
    p.set_graph(64)
    p.set_graph(0)
    p.close()
    bp = BatchPlan([(8, 9, 10, None)], dt, h, h, h)
    with pytest.raises(FdtdError, match="EINVAL"):
        bp.set_graph(4)
    bp.close()
    cn = Plan(8, 9, 10, dt, h, h, h, scheme="crank_nicolson", dtype=torch.float64)
    with pytest.raises(FdtdError, match="EUNSUPPORTED"):
        cn.set_graph(4)
    cn.close()


def test_graph_energy_trace_runs_directly(case):
    """A run with an energy trace does not use the graph and still equals the
    graph-replayed run of the same steps."""
    dtype = torch.float32
    pg = _plan(case, "adi", "fundamental", "f32", 8)
    fields = []
    for _ in range(2):
        fields.append(([torch.tensor(a, dtype=dtype, device=DEV) for a in case["u0"][:3]],
                       [torch.tensor(a, dtype=dtype, device=DEV) for a in case["u0"][3:]]))
    pg.run(*fields[0], 20)
    tr = pg.run(*fields[1], 20, energy_every=5)
    torch.cuda.synchronize()
    assert len(tr) == 5 and np.all(np.isfinite(tr))
    for a, b in zip(fields[0][0] + fields[0][1], fields[1][0] + fields[1][1]):
        assert torch.equal(a, b)
    pg.close()
