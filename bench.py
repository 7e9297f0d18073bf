#!/usr/bin/env python3
"""Benchmark: Mcell-updates/s per full time step of the implicit FDTD schemes on one GPU.

Workload (the 512^3 configuration): 512^3 cells, 1 mm cubic cells, PEC box,
eps_r piecewise constant over 32 seeded random boxes U[1,12], mu_r = 1, zero
initial fields, an Ez modulated-Gaussian point source (10 GHz) at a seeded
interior cell, CFL number 5.  Headline: fundamental ADI, FP32 fields.
Also measured on the same workload: conventional ADI, FP64, the FP32-storage /
FP64-solve variant, and the other fundamental schemes.

One "step" = one full time step (every line pass of the scheme).  The timed
region is plan.run(K steps) bracketed by torch.cuda.synchronize(), inputs
already resident in HBM; it includes the scheme's input/output processing.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s per step, fundamental vs conventional ADI, FP32 vs FP64, %HBM"
HBM_PEAK_GBS = 8000.0


# HBM traffic of the dominant kernel from rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE in KiB per dispatch, median over its y and z dispatches;
# calibration factors from a 1 GiB device copy).  Valid only for the kernel
# sources whose hash is recorded, the profiled y/z configuration and the same
# refinement; otherwise the bench reports traffic = null.
PROFILED = {
    "kernel_hash": "2fefdd7333065000",
    "config": [16, 16, 512, 1],                              # chunk, tile_x, block_threads, remap (y and z)
    "refined": True,
    "fetch_kib": 595772.6,                                   # median over the y and z dispatches
    "write_kib": 1068013.2,
    "fetch_factor": 1048576.0 / 524299.5,                    # 1 GiB copy: FETCH_SIZE 524299.5 KiB
    "write_factor": 1.0,                                     # 1 GiB copy: WRITE_SIZE 1048576 KiB
    "profile": "profiles/pass_kernels_adi_fundamental_f32_512cube.md",
}


def kernel_hash():
    import hashlib
    hsh = hashlib.sha256()
    for f in ("pass_kernels.hpp", "line_solver.hpp"):
        with open(os.path.join(ROOT, "paper_2011_14043_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    return hsh.hexdigest()[:16]


def profiled_traffic(cfg_y, cfg_z, refined):
    pr = PROFILED
    if not pr or pr["kernel_hash"] != kernel_hash() or pr.get("refined") != refined:
        return None
    want = pr["config"]
    for c in (cfg_y, cfg_z):
        if [c["chunk"], c["tile_x"], c["block_threads"], c["remap"]] != want:
            return None
    return pr["fetch_kib"] * 1024 * pr["fetch_factor"] + pr["write_kib"] * 1024 * pr["write_factor"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(n, seed_eps=2, seed_src=2):
    import numpy as np
    import workloads as W
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    eps = W.random_box_eps(n, n, n, seed=seed_eps, nboxes=32)
    ci = W.interior_cell(n, n, n, seed=seed_src, margin=8)
    return h, dt, eps, ci


def bytes_per_slot(prec, conv_adi=False, material_index=False):
    """Bytes one line pass moves per (E, H) slot: read E and H (and, for
    conventional ADI, the two cross-coupled arrays), read the medium, write E
    and H.  Algorithmic (the default): the medium is the FP32 eps_r, the
    per-unit figure the roofline is priced on (20 B FP32, 36 B FP64, 28 / 52 B
    conventional ADI).  material_index: the plan's actual medium read, a
    one-byte material index (this workload has 33 materials)."""
    w = 8 if prec == "f64" else 4
    words = 6 if conv_adi else 4
    return words * w + (1 if material_index else 4)


def order4_moved_bytes_per_slot(prec, material_index=True):
    """Bytes a fourth-order line pass moves per slot, averaged over a step's
    four y/z and two x passes: the forward sweep reads E, H and the medium and
    writes the substituted right side y, the backward sweep reads y and the
    medium again with E and H and writes E and H; the factorization state (6
    solve words) is written and read back once per segment of K = 8 rows.  An
    x pass runs on a transposed copy of its pair: E and H are read and written
    once more on the way in and once more on the way out.  With the one-byte
    material index: 50.7 B FP32, 99.3 B FP64, 64.7 B FP32 fields with FP64
    solves (f32s64, and f32: order-4 FDTD_F32 plans solve in FP64)."""
    t = 8 if prec == "f64" else 4
    sv = 4 if prec == "f32p" else 8
    med = 1 if material_index else 4
    k = 8
    yz = 6 * t + 2 * sv + 12 * sv / k + 2 * med
    x = yz + 8 * t
    return (4 * yz + 2 * x) / 6


def run_order4(n, precs, steps, warmup, inputs, refs):
    """Fundamental ADI with the fourth-order differences on the n^3 workload:
    per precision the run, the per-pass times and the fraction of 8 TB/s on
    the scope's bytes (20 / 36 B per slot) and on the bytes the passes move.
    f32p: plain FP32 solves; f32: FDTD_F32, which solves in FP64 at order 4."""
    rows = []
    for prec in precs:
        r = run_variant(n, "adi", "fundamental", prec, steps, warmup, inputs, tune=False, refs=refs, order=4)
        r["solves"] = "fp32" if prec == "f32p" else "fp64"
        main = r["main_ms"] / steps
        npass = 6
        r["main_ms_per_step"] = main
        r["moved_bytes_per_slot"] = order4_moved_bytes_per_slot(prec)
        r["hbm_frac_moved_bytes_main"] = npass * pass_nodes(n) * r["moved_bytes_per_slot"] / (main * 1e-3) / 1e9 \
            / HBM_PEAK_GBS
        r["hbm_frac_alg_main"] = npass * pass_nodes(n) * bytes_per_slot(prec) / (main * 1e-3) / 1e9 / HBM_PEAK_GBS
        rows.append(r)
    return rows


def pass_nodes(n):
    # every pass of a cubic n^3 grid covers n * (n-1) lines of n slots
    return n * (n - 1) * n


# HIP events bracket every line pass of every TIMING_EVERY-th step of a timed
# run (each event pair costs a few microseconds between launches; on every
# step they slow the 512^3 step by 1.5 %).
TIMING_EVERY = 8


# precision keys: f32 = FP32 fields and solves as the library chooses (refined
# wherever refined passes are built), f32r = refined, f32p = plain FP32
# solves, f32s64 = FP32 fields with FP64 solves, f64
REFINE = {"f32r": True, "f32p": False}


class Fp64Refs:
    """FP64 GPU runs of the same workload (fundamental form of each scheme;
    the FP64 path matches the FP64 oracle to 1e-11), the reference of the
    relative L2 error reported for every result.  Kept per (n, scheme, dt,
    warmup, steps); cleared when the grid size changes."""

    def __init__(self):
        self.cache = {}
        self.n = None
        self.diff_plan = None

    def _clear(self):
        if self.diff_plan is not None:
            self.diff_plan.close()
        self.cache, self.diff_plan = {}, None

    def get(self, n, scheme, steps, warmup, inputs, order=2):
        import torch
        from paper_2011_14043_amd import Plan, Source
        if n != self.n:
            self._clear()
            self.n = n
        h, dt, eps, ci = inputs
        base = {"dyakonov": "adi", "douglas_gunn": "adi"}.get(scheme, scheme)
        key = (base, dt, warmup, steps, order)
        if key not in self.cache:
            dev = torch.device("cuda", 0)
            shape = (n + 1, n + 1, n + 1)
            E = [torch.zeros(shape, dtype=torch.float64, device=dev) for _ in range(3)]
            H = [torch.zeros(shape, dtype=torch.float64, device=dev) for _ in range(3)]
            src = Source(*ci, f0=10e9, tau=0.1e-9, t0=0.4e-9, amp=1.0e10)
            plan = Plan(n, n, n, dt, h, h, h, scheme=base, form="fundamental", dtype=torch.float64,
                        eps_r=torch.from_numpy(eps))
            if order != 2:
                plan.set_order(order)
            if warmup:
                plan.run(E, H, warmup, source=src)
            plan.set_step(0)
            plan.run(E, H, steps, source=src)
            torch.cuda.synchronize()
            if self.diff_plan is None:
                self.diff_plan = plan
            else:
                plan.close()
            self.cache[key] = (E, H)
        return self.cache[key]

    def rel_l2(self, n, scheme, steps, warmup, inputs, E, H, order=2):
        """Energy-weighted relative L2 distance (fdtd_diff_norm, FP64 on the
        device) of E, H from the FP64 reference run."""
        import math
        import torch
        Er, Hr = self.get(n, scheme, steps, warmup, inputs, order)
        Ed = [t.to(torch.float64) for t in E]
        Hd = [t.to(torch.float64) for t in H]
        num, den = self.diff_plan.diff_norm(Ed, Hd, Er, Hr)
        del Ed, Hd
        return math.sqrt(num / den) if den > 0 else None

    def close(self):
        self._clear()


def run_variant(n, scheme, form, prec, steps, warmup, inputs, per_launch=TIMING_EVERY, tune=True, tune_reps=5,
                refs=None, order=2):
    import torch
    from paper_2011_14043_amd import Plan, Source
    h, dt, eps, ci = inputs
    dtype = torch.float64 if prec == "f64" else torch.float32
    solve = torch.float64 if prec in ("f64", "f32s64") else torch.float32
    dev = torch.device("cuda", 0)
    shape = (n + 1, n + 1, n + 1)
    E = [torch.zeros(shape, dtype=dtype, device=dev) for _ in range(3)]
    H = [torch.zeros(shape, dtype=dtype, device=dev) for _ in range(3)]
    src = Source(*ci, f0=10e9, tau=0.1e-9, t0=0.4e-9, amp=1.0e10)
    plan = Plan(n, n, n, dt, h, h, h, scheme=scheme, form=form, dtype=dtype, solve_dtype=solve,
                eps_r=torch.from_numpy(eps), refine=REFINE.get(prec))
    if order != 2:
        plan.set_order(order)
    refined = plan.refined
    if tune:
        plan.autotune(tune_reps)
    cfg = [plan.kernel_config(ax) for ax in range(3)]
    if warmup:
        plan.run(E, H, warmup, source=src)
    torch.cuda.synchronize()
    plan.set_timing(per_launch)
    plan.set_step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(E, H, steps, source=src)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = plan.last_timing()
    finite = all(bool(torch.isfinite(t).all()) for t in E + H)
    plan.close()
    ms = (t1 - t0) * 1e3 / steps
    cells = n ** 3
    mcells = cells / (ms * 1e-3) / 1e6
    npass = 9 if scheme == "ss2" else 6
    conv_adi = scheme == "adi" and form == "conventional"
    alg_bytes_step = npass * pass_nodes(n) * bytes_per_slot(prec, conv_adi)          # line passes only
    act_bytes_step = npass * pass_nodes(n) * bytes_per_slot(prec, conv_adi, material_index=True)
    out = dict(scheme=scheme, form=form, prec=prec, refined=refined, ms_per_step=ms, mcells_per_s=mcells,
               alg_bytes_per_step=alg_bytes_step,
               hbm_frac_alg=alg_bytes_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               hbm_frac_actual_bytes=act_bytes_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, main_ms=tm["main_ms"],
               yz_ms_avg=tm["yz_ms_avg"], x_ms_avg=tm["x_ms_avg"], yz_launches=tm["yz_launches"],
               x_launches=tm["x_launches"], finite=finite, kernel_config=cfg)
    if order != 2:
        out["order"] = order
    if refs is not None:
        out["rel_l2_vs_gpu_fp64"] = refs.rel_l2(n, scheme, steps, warmup, inputs, E, H, order)
    del E, H
    torch.cuda.empty_cache()
    log(json.dumps(out))
    return out


def run_batch(steps, warmup, prec="f32", singles=True):
    """64 independent PEC cavities, sizes U[16, 96] per axis (seed 4), random-box
    eps_r and N(0,1) fields per cavity, fundamental ADI, CFL 5: one launch per
    line pass over the cavities of a group (groups that fit the MALL), captured
    graphs of eight steps.  Beside it, the same cavities stepped one after the
    other through single-grid plans."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2011_14043_amd import BatchPlan
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    sizes = W.cavity_batch(64, seed=4)
    dtype = torch.float64 if prec == "f64" else torch.float32
    solve = torch.float64 if prec in ("f64", "f32s64") else torch.float32
    dev = torch.device("cuda", 0)
    grids, fields = [], []
    for g, (nx, ny, nz) in enumerate(sizes):
        eps = W.random_box_eps(nx, ny, nz, seed=1000 + g, nboxes=32)
        u0 = W.random_fields(nx, ny, nz, seed=1100 + g)
        grids.append((nx, ny, nz, torch.from_numpy(eps)))
        fields.append(([torch.tensor(a, dtype=dtype, device=dev) for a in u0[:3]],
                       [torch.tensor(a, dtype=dtype, device=dev) for a in u0[3:]]))
    plan = BatchPlan(grids, dt, h, h, h, scheme="adi", dtype=dtype, solve_dtype=solve, refine=REFINE.get(prec))
    refined = plan.refined
    plan.autotune(3)
    cfg = [plan.kernel_config(ax) for ax in range(3)]
    plan.run(fields, warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run(fields, steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = plan.last_timing()
    finite = all(bool(torch.isfinite(t).all()) for E, H in fields for t in E + H)
    plan.close()
    cells = int(sum(np.prod(sz) for sz in sizes))
    ms = (t1 - t0) * 1e3 / steps
    main_ms = tm["main_ms"] / steps
    out = dict(workload="64 cavities U[16,96]^3, fundamental ADI, CFL 5", prec=prec, refined=refined, cells=cells,
               steps=steps, ms_per_step=ms, mcells_per_s=cells / (ms * 1e-3) / 1e6, main_ms_per_step=main_ms,
               hbm_frac_alg=6 * cells * bytes_per_slot(prec) / (main_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
               kernel_config=cfg, finite=finite)
    if singles:
        # the same cavities one after the other, each its own (autotuned) single-grid plan
        from paper_2011_14043_amd import Plan
        plans = []
        for (nx, ny, nz, eps) in grids:
            sp = Plan(nx, ny, nz, dt, h, h, h, scheme="adi", dtype=dtype, solve_dtype=solve, eps_r=eps,
                      refine=REFINE.get(prec))
            sp.autotune(1)
            plans.append(sp)
        for sp, (E, H) in zip(plans, fields):
            sp.run(E, H, max(warmup, 17))   # long enough to capture the plans' step graphs
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for sp, (E, H) in zip(plans, fields):
            sp.run(E, H, steps)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for sp in plans:
            sp.close()
        seq_ms = (t3 - t2) * 1e3 / steps
        out["sequential_single_ms_per_step"] = seq_ms
        out["sequential_single_mcells_per_s"] = cells / (seq_ms * 1e-3) / 1e6
    log(json.dumps(out))
    return out


def run_adjoint(prec="f32", steps=500, ckpt=50):
    """dJ/d eps_r of the probe energy over a 64 x 64 x 16 design box in a
    128 x 128 x 64 PEC box, 500 steps at CFL 5, checkpoints every 50 steps."""
    import torch
    import workloads as W
    from paper_2011_14043_amd import Plan, Source
    p = W.design_problem(seed=5)
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    dtype = torch.float64 if prec == "f64" else torch.float32
    solve = torch.float64 if prec in ("f64", "f32s64") else torch.float32
    dev = torch.device("cuda", 0)
    shape = (p["nz"] + 1, p["ny"] + 1, p["nx"] + 1)
    E = [torch.zeros(shape, dtype=dtype, device=dev) for _ in range(3)]
    H = [torch.zeros(shape, dtype=dtype, device=dev) for _ in range(3)]
    plan = Plan(p["nx"], p["ny"], p["nz"], dt, h, h, h, dtype=dtype, solve_dtype=solve,
                eps_r=torch.from_numpy(p["eps"]))
    plan.autotune(3)
    src = Source(*p["src"])
    plan.grad_eps(E, H, 20, p["probe"], src, p["design_box"], ckpt)      # warm-up, allocations
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J0, _ = plan.grad_eps(E, H, steps, p["probe"], src)
    t1 = time.perf_counter()
    J, g = plan.grad_eps(E, H, steps, p["probe"], src, p["design_box"], ckpt)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    plan.close()
    cells = p["nx"] * p["ny"] * p["nz"]
    out = dict(workload="adjoint dJ/deps_r, 128x128x64, design box 64x64x16, 500 steps, CFL 5, ckpt 50",
               prec=prec, forward_ms=(t1 - t0) * 1e3, gradient_ms=(t2 - t1) * 1e3,
               gradient_over_forward=(t2 - t1) / (t1 - t0),
               forward_mcells_per_s=cells * steps / (t1 - t0) / 1e6, J=J, finite=bool(torch.isfinite(g).all()))
    log(json.dumps(out))
    return out


def run_graphs(steps=500, warmup=20):
    """Forward runs of the 128 x 128 x 64 design workload's grid and source
    (FP32, CFL 5) with the main steps replayed from captured graphs of 8
    steps (the default) and with every pass launched directly."""
    import torch
    import workloads as W
    from paper_2011_14043_amd import Plan, Source
    p = W.design_problem(seed=5)
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    shape = (p["nz"] + 1, p["ny"] + 1, p["nx"] + 1)
    out = {"workload": "128x128x64, design-box eps_r, Ez source, CFL 5, fundamental ADI, FP32", "steps": steps}
    for graph in (8, 0):
        E = [torch.zeros(shape, dtype=torch.float32, device="cuda") for _ in range(3)]
        H = [torch.zeros(shape, dtype=torch.float32, device="cuda") for _ in range(3)]
        plan = Plan(p["nx"], p["ny"], p["nz"], dt, h, h, h, dtype=torch.float32, eps_r=torch.from_numpy(p["eps"]))
        plan.autotune(3)
        plan.set_graph(graph)
        src = Source(*p["src"])
        plan.run(E, H, warmup, source=src)
        torch.cuda.synchronize()
        plan.set_step(0)
        t0 = time.perf_counter()
        plan.run(E, H, steps, source=src)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        key = "graphs" if graph else "direct"
        out[f"{key}_ms_per_step"] = ms
        out[f"{key}_mcells_per_s"] = p["nx"] * p["ny"] * p["nz"] / (ms * 1e-3) / 1e6
        plan.close()
    out["direct_over_graphs"] = out["direct_ms_per_step"] / out["graphs_ms_per_step"]
    log(json.dumps(out))
    return out


def run_cn(n=256, steps=10, tol=1e-12):
    """Crank-Nicolson without factorization (FP64, one CG solve per step), in
    fundamental and classical form, against fundamental ADI (FP64) on the same
    n^3 random-box medium at CFL 5, from the same seeded N(0,1) fields."""
    import torch
    from paper_2011_14043_amd import Plan
    h, dt, eps, _ = make_inputs(n)
    dev = torch.device("cuda", 0)
    shape = (n + 1, n + 1, n + 1)
    out = dict(workload=f"{n}^3 random-box eps_r, CFL 5, N(0,1) initial fields, no source", prec="f64", steps=steps,
               cg_tol=tol)
    for scheme, form, key in (("crank_nicolson", "fundamental", "cn"), ("crank_nicolson", "conventional", "cn_conv"),
                              ("adi", "fundamental", "adi")):
        gen = torch.Generator(device=dev).manual_seed(11)
        E = [torch.empty(shape, dtype=torch.float64, device=dev).normal_(generator=gen) for _ in range(3)]
        H = [torch.empty(shape, dtype=torch.float64, device=dev).normal_(generator=gen) for _ in range(3)]
        plan = Plan(n, n, n, dt, h, h, h, scheme=scheme, form=form, dtype=torch.float64, eps_r=torch.from_numpy(eps))
        if scheme == "adi":
            plan.autotune(3)
        else:
            plan.set_cg(tol, 5000)
        plan.run(E, H, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.run(E, H, steps)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        out[f"{key}_ms_per_step"] = ms
        out[f"{key}_mcells_per_s"] = n ** 3 / (ms * 1e-3) / 1e6
        if scheme == "crank_nicolson":
            st = plan.last_cg()
            it = st["iterations"] / steps
            out[f"{key}_cg_iterations_per_step"] = it
            out[f"{key}_cg_rel_residual_max"] = st["rel_residual"]
            # algorithmic bytes of one CG iteration: 276 B per node in FP64
            # (apply: p, eps -> q; update: x, p, r, q, eps -> x, r; direction:
            # r, p, eps -> p), kernels over all (n+1)^3 nodes
            out[f"{key}_cg_iteration_gbs"] = 276 * (n + 1) ** 3 * it / (ms * 1e-3) / 1e9
        out[f"{key}_finite"] = all(bool(torch.isfinite(t).all()) for t in E + H)
        plan.close()
        del E, H
        torch.cuda.empty_cache()
    out["cn_over_adi"] = out["cn_ms_per_step"] / out["adi_ms_per_step"]
    out["cn_conventional_over_fundamental"] = out["cn_conv_ms_per_step"] / out["cn_ms_per_step"]
    log(json.dumps(out))
    return out


def _pinned_one_core():
    """Context: run on one core of the allowed set (sched_setaffinity), one BLAS thread."""
    import contextlib
    from threadpoolctl import threadpool_limits

    @contextlib.contextmanager
    def ctx():
        old = os.sched_getaffinity(0) if hasattr(os, "sched_getaffinity") else None
        core = min(old) if old else None
        try:
            if core is not None:
                os.sched_setaffinity(0, {core})
            with threadpool_limits(limits=1):
                yield core
        finally:
            if old is not None:
                os.sched_setaffinity(0, old)
    return ctx()


def cpu_baseline(n=256, steps=3):
    """The FP64 oracle on the host, one thread pinned to one core, on bounded
    samples of the workloads: the headline sample (fundamental ADI on n^3
    cells of the 512^3 workload's medium and source, `steps` steps) and, as
    detail, both forms of ADI on the 24^3 cavity (200 steps, full), the 128^3
    precision-sweep grid (2 steps, with the time 1000 steps would take) and
    the conventional form of the headline sample."""
    import numpy as np
    import oracle
    import workloads as W
    from oracle.source import Source as OSource
    h, dt, eps, ci = make_inputs(n)
    g = oracle.Grid(n, n, n, h, h, h, dt, eps)
    detail = []

    def timed(label, scheme, form, grid, u0, nsteps, src, cells, full_steps=None):
        t0 = time.perf_counter()
        oracle.run(scheme, form, grid, u0, nsteps, src)
        t1 = time.perf_counter()
        row = {"sample": label, "scheme": scheme, "form": form, "cells": cells, "steps": nsteps,
               "seconds": t1 - t0, "mcells_per_s": cells * nsteps / (t1 - t0) / 1e6}
        if full_steps:
            row["seconds_for_%d_steps" % full_steps] = (t1 - t0) / nsteps * full_steps
        detail.append(row)
        return row

    with _pinned_one_core() as core:
        head = timed(f"{n}^3 random boxes + source", "adi", "fundamental", g, W.zero_fields(n, n, n), steps,
                     OSource(*ci), n ** 3)
        timed(f"{n}^3 random boxes + source", "adi", "conventional", g, W.zero_fields(n, n, n), 2, OSource(*ci),
              n ** 3)
        h1 = 1e-3
        g1 = oracle.Grid(24, 24, 24, h1, h1, h1, W.yee_dt(h1, h1, h1, 4.0))
        u1 = W.random_fields(24, 24, 24, seed=1)
        for form in ("fundamental", "conventional"):
            timed("24^3 vacuum cavity, CFL 4 (full)", "adi", form, g1, u1, 200, None, 24 ** 3)
        g3 = oracle.Grid(128, 128, 128, h1, h1, h1, W.yee_dt(h1, h1, h1, 10.0),
                         W.random_box_eps(128, 128, 128, seed=2, nboxes=32))
        u3 = W.random_fields(128, 128, 128, seed=3)
        for form in ("fundamental", "conventional"):
            timed("128^3 precision sweep, CFL 10", "adi", form, g3, u3, 2, None, 128 ** 3, full_steps=1000)
    return {"value": head["mcells_per_s"], "unit": "Mcell/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy oracle, fundamental ADI, {n}^3 cells of the same random-box/source "
                      f"workload, {steps} step(s), one thread pinned to core {core} ({head['seconds']:.1f} s)",
            "host": host_info(), "detail": detail}


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": os.cpu_count()}


def cpu_schemes(n=96, steps=2):
    """The FP64 oracle, single thread, per scheme and form on n^3 cells of the
    random-box workload with its source (the D'Yakonov and Douglas-Gunn
    splittings from N(0,1) fields, without source); Mcell/s."""
    import oracle
    import workloads as W
    from oracle.source import Source as OSource
    from threadpoolctl import threadpool_limits
    h, dt, eps, ci = make_inputs(n)
    g = oracle.Grid(n, n, n, h, h, h, dt, eps)
    rows = []
    with threadpool_limits(limits=1):
        for scheme in oracle.SCHEMES + oracle.SPLITTINGS:
            for form in oracle.FORMS:
                split = scheme in oracle.SPLITTINGS
                u0 = W.random_fields(n, n, n, seed=3) if split else W.zero_fields(n, n, n)
                t0 = time.perf_counter()
                oracle.run(scheme, form, g, u0, steps, None if split else OSource(*ci))
                t1 = time.perf_counter()
                rows.append({"scheme": scheme, "form": form, "mcells_per_s": n ** 3 * steps / (t1 - t0) / 1e6,
                             "seconds": t1 - t0})
                log(json.dumps(rows[-1]))
    return {"workload": f"{n}^3 random-box eps_r, CFL 5, {steps} steps, FP64 NumPy oracle, single thread",
            "host": host_info(), "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--variants", default="all", help="'all', 'none' or comma list scheme/form/prec")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched-cavity and adjoint lines")
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--only", choices=["batch", "adjoint", "cn", "graphs", "order4"], default=None,
                    help="run only the batched-cavity or the adjoint measurement and print its JSON")
    ap.add_argument("--cpu-schemes", action="store_true",
                    help="only time the FP64 oracle per scheme and form on the host (no GPU) and print its JSON")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU slab decomposition is a design, not built", file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    if args.cpu_schemes:
        print(json.dumps(cpu_schemes()), flush=True)
        return
    import torch
    if args.copy_probe:
        nel = args.copy_probe * (1 << 20) // 4
        a = torch.ones(nel, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nel * 4, "copies": 5}), flush=True)
        return
    if args.only == "batch":
        print(json.dumps([run_batch(args.batch_steps, 5),
                          run_batch(args.batch_steps, 5, prec="f32p", singles=False)]), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(run_adjoint()), flush=True)
        return
    if args.only == "cn":
        print(json.dumps(run_cn()), flush=True)
        return
    if args.only == "graphs":
        print(json.dumps(run_graphs()), flush=True)
        return
    if args.only == "order4":
        refs = Fp64Refs()
        rows = run_order4(args.n, ("f32p", "f32", "f64"), 10, 2, make_inputs(args.n), refs)
        refs.close()
        print(json.dumps(rows), flush=True)
        return
    n = args.n
    inputs = make_inputs(n)
    log(f"[bench] {n}^3, {args.steps} steps, warmup {args.warmup}")
    refs = Fp64Refs()
    head = run_variant(n, "adi", "fundamental", "f32", args.steps, args.warmup, inputs, tune_reps=10, refs=refs)
    variants = []
    extras = {}
    if args.variants != "none":
        todo = [("adi", "conventional", "f32"), ("adi", "fundamental", "f32p"), ("adi", "fundamental", "f32s64"),
                ("adi", "conventional", "f32s64"),
                ("adi", "fundamental", "f64"), ("adi", "conventional", "f64"),
                ("lod1", "fundamental", "f32"), ("ss2", "fundamental", "f32"), ("lod2", "fundamental", "f32"),
                ("lod1", "conventional", "f32"), ("ss2", "conventional", "f32"), ("lod2", "conventional", "f32"),
                ("lod1", "fundamental", "f32p"), ("ss2", "fundamental", "f32p"), ("lod2", "fundamental", "f32p"),
                ("dyakonov", "fundamental", "f32"), ("douglas_gunn", "fundamental", "f32"),
                ("lod1", "fundamental", "f64"), ("ss2", "fundamental", "f64"), ("lod2", "fundamental", "f64"),
                ("lod1", "conventional", "f64"), ("ss2", "conventional", "f64"), ("lod2", "conventional", "f64")]
        if args.variants != "all":
            todo = [tuple(v.split("/")) for v in args.variants.split(",")]
        vsteps = max(10, args.steps // 4)
        for sch, form, prec in todo:
            variants.append(run_variant(n, sch, form, prec, vsteps, 2, inputs, refs=refs))
    if not args.no_extras:
        # the other CFL numbers of the 512^3 workload: the passes have no
        # data-dependent control flow, so the step time moves only where
        # FDTD_F32 (refined) and plain FP32 solves at both ends of the CFL range
        import workloads as W
        h0, _, eps0, ci0 = inputs
        cfl_rows = []
        for cfl in (1.0, 10.0):
            for prec in ("f32", "f32p"):
                r = run_variant(n, "adi", "fundamental", prec, max(10, args.steps // 4), 2,
                                (h0, W.yee_dt(h0, h0, h0, cfl), eps0, ci0), refs=refs)
                r["cfl"] = cfl
                cfl_rows.append(r)
        extras["adi_fundamental_512cube_cfl_1_and_10"] = cfl_rows
        refs.close()
        extras["batch_64_cavities"] = run_batch(args.batch_steps, 5)
        extras["batch_64_cavities_plain_f32"] = run_batch(args.batch_steps, 5, prec="f32p", singles=False)
        extras["adjoint_gradient"] = run_adjoint()
        extras["graphs_128x128x64"] = run_graphs()
        extras["crank_nicolson_256cube"] = run_cn()
        # fourth-order differences (fdtd_set_order), fundamental ADI on the same 512^3 workload
        extras["adi_fundamental_order4_512cube"] = run_order4(n, ("f32p", "f32"), 10, 2, inputs, refs)
        # the smaller size of the same workload (256^3), FP32 as the library runs it and plain
        in256 = make_inputs(256)
        extras["adi_fundamental_256cube"] = [run_variant(256, "adi", "fundamental", prec, 100, 5, in256, refs=refs)
                                             for prec in ("f32", "f32p")]
    refs.close()
    # roofline of the dominant kernel: the y/z-line pass (4 of the 6 passes
    # per step), priced on the algorithmic bytes per slot (read E, H, FP32
    # eps_r; write E, H: 20 B); the plan actually reads a one-byte material
    # index instead of eps_r (17 B), reported beside it
    yz_bytes = pass_nodes(n) * bytes_per_slot("f32")
    yz_bytes_act = pass_nodes(n) * bytes_per_slot("f32", material_index=True)
    yz_ms = head["yz_ms_avg"]
    achieved = yz_bytes / (yz_ms * 1e-3) / 1e9 if yz_ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(head["kernel_config"][1], head["kernel_config"][2], head["refined"]),
            "kernel": "pass_yz_kernel (fundamental, FP32%s)" % (", refined solves" if head["refined"] else ""),
            "bytes_per_slot": bytes_per_slot("f32"), "slots_per_launch": pass_nodes(n),
            "bytes_per_launch": yz_bytes, "avg_launch_ms": yz_ms, "launches": head["yz_launches"],
            "bytes_per_slot_actual": bytes_per_slot("f32", material_index=True),
            "frac_actual_bytes": yz_bytes_act / (yz_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if yz_ms > 0 else 0.0}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()
    line = {
        "metric": METRIC, "value": head["mcells_per_s"], "unit": "Mcell/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"fundamental ADI, {n}^3 cells, random-box eps_r (32 boxes, U[1,12]), "
                               f"Ez Gaussian-pulse source, CFL 5, PEC",
                   "cells": n ** 3, "scheme": "adi", "form": "fundamental", "fields": "f32",
                   "solve": "f32, refined once" if head["refined"] else "f32"},
        "hbm_frac_alg": head["hbm_frac_alg"],
        "hbm_frac_actual_bytes": head["hbm_frac_actual_bytes"],
        "rel_l2_vs_gpu_fp64": head.get("rel_l2_vs_gpu_fp64"),
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
        "extras": extras,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
