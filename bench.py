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


def bytes_per_node(dtype_code, material_index=True):
    # read E, H and the medium; write E, H.  The medium is a one-byte material
    # index when the plan has <= 256 distinct eps_r values (this workload has
    # 33), else an FP32 eps_r.
    w = 8 if dtype_code == "f64" else 4
    return 4 * w + (1 if material_index else 4)


def pass_nodes(n):
    # every pass of a cubic n^3 grid covers n * (n-1) lines of n slots
    return n * (n - 1) * n


def run_variant(n, scheme, form, prec, steps, warmup, inputs, per_launch=True, tune=True):
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
                eps_r=torch.from_numpy(eps))
    if tune:
        plan.autotune(3)
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
    del E, H
    torch.cuda.empty_cache()
    ms = (t1 - t0) * 1e3 / steps
    cells = n ** 3
    mcells = cells / (ms * 1e-3) / 1e6
    bpn = bytes_per_node(prec)
    npass = 9 if scheme == "ss2" else 6
    alg_bytes_step = npass * pass_nodes(n) * bpn          # line passes only
    if scheme == "adi" and form == "conventional":           # + the two cross-coupled arrays
        alg_bytes_step = npass * pass_nodes(n) * (bpn + 2 * (8 if prec == "f64" else 4))
    hbm_frac = alg_bytes_step / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    out = dict(scheme=scheme, form=form, prec=prec, ms_per_step=ms, mcells_per_s=mcells,
               alg_bytes_per_step=alg_bytes_step, hbm_frac_alg=hbm_frac, main_ms=tm["main_ms"],
               yz_ms_avg=tm["yz_ms_avg"], x_ms_avg=tm["x_ms_avg"], yz_launches=tm["yz_launches"],
               x_launches=tm["x_launches"], finite=finite, kernel_config=cfg)
    log(json.dumps(out))
    return out


def cpu_baseline(n=256, steps=1):
    """The FP64 oracle (fundamental ADI) on the host, single thread, on a
    bounded sample of the same workload (n^3 cells, `steps` steps)."""
    import numpy as np
    import oracle
    import workloads as W
    from oracle.source import Source as OSource
    h, dt, eps, ci = make_inputs(n)
    g = oracle.Grid(n, n, n, h, h, h, dt, eps)
    u0 = W.zero_fields(n, n, n)
    src = OSource(*ci)
    t0 = time.perf_counter()
    oracle.run("adi", "fundamental", g, u0, steps, src)
    t1 = time.perf_counter()
    rate = n ** 3 * steps / (t1 - t0) / 1e6
    return {"value": rate, "unit": "Mcell/s", "cores": 1, "kind": "oracle",
            "sample": f"FP64 NumPy oracle, fundamental ADI, {n}^3 cells of the same random-box/source "
                      f"workload, {steps} step(s), single thread ({t1 - t0:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--variants", default="all", help="'all', 'none' or comma list scheme/form/prec")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU slab decomposition is a design, not built", file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
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
    n = args.n
    inputs = make_inputs(n)
    log(f"[bench] {n}^3, {args.steps} steps, warmup {args.warmup}")
    head = run_variant(n, "adi", "fundamental", "f32", args.steps, args.warmup, inputs)
    variants = []
    if args.variants != "none":
        todo = [("adi", "conventional", "f32"), ("adi", "fundamental", "f32s64"), ("adi", "conventional", "f32s64"),
                ("adi", "fundamental", "f64"), ("adi", "conventional", "f64"),
                ("lod1", "fundamental", "f32"), ("ss2", "fundamental", "f32"), ("lod2", "fundamental", "f32"),
                ("lod1", "conventional", "f32"), ("ss2", "conventional", "f32"), ("lod2", "conventional", "f32")]
        if args.variants != "all":
            todo = [tuple(v.split("/")) for v in args.variants.split(",")]
        vsteps = max(10, args.steps // 4)
        for sch, form, prec in todo:
            variants.append(run_variant(n, sch, form, prec, vsteps, 2, inputs))
    # roofline of the dominant kernel: the y/z-line pass (4 of the 6 passes per step)
    bpn = bytes_per_node("f32")
    yz_bytes = pass_nodes(n) * bpn
    yz_ms = head["yz_ms_avg"]
    achieved = yz_bytes / (yz_ms * 1e-3) / 1e9 if yz_ms > 0 else 0.0
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "kernel": "pass_yz_kernel (fundamental, FP32)", "bytes_per_launch": yz_bytes,
            "avg_launch_ms": yz_ms, "launches": head["yz_launches"]}
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
                   "cells": n ** 3, "scheme": "adi", "form": "fundamental", "fields": "f32", "solve": "f32"},
        "hbm_frac_alg": head["hbm_frac_alg"],
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": variants,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
