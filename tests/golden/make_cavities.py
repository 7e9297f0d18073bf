"""Write tests/golden/cavities_64.npz: FP64 oracle reference for the batch of
64 PEC cavities (sizes U{16..96} per axis from workloads.cavity_batch(64,
seed=4); cavity g: 32 random eps_r boxes with seed 1000 + g, N(0,1) fields with
seed 1100 + g; 1 mm cells, CFL 5, fundamental ADI, no source).

Stored (calls only oracle/ and workloads/):
  sizes                 (64, 3) nx, ny, nz
  steps_all             50: every cavity after this many steps
  idx_<comp>_<g>        flat node indices of up to 512 seeded samples per component
  val_<comp>_<g>        oracle values there after steps_all steps
  norm2_<g>             energy-weighted squared norm of the whole field then
  small                 the 4 smallest cavities (by cell count)
  steps_small           500
  sval_<comp>_<g>, snorm2_<g>   the same at steps_small for the 4 smallest

Usage: python tests/golden/make_cavities.py [workers]
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import yee  # noqa: E402

N_SAMPLES = 512
STEPS_ALL = 50
STEPS_SMALL = 500


def cavity(g, nx, ny, nz):
    eps = W.random_box_eps(nx, ny, nz, seed=1000 + g, nboxes=32)
    u0 = W.random_fields(nx, ny, nz, seed=1100 + g)
    return eps, u0


def one(args):
    g, (nx, ny, nz), steps_list = args
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    eps, u0 = cavity(g, nx, ny, nz)
    gr = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    rng = np.random.default_rng(5000 + g)
    size = (nx + 1) * (ny + 1) * (nz + 1)
    idx = {c: np.sort(rng.choice(size, min(N_SAMPLES, size), replace=False)) for c in yee.COMPONENTS}
    out = {f"idx_{c}_{g}": idx[c] for c in yee.COMPONENTS}
    for steps, tag in steps_list:
        u, _ = oracle.run("adi", "fundamental", gr, u0, steps)
        for k, c in enumerate(yee.COMPONENTS):
            out[f"{tag}val_{c}_{g}"] = u[k].ravel()[idx[c]]
        out[f"{tag}norm2_{g}"] = np.float64(yee.energy(u, gr))
    return out


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 8
    sizes = W.cavity_batch(64, seed=4)
    small = sorted(range(len(sizes)), key=lambda g: int(np.prod(sizes[g])))[:4]
    jobs = []
    for g, sz in enumerate(sizes):
        steps_list = [(STEPS_ALL, "")] + ([(STEPS_SMALL, "s")] if g in small else [])
        jobs.append((g, tuple(int(v) for v in sz), steps_list))
    out = {"sizes": np.array(sizes, dtype=np.int64), "steps_all": np.int64(STEPS_ALL),
           "small": np.array(small, dtype=np.int64), "steps_small": np.int64(STEPS_SMALL)}
    with Pool(workers) as pool:
        for part in pool.imap_unordered(one, jobs):
            out.update(part)
            print(".", end="", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cavities_64.npz")
    np.savez_compressed(path, **out)
    print("\nwrote", path)


if __name__ == "__main__":
    main()
