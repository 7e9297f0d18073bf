"""Write tests/golden/precision_sweep_<scheme>.npz: FP64 oracle reference for
the precision sweep (128^3 cells, 1 mm, random-box eps_r (32 boxes, seed 2),
N(0,1) fields (seed 3), CFL number 10 (or the one given), no source, 1000 steps).

Stored (calls only oracle/ and workloads/):
  steps            [100, 500, 1000]
  idx_<comp>       flat node indices of 4096 seeded samples per component
  val_<comp>       (3, 4096) oracle values at those nodes at each stored step
  norm2            (3,) energy-weighted squared norm of the whole field
  trace            invariant energy every 10 steps (101 values)

Usage: python tests/golden/make_precision_sweep.py <scheme> [n] [steps] [cfl]
(cfl other than 10 writes precision_sweep_<scheme>_cfl<cfl>.npz)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from oracle import conventional, fundamental, yee  # noqa: E402

N_SAMPLES = 4096


def main():
    scheme = sys.argv[1]
    n = int(sys.argv[2]) if len(sys.argv) > 2 else 128
    steps = int(sys.argv[3]) if len(sys.argv) > 3 else 1000
    cfl = float(sys.argv[4]) if len(sys.argv) > 4 else 10.0
    h = 1e-3
    dt = W.yee_dt(h, h, h, cfl)
    eps = W.random_box_eps(n, n, n, seed=2, nboxes=32)
    u0 = W.random_fields(n, n, n, seed=3)
    g = oracle.Grid(n, n, n, h, h, h, dt, eps)
    rng = np.random.default_rng(17)
    size = (n + 1) ** 3
    ns = min(N_SAMPLES, size)
    idx = {c: np.sort(rng.choice(size, ns, replace=False)) for c in yee.COMPONENTS}
    marks = [s for s in (steps // 10, steps // 2, steps)]
    vals = {c: np.zeros((len(marks), ns)) for c in yee.COMPONENTS}
    norm2 = np.zeros(len(marks))
    trace = []
    u = yee.clean(u0, g)

    def record(fields, m):
        for k, c in enumerate(yee.COMPONENTS):
            vals[c][m] = fields[k].ravel()[idx[c]]
        norm2[m] = yee.energy(fields, g)

    if scheme == "adi":
        st = fundamental.FundamentalADI(u, g)
        trace.append(st.invariant())
        for s in range(1, steps + 1):
            st.step()
            if s % 10 == 0:
                trace.append(st.invariant())
            if s in marks:
                record(st.fields(), marks.index(s))
            print(scheme, s, flush=True) if s % 50 == 0 else None
    else:
        if scheme == "lod2":
            u = fundamental.lod2_input(u, g)
        trace.append(yee.energy(u, g))
        for s in range(1, steps + 1):
            u = fundamental.lod_step(scheme, u, g, s - 1)
            if s % 10 == 0:
                trace.append(yee.energy(u, g))
            if s in marks:
                out = fundamental.lod2_output(u, g) if scheme == "lod2" else u
                record(out, marks.index(s))
            print(scheme, s, flush=True) if s % 50 == 0 else None
    tag = "" if cfl == 10.0 else f"_cfl{cfl:g}"
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"precision_sweep_{scheme}{tag}.npz")
    np.savez_compressed(out, steps=np.array(marks), norm2=norm2, trace=np.array(trace),
                        n=n, cfl=cfl, **{f"idx_{c}": idx[c] for c in yee.COMPONENTS},
                        **{f"val_{c}": vals[c] for c in yee.COMPONENTS})
    print("wrote", out)


if __name__ == "__main__":
    main()
