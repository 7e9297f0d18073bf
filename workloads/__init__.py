"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module holds input generation only: random field states, random-box
permittivity maps, source/probe cell picks and batches of cavity sizes.  It
contains none of the time-stepping arithmetic, so both the oracle and the GPU
path can be driven from the same inputs without sharing any of the method.

Geometry conventions (Yee grid, PEC box of nx*ny*nz cells, 1-based "cell"
counts, 0-based node indices):

* every field component is stored as a node array of shape (nz+1, ny+1, nx+1),
  indexed [k, j, i], x fastest;
* the component stored at [k, j, i] sits at the usual Yee position:
  Ex (i+1/2, j, k), Ey (i, j+1/2, k), Ez (i, j, k+1/2),
  Hx (i, j+1/2, k+1/2), Hy (i+1/2, j, k+1/2), Hz (i+1/2, j+1/2, k);
* entries whose position lies outside the box are "out of extent" and are 0;
* E entries tangential to a PEC wall are 0;
* H entries normal to a wall are kept (they are static under the method).

All random numbers come from ``numpy.random.default_rng(seed)`` (PCG64).
"""
from __future__ import annotations

import math

import numpy as np

EPS0 = 8.8541878128e-12  # F/m
MU0 = 1.25663706212e-6  # H/m
C0 = 1.0 / math.sqrt(EPS0 * MU0)

COMPONENTS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def yee_dt(dx: float, dy: float, dz: float, cfl_number: float) -> float:
    """Time step that is `cfl_number` times the vacuum Yee (explicit FDTD) limit."""
    return cfl_number / (C0 * math.sqrt(dx ** -2 + dy ** -2 + dz ** -2))


def extent_mask(comp: str, nx: int, ny: int, nz: int) -> np.ndarray:
    """True where the component's Yee position lies inside the box (incl. walls)."""
    m = np.ones((nz + 1, ny + 1, nx + 1), dtype=bool)
    if comp in ("Ex", "Hy", "Hz"):
        m[:, :, nx] = False  # x index i+1/2 with i = nx is outside
    if comp in ("Ey", "Hx", "Hz"):
        m[:, ny, :] = False
    if comp in ("Ez", "Hx", "Hy"):
        m[nz, :, :] = False
    return m


def wall_tangential_mask(comp: str, nx: int, ny: int, nz: int) -> np.ndarray:
    """True at E entries lying on a PEC wall they are tangential to (forced 0)."""
    m = np.zeros((nz + 1, ny + 1, nx + 1), dtype=bool)
    if comp == "Ex":
        m[:, [0, ny], :] = True
        m[[0, nz], :, :] = True
    elif comp == "Ey":
        m[:, :, [0, nx]] = True
        m[[0, nz], :, :] = True
    elif comp == "Ez":
        m[:, :, [0, nx]] = True
        m[:, [0, ny], :] = True
    return m


def random_fields(nx: int, ny: int, nz: int, seed: int) -> list[np.ndarray]:
    """I.i.d. N(0,1) fields (FP64), generated component by component in the order
    Ex, Ey, Ez, Hx, Hy, Hz from one PCG64 stream; out-of-extent entries and
    wall-tangential E are then set to 0 (normal H on the walls stays random)."""
    rng = np.random.default_rng(seed)
    out = []
    for c in COMPONENTS:
        a = rng.standard_normal((nz + 1, ny + 1, nx + 1))
        a[~extent_mask(c, nx, ny, nz)] = 0.0
        if c.startswith("E"):
            a[wall_tangential_mask(c, nx, ny, nz)] = 0.0
        out.append(a)
    return out


def zero_fields(nx: int, ny: int, nz: int) -> list[np.ndarray]:
    return [np.zeros((nz + 1, ny + 1, nx + 1)) for _ in COMPONENTS]


def random_box_eps(nx: int, ny: int, nz: int, seed: int, nboxes: int = 32,
                   ext_lo: float = 1 / 16, ext_hi: float = 1 / 4,
                   vmin: float = 1.0, vmax: float = 12.0) -> np.ndarray:
    """Piecewise-constant relative permittivity per cell, shape (nz, ny, nx), FP32.

    Background 1.  Box b: its lower corner is uniform over the cells, its extent
    along each axis is uniform in [n*ext_lo, n*ext_hi] (at least 1 cell), it is
    clipped to the grid, and its value is U[vmin, vmax] rounded to FP32.  Later
    boxes overwrite earlier ones.
    """
    rng = np.random.default_rng(seed)
    eps = np.ones((nz, ny, nx), dtype=np.float32)
    dims = (nx, ny, nz)
    for _ in range(nboxes):
        lo = [int(rng.integers(0, n)) for n in dims]
        ext = [int(rng.integers(max(1, int(n * ext_lo)), max(1, int(n * ext_hi)) + 1))
               for n in dims]
        val = np.float32(rng.uniform(vmin, vmax))
        (x0, y0, z0), (ex, ey, ez) = lo, ext
        eps[z0:min(nz, z0 + ez), y0:min(ny, y0 + ey), x0:min(nx, x0 + ex)] = val
    return eps


def random_mu(nx: int, ny: int, nz: int, seed: int, vmin: float = 1.0, vmax: float = 3.0) -> np.ndarray:
    """Relative permeability per cell, shape (nz, ny, nx), FP32: U[vmin, vmax]
    independently in every cell (the most irregular medium: every H sample of
    a line differs from its neighbours)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(vmin, vmax, (nz, ny, nx)).astype(np.float32)


def design_region_eps(nx: int, ny: int, nz: int, box: tuple[int, int, int, int, int, int],
                      seed: int) -> np.ndarray:
    """eps_r = 1 outside the design box (x0, y0, z0, sx, sy, sz); per-voxel U[1,12]
    inside, FP32."""
    rng = np.random.default_rng(seed)
    x0, y0, z0, sx, sy, sz = box
    eps = np.ones((nz, ny, nx), dtype=np.float32)
    eps[z0:z0 + sz, y0:y0 + sy, x0:x0 + sx] = rng.uniform(1.0, 12.0, (sz, sy, sx)).astype(np.float32)
    return eps


def interior_cell(nx: int, ny: int, nz: int, seed: int, margin: int = 8) -> tuple[int, int, int]:
    """A seeded cell index (i, j, k) at least `margin` cells from every wall
    (the margin shrinks on small grids so that a cell always exists)."""
    rng = np.random.default_rng(seed)
    out = []
    for n in (nx, ny, nz):
        m = min(margin, (n - 1) // 2)
        out.append(int(rng.integers(max(1, m), max(2, n - m))))
    return tuple(out)


def cavity_batch(count: int, seed: int, lo: int = 16, hi: int = 96) -> list[tuple[int, int, int]]:
    """`count` cavity sizes (nx, ny, nz), each uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return [tuple(int(v) for v in rng.integers(lo, hi + 1, 3)) for _ in range(count)]


def design_problem(seed: int, nx: int = 128, ny: int = 128, nz: int = 64,
                   box_size: tuple[int, int, int] = (64, 64, 16)) -> dict:
    """Differentiable-cavity workload: a centred design box of box_size cells
    (eps_r U[1,12] per voxel, 1 elsewhere), an Ez source cell below the box
    and a probe node above it, both seeded.  Returns a dict with nx, ny, nz,
    design_box = (i0, i1, j0, j1, k0, k1), eps (nz, ny, nx) FP32, src, probe."""
    sx, sy, sz = box_size
    x0, y0, z0 = (nx - sx) // 2, (ny - sy) // 2, (nz - sz) // 2
    eps = design_region_eps(nx, ny, nz, (x0, y0, z0, sx, sy, sz), seed)
    rng = np.random.default_rng(seed + 1000)
    def cell(klo, khi):
        return (int(rng.integers(max(1, nx // 4), max(2, 3 * nx // 4))),
                int(rng.integers(max(1, ny // 4), max(2, 3 * ny // 4))),
                int(rng.integers(klo, max(klo + 1, khi))))
    src = cell(max(1, z0 // 3), max(2, z0 - 2))
    probe = cell(min(nz - 2, z0 + sz + 2), max(z0 + sz + 3, nz - max(1, z0 // 3)))
    return dict(nx=nx, ny=ny, nz=nz, design_box=(x0, x0 + sx, y0, y0 + sy, z0, z0 + sz), eps=eps,
                src=src, probe=probe)
