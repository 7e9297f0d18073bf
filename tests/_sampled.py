"""Sampled outputs of one LOD1 (SS1) step, fundamental or conventional form,
at any grid size, for parity at sizes the oracle's whole-grid steps do not
reach.

One LOD1 step applies the A sub-step, then the B sub-step, both with
theta = dt/2 (Sec. III for the fundamental form, eq. (orgLOD) for the
conventional one, whose right side applies the same operator).  Every pair pass couples samples
along its own line only, so Ex and Hy on one z line (i0, j0) after the step
depend on:
* Ex after A on that line: the A pass of the pair (Ex, Hz) along y, whose
  lines at x index i0 use Ex, Hz and the cells of the plane x = i0;
* Hy after A on that line: the A pass of the pair (Ez, Hy) along x, whose
  lines at y index j0 use Ez, Hy and the cells of the plane y = j0;
and then on the B pass of the pair (Ex, Hy) along z on that line.
The oracle's own sub-step (``oracle.fundamental.lod_substep``, or
``oracle.conventional.substep`` with X = Y) runs each of
these on a thin grid that holds exactly those lines: one cell wide in x
(x = i0) or two cells wide in y (cells j0 - 1 and j0, so that y index j0 is
interior), with the same cells, hence the same per-node eps_r (the node
owns the cell with its index) and the same walls on the line axis.  This
module only cuts and places arrays; the arithmetic is the oracle's.
It is pinned against whole-grid oracle steps in ``test_sampled_pins.py``.
"""
from __future__ import annotations

import numpy as np

import oracle
from oracle import conventional
from oracle.fundamental import LOD_MAIN, lod_substep
from oracle.yee import CIDX


def _substep(form):
    if form == "fundamental":
        return lod_substep
    assert form == "conventional"
    return lambda u, op, theta, g: conventional.substep(u, op, op, theta, g)


def _zeros(nx, ny, nz):
    return [np.zeros((nz + 1, ny + 1, nx + 1)) for _ in range(6)]


def lod1_zline(eps_r, ex_x, hz_x, ez_y, hy_y, i0, j0, h, dt, form="fundamental"):
    """Ex and Hy on the z line (x index i0, y index j0) after one LOD1 step.

    eps_r: cells (nz, ny, nx); ex_x, hz_x: Ex and Hz at x index i0, arrays
    (nz+1, ny+1); ez_y, hy_y: Ez and Hy at y index j0, arrays (nz+1, nx+1).
    Needs 0 <= i0 < nx and 1 <= j0 <= ny - 1 (Ex and Hy exist there).
    Returns (Ex, Hy), each of length nz + 1 (FP64)."""
    nz, ny, nx = eps_r.shape
    assert 0 <= i0 < nx and 1 <= j0 <= ny - 1
    (op_a, fa, _), (op_b, fb, _) = LOD_MAIN["lod1"]
    assert (op_a, op_b) == ("A", "B")
    assert [m[:3] for m in conventional.MAIN["lod1"]] == [("A", "A", fa), ("B", "B", fb)]
    sub = _substep(form)
    # A: pair (Ex, Hz) along y on the plane x = i0
    g1 = oracle.Grid(1, ny, nz, h, h, h, dt, eps_r[:, :, i0:i0 + 1])
    u = _zeros(1, ny, nz)
    u[CIDX["Ex"]][:, :, 0] = ex_x
    u[CIDX["Hz"]][:, :, 0] = hz_x
    ex_a = sub(u, "A", fa * dt, g1)[CIDX["Ex"]][:, j0, 0]
    # A: pair (Ez, Hy) along x on the plane y = j0
    g2 = oracle.Grid(nx, 2, nz, h, h, h, dt, eps_r[:, j0 - 1:j0 + 1, :])
    u = _zeros(nx, 2, nz)
    u[CIDX["Ez"]][:, 1, :] = ez_y
    u[CIDX["Hy"]][:, 1, :] = hy_y
    hy_a = sub(u, "A", fa * dt, g2)[CIDX["Hy"]][:, 1, i0]
    # B: pair (Ex, Hy) along z on the line (i0, j0)
    g3 = oracle.Grid(1, 2, nz, h, h, h, dt, eps_r[:, j0 - 1:j0 + 1, i0:i0 + 1])
    u = _zeros(1, 2, nz)
    u[CIDX["Ex"]][:, 1, 0] = ex_a
    u[CIDX["Hy"]][:, 1, 0] = hy_a
    out = sub(u, "B", fb * dt, g3)
    return out[CIDX["Ex"]][:, 1, 0], out[CIDX["Hy"]][:, 1, 0]


def lod1_xline(eps_r, ey_y, hx_y, ex_z, hz_z, j0, k0, h, dt, form="fundamental"):
    """Ey and Hz on the x line (y index j0, z index k0) after one LOD1 step.

    Ey after A on that line comes from the pair (Ey, Hx) along z on the
    plane y = j0 (a grid one cell wide in y), Hz after A from the pair
    (Ex, Hz) along y on the plane z = k0 (cells k0 - 1 and k0, so that z
    index k0 is interior); then the B pass of the pair (Ey, Hz) along x.
    ey_y, hx_y: Ey and Hx at y index j0, arrays (nz+1, nx+1); ex_z, hz_z:
    Ex and Hz at z index k0, arrays (ny+1, nx+1).  Needs 0 <= j0 < ny and
    1 <= k0 <= nz - 1.  Returns (Ey, Hz), each of length nx + 1 (FP64)."""
    nz, ny, nx = eps_r.shape
    assert 0 <= j0 < ny and 1 <= k0 <= nz - 1
    (_, fa, _), (_, fb, _) = LOD_MAIN["lod1"]
    sub = _substep(form)
    # A: pair (Ey, Hx) along z on the plane y = j0
    g1 = oracle.Grid(nx, 1, nz, h, h, h, dt, eps_r[:, j0:j0 + 1, :])
    u = _zeros(nx, 1, nz)
    u[CIDX["Ey"]][:, 0, :] = ey_y
    u[CIDX["Hx"]][:, 0, :] = hx_y
    ey_a = sub(u, "A", fa * dt, g1)[CIDX["Ey"]][k0, 0, :]
    # A: pair (Ex, Hz) along y on the plane z = k0
    g2 = oracle.Grid(nx, ny, 2, h, h, h, dt, eps_r[k0 - 1:k0 + 1, :, :])
    u = _zeros(nx, ny, 2)
    u[CIDX["Ex"]][1, :, :] = ex_z
    u[CIDX["Hz"]][1, :, :] = hz_z
    hz_a = sub(u, "A", fa * dt, g2)[CIDX["Hz"]][1, j0, :]
    # B: pair (Ey, Hz) along x on the line (j0, k0)
    g3 = oracle.Grid(nx, 1, 2, h, h, h, dt, eps_r[k0 - 1:k0 + 1, j0:j0 + 1, :])
    u = _zeros(nx, 1, 2)
    u[CIDX["Ey"]][1, 0, :] = ey_a
    u[CIDX["Hz"]][1, 0, :] = hz_a
    out = sub(u, "B", fb * dt, g3)
    return out[CIDX["Ey"]][1, 0, :], out[CIDX["Hz"]][1, 0, :]


def lod1_yline(eps_r, ez_z, hy_z, ey_x, hx_x, k0, i0, h, dt, form="fundamental"):
    """Ez and Hx on the y line (z index k0, x index i0) after one LOD1 step.

    Ez after A on that line comes from the pair (Ez, Hy) along x on the
    plane z = k0 (a grid one cell wide in z), Hx after A from the pair
    (Ey, Hx) along z on the plane x = i0 (cells i0 - 1 and i0, so that x
    index i0 is interior); then the B pass of the pair (Ez, Hx) along y.
    ez_z, hy_z: Ez and Hy at z index k0, arrays (ny+1, nx+1); ey_x, hx_x:
    Ey and Hx at x index i0, arrays (nz+1, ny+1).  Needs 0 <= k0 < nz and
    1 <= i0 <= nx - 1.  Returns (Ez, Hx), each of length ny + 1 (FP64)."""
    nz, ny, nx = eps_r.shape
    assert 0 <= k0 < nz and 1 <= i0 <= nx - 1
    (_, fa, _), (_, fb, _) = LOD_MAIN["lod1"]
    sub = _substep(form)
    # A: pair (Ez, Hy) along x on the plane z = k0
    g1 = oracle.Grid(nx, ny, 1, h, h, h, dt, eps_r[k0:k0 + 1, :, :])
    u = _zeros(nx, ny, 1)
    u[CIDX["Ez"]][0, :, :] = ez_z
    u[CIDX["Hy"]][0, :, :] = hy_z
    ez_a = sub(u, "A", fa * dt, g1)[CIDX["Ez"]][0, :, i0]
    # A: pair (Ey, Hx) along z on the plane x = i0
    g2 = oracle.Grid(2, ny, nz, h, h, h, dt, eps_r[:, :, i0 - 1:i0 + 1])
    u = _zeros(2, ny, nz)
    u[CIDX["Ey"]][:, :, 1] = ey_x
    u[CIDX["Hx"]][:, :, 1] = hx_x
    hx_a = sub(u, "A", fa * dt, g2)[CIDX["Hx"]][k0, :, 1]
    # B: pair (Ez, Hx) along y on the line (k0, i0)
    g3 = oracle.Grid(2, ny, 1, h, h, h, dt, eps_r[k0:k0 + 1, :, i0 - 1:i0 + 1])
    u = _zeros(2, ny, 1)
    u[CIDX["Ez"]][0, :, 1] = ez_a
    u[CIDX["Hx"]][0, :, 1] = hx_a
    out = sub(u, "B", fb * dt, g3)
    return out[CIDX["Ez"]][0, :, 1], out[CIDX["Hx"]][0, :, 1]
