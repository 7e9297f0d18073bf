"""The sampled LOD1 step of ``_sampled.py`` against the oracle's whole-grid
step (brute force on small grids): the lines it returns must equal the
whole-grid result, including lines next to the walls."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import conventional
from oracle.fundamental import lod_step
from oracle.yee import CIDX
from ._sampled import lod1_xline, lod1_yline, lod1_zline


@pytest.mark.parametrize("form", ["fundamental", "conventional"])
@pytest.mark.parametrize("nx,ny,nz,seed", [(9, 11, 13, 1), (16, 7, 10, 2)])
def test_sampled_lod1_equals_whole_grid(nx, ny, nz, seed, form):
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    eps = W.random_box_eps(nx, ny, nz, seed=seed, nboxes=6).astype(np.float64)
    u0 = W.random_fields(nx, ny, nz, seed=seed + 10)
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    ref = lod_step("lod1", u0, g, 0) if form == "fundamental" else conventional.step("lod1", u0, g, 0)
    for i0, j0 in [(0, 1), (nx // 2, ny // 2), (nx - 1, ny - 1), (1, ny - 2)]:
        ex, hy = lod1_zline(eps, u0[CIDX["Ex"]][:, :, i0], u0[CIDX["Hz"]][:, :, i0],
                            u0[CIDX["Ez"]][:, j0, :], u0[CIDX["Hy"]][:, j0, :], i0, j0, h, dt, form)
        want_ex = ref[CIDX["Ex"]][:, j0, i0]
        want_hy = ref[CIDX["Hy"]][:, j0, i0]
        assert np.max(np.abs(want_ex)) > 0.1 and np.max(np.abs(want_hy)) > 1e-4
        assert np.max(np.abs(ex - want_ex)) <= 1e-13 * np.max(np.abs(want_ex))
        assert np.max(np.abs(hy - want_hy)) <= 1e-13 * np.max(np.abs(want_hy))


@pytest.mark.parametrize("form", ["fundamental", "conventional"])
@pytest.mark.parametrize("nx,ny,nz,seed", [(9, 11, 13, 1), (16, 7, 10, 2)])
def test_sampled_lod1_xline_equals_whole_grid(nx, ny, nz, seed, form):
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    eps = W.random_box_eps(nx, ny, nz, seed=seed, nboxes=6).astype(np.float64)
    u0 = W.random_fields(nx, ny, nz, seed=seed + 10)
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    ref = lod_step("lod1", u0, g, 0) if form == "fundamental" else conventional.step("lod1", u0, g, 0)
    for j0, k0 in [(0, 1), (ny // 2, nz // 2), (ny - 1, nz - 1), (1, nz - 2)]:
        ey, hz = lod1_xline(eps, u0[CIDX["Ey"]][:, j0, :], u0[CIDX["Hx"]][:, j0, :],
                            u0[CIDX["Ex"]][k0, :, :], u0[CIDX["Hz"]][k0, :, :], j0, k0, h, dt, form)
        want_ey = ref[CIDX["Ey"]][k0, j0, :]
        want_hz = ref[CIDX["Hz"]][k0, j0, :]
        assert np.max(np.abs(want_ey)) > 0.1 and np.max(np.abs(want_hz)) > 1e-4
        assert np.max(np.abs(ey - want_ey)) <= 1e-13 * np.max(np.abs(want_ey))
        assert np.max(np.abs(hz - want_hz)) <= 1e-13 * np.max(np.abs(want_hz))


@pytest.mark.parametrize("form", ["fundamental", "conventional"])
@pytest.mark.parametrize("nx,ny,nz,seed", [(9, 11, 13, 1), (16, 7, 10, 2)])
def test_sampled_lod1_yline_equals_whole_grid(nx, ny, nz, seed, form):
    h = 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    eps = W.random_box_eps(nx, ny, nz, seed=seed, nboxes=6).astype(np.float64)
    u0 = W.random_fields(nx, ny, nz, seed=seed + 10)
    g = oracle.Grid(nx, ny, nz, h, h, h, dt, eps)
    ref = lod_step("lod1", u0, g, 0) if form == "fundamental" else conventional.step("lod1", u0, g, 0)
    for k0, i0 in [(0, 1), (nz // 2, nx // 2), (nz - 1, nx - 1), (1, nx - 2)]:
        ez, hx = lod1_yline(eps, u0[CIDX["Ez"]][k0, :, :], u0[CIDX["Hy"]][k0, :, :],
                            u0[CIDX["Ey"]][:, :, i0], u0[CIDX["Hx"]][:, :, i0], k0, i0, h, dt, form)
        want_ez = ref[CIDX["Ez"]][k0, :, i0]
        want_hx = ref[CIDX["Hx"]][k0, :, i0]
        assert np.max(np.abs(want_ez)) > 0.1 and np.max(np.abs(want_hx)) > 1e-4
        assert np.max(np.abs(ez - want_ez)) <= 1e-13 * np.max(np.abs(want_ez))
        assert np.max(np.abs(hx - want_hx)) <= 1e-13 * np.max(np.abs(want_hx))


def test_sampled_lod1_sees_a_planted_error():
    """A mistake on either input plane shows in the sampled line."""
    nx, ny, nz, h = 9, 11, 13, 1e-3
    dt = W.yee_dt(h, h, h, 5.0)
    eps = W.random_box_eps(nx, ny, nz, seed=1, nboxes=6).astype(np.float64)
    u0 = W.random_fields(nx, ny, nz, seed=11)
    args = [u0[CIDX["Ex"]][:, :, 4], u0[CIDX["Hz"]][:, :, 4], u0[CIDX["Ez"]][:, 5, :], u0[CIDX["Hy"]][:, 5, :]]
    base = lod1_zline(eps, *args, 4, 5, h, dt)
    for m in range(4):
        bad = [a.copy() for a in args]
        bad[m][6, 3 if m < 2 else 6] += 1.0
        got = lod1_zline(eps, *bad, 4, 5, h, dt)
        assert max(np.max(np.abs(got[0] - base[0])), np.max(np.abs(got[1] - base[1])) * 377) > 1e-6
