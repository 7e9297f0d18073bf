"""Pins of the oracle with the fourth-order staggered differences (grid order
4; the closing remark of Sec. III-A leaves the difference operators of the
updating equations open), against things other than the code under test:

* the difference itself: exact for cubics away from the walls, and the
  image matrices satisfy D_int = -D_half^T (so A and B are skew-adjoint);
* the operators assembled node by node (``dense``, an independent loop over
  the stencil) equal the vectorized ones and are skew-adjoint in the energy
  norm;
* closed forms: PEC cavity modes are exact eigenvectors with
  K4 = (27 sin(k h/2) - sin(3 k h/2)) / (12 h), every scheme evolves them as
  the 6x6 Cayley products, the closed-form ADI dispersion holds with K4, and
  the semi-discrete frequency converges to the exact one at fourth order
  (second order for the Yee differences);
* every scheme, both forms, with a source, random eps and mu and anisotropic
  cells, against the dense matrix formulas; every implicit stage against a
  dense solve; exact energy conservation; D'Yakonov and Douglas-Gunn equal
  ADI.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import dense, yee
from oracle.implicit import diff4_matrices, solve_implicit
from oracle.source import Source

from . import _analytic as an


def grid4(nx=5, ny=4, nz=6, cfl=4.0, seed=0, mu=True, spacing=(1e-3, 1.2e-3, 0.8e-3)):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1, 12, (nz, ny, nx))
    mur = rng.uniform(1, 3, (nz, ny, nx)) if mu else None
    dt = yee.cfl_dt(*spacing, cfl)
    return yee.Grid(nx, ny, nz, *spacing, dt, eps, mur, order=4)


def test_difference_exact_for_cubics():
    """Interior samples of a cubic: the fourth-order difference returns its
    derivative exactly (the second-order one does not)."""
    n, h = 12, 0.37
    x = np.arange(n + 1) * h                          # integer positions
    f = lambda t: 0.3 * t ** 3 - 1.1 * t ** 2 + 0.5 * t + 2.0   # noqa: E731
    df = lambda t: 0.9 * t ** 2 - 2.2 * t + 0.5                   # noqa: E731
    e = np.zeros((1, 1, n + 1))
    e[0, 0, :] = f(x)
    got = yee.diff4_to_half(e, "x", h)[0, 0]
    mid = (np.arange(n) + 0.5) * h
    inner = slice(1, n - 1)                           # stencils that stay off the walls
    assert np.allclose(got[inner], df(mid)[inner], rtol=1e-12, atol=1e-12)
    # H at half positions -> E positions
    hh = np.zeros((1, 1, n + 1))
    hh[0, 0, :n] = f(mid)
    got = yee.diff4_to_integer(hh, "x", h)[0, 0]
    assert np.allclose(got[2:n - 1], df(x)[2:n - 1], rtol=1e-12, atol=1e-12)
    second = yee.diff_to_half(e, "x", h)[0, 0]
    assert np.abs(second[inner] - df(mid)[inner]).max() > 1e-3


@pytest.mark.parametrize("n", [2, 3, 4, 5, 7, 12])
def test_image_matrices_are_negative_transposes(n):
    Dh, Di = diff4_matrices(n, 0.7)
    assert np.allclose(Di, -Dh.T, rtol=0, atol=1e-15)
    # and they are what the vectorized differences apply
    rng = np.random.default_rng(n)
    e = np.zeros((1, 1, n + 1))
    e[0, 0, 1:n] = rng.standard_normal(n - 1)
    assert np.allclose(yee.diff4_to_half(e, "x", 0.7)[0, 0, :n], Dh @ e[0, 0, 1:n], atol=1e-14)
    hh = np.zeros((1, 1, n + 1))
    hh[0, 0, :n] = rng.standard_normal(n)
    assert np.allclose(yee.diff4_to_integer(hh, "x", 0.7)[0, 0, 1:n], Di @ hh[0, 0, :n], atol=1e-14)


def test_dense_operators_equal_vectorized_and_skew_adjoint():
    g = grid4(seed=1)
    ds = dense.DenseSystem(g)
    u = yee.clean(W.random_fields(g.nx, g.ny, g.nz, 2), g)
    Wm = np.diag(ds.w)
    for name in ("A", "B"):
        M = ds.op(name)
        got = ds.to_vec(yee.apply_operator(name, u, g))
        ref = M @ ds.to_vec(u)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        assert np.abs(M.T @ Wm + Wm @ M).max() <= 1e-14 * np.abs(Wm @ M).max()


@pytest.mark.parametrize("mnp", [(1, 1, 1), (2, 1, 3), (3, 2, 1)])
def test_operators_on_cavity_mode(mnp):
    nx, ny, nz, dx, dy, dz = 8, 6, 7, 1e-3, 1.3e-3, 0.9e-3
    g = yee.Grid(nx, ny, nz, dx, dy, dz, 1e-12, order=4)
    a = np.random.default_rng(2).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(nx, ny, nz, dx, dy, dz, *mnp, order=4)
    u = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, a)
    ds = dense.DenseSystem(g)
    for name, M6 in (("A", A6), ("B", B6)):
        ref = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, M6 @ a)
        got = yee.apply_operator(name, u, g)
        for x, y in zip(got, ref):
            assert np.abs(x - y).max() <= 1e-12 * max(np.abs(y).max(), 1e-300) + 1e-300
        gd = ds.op(name) @ ds.to_vec(u)
        assert np.allclose(gd, ds.to_vec(ref), rtol=1e-12, atol=1e-12 * np.abs(gd).max())


@pytest.mark.parametrize("op", ["A", "B"])
@pytest.mark.parametrize("theta_scale", [0.5, -0.25])
def test_implicit_stage_matches_dense(op, theta_scale):
    g = grid4(seed=3)
    ds = dense.DenseSystem(g)
    theta = theta_scale * g.dt
    f = W.random_fields(g.nx, g.ny, g.nz, 7)
    got = solve_implicit(op, yee.PAIRS[op], yee.clean(f, g), theta, g)
    ref = np.linalg.solve(np.eye(ds.n) - theta * ds.op(op), ds.to_vec(f))
    assert np.allclose(ds.to_vec(got), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def _src(g):
    return Source(1, 1, 2, amp=1e12, t0=2 * g.dt, tau=3 * g.dt, f0=1 / (8 * g.dt))


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
@pytest.mark.parametrize("form", oracle.FORMS)
def test_scheme_matches_dense_formula(scheme, form):
    g = grid4(seed=5)
    ds = dense.DenseSystem(g)
    u0 = W.random_fields(g.nx, g.ny, g.nz, 11)
    src = _src(g)
    x_ref, _ = dense.run_original(ds, scheme, ds.to_vec(u0), 10, src)
    u, _ = oracle.run(scheme, form, g, u0, 10, src)
    scale = np.sqrt(ds.w)
    err = np.linalg.norm((ds.to_vec(u) - x_ref) * scale) / np.linalg.norm(x_ref * scale)
    assert err < 1e-12, err


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_dense_fundamental_equals_original(scheme):
    g = grid4(seed=6, cfl=20.0)
    ds = dense.DenseSystem(g)
    x0 = ds.to_vec(W.random_fields(g.nx, g.ny, g.nz, 12))
    xo, to = dense.run_original(ds, scheme, x0, 12, _src(g))
    xf, tf = dense.run_fundamental(ds, scheme, x0, 12, _src(g))
    scale = np.sqrt(ds.w)
    assert np.linalg.norm((xf - xo) * scale) / np.linalg.norm(xo * scale) < 1e-12
    assert np.allclose(to, tf, rtol=1e-12)


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
@pytest.mark.parametrize("cfl", [1.0, 20.0])
def test_energy_invariant_conserved(scheme, cfl):
    nx, ny, nz = 9, 8, 7
    eps = W.random_box_eps(nx, ny, nz, seed=9, nboxes=6)
    g = yee.Grid(nx, ny, nz, 1e-3, 1e-3, 1e-3, yee.cfl_dt(1e-3, 1e-3, 1e-3, cfl), eps, order=4)
    u0 = W.random_fields(nx, ny, nz, 10)
    _, tr = oracle.run(scheme, "fundamental", g, u0, 30, None, 1)
    tr = np.array(tr)
    assert np.abs(tr - tr[0]).max() / tr[0] < 1e-12


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_cavity_mode_evolution_matches_6x6_matrix_power(scheme):
    nx, ny, nz, dx, dy, dz = 10, 8, 9, 1e-3, 1.1e-3, 0.9e-3
    mnp = (2, 1, 3)
    dt = yee.cfl_dt(dx, dy, dz, 6.0)
    g = yee.Grid(nx, ny, nz, dx, dy, dz, dt, order=4)
    a = np.random.default_rng(4).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(nx, ny, nz, dx, dy, dz, *mnp, order=4)
    M = an.scheme_matrix(scheme, A6, B6, dt)
    N = 20
    amp = np.linalg.matrix_power(M, N) @ a
    if scheme == "lod2":
        Min, Mout = an.lod2_io(B6, dt)
        amp = Mout @ np.linalg.matrix_power(M, N) @ Min @ a
    ref = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, amp)
    u0 = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, a)
    for form in oracle.FORMS:
        u, _ = oracle.run(scheme, form, g, u0, N)
        assert yee.weighted_rel_l2(u, ref, g) < 1e-12


@pytest.mark.parametrize("cfl", [1.0, 20.0])
@pytest.mark.parametrize("mnp", [(1, 1, 1), (5, 3, 7)])
def test_adi_dispersion_closed_form(cfl, mnp):
    n, h = 24, 1e-3
    dt = yee.cfl_dt(h, h, h, cfl)
    A6, B6 = an.mode_matrices(n, n, n, h, h, h, *mnp, order=4)
    ev = np.linalg.eigvals(an.scheme_matrix("adi", A6, B6, dt))
    assert np.allclose(np.abs(ev), 1.0, atol=1e-12)
    cosw = an.adi_dispersion_cos(n, n, n, h, h, h, *mnp, dt, order=4)
    re = np.sort(ev.real)
    assert abs(re[0] - cosw) < 1e-12 and abs(re[1] - cosw) < 1e-12


def test_spatial_order_four():
    """Semi-discrete frequency of a cavity mode (eigenvalues of the 6x6 A + B
    that the oracle's operators reproduce) against the exact resonance, on a
    box of fixed size refined twice: the error falls 16-fold per halving with
    the fourth-order differences (4-fold with the Yee ones)."""
    L = 24e-3
    mnp = (3, 2, 1)
    exact = an.C0 * math.pi * math.sqrt(sum((m / L) ** 2 for m in mnp))
    ratios = {}
    for order in (2, 4):
        errs = []
        for n in (12, 24, 48):
            h = L / n
            A6, B6 = an.mode_matrices(n, n, n, h, h, h, *mnp, order=order)
            w = np.max(np.abs(np.linalg.eigvals(A6 + B6).imag))
            errs.append(abs(w - exact) / exact)
        ratios[order] = (errs[0] / errs[1], errs[1] / errs[2])
    assert all(3.8 < r < 4.2 for r in ratios[2]), ratios
    assert all(15.0 < r < 17.0 for r in ratios[4]), ratios


@pytest.mark.parametrize("scheme", oracle.SPLITTINGS)
def test_splittings_equal_adi(scheme):
    nx, ny, nz = 8, 7, 9
    eps = W.random_box_eps(nx, ny, nz, seed=21, nboxes=5)
    g = yee.Grid(nx, ny, nz, 1e-3, 1e-3, 1e-3, yee.cfl_dt(1e-3, 1e-3, 1e-3, 8.0), eps, order=4)
    u0 = W.random_fields(nx, ny, nz, 22)
    src = Source(*W.interior_cell(nx, ny, nz, 23, margin=2), amp=1e12, t0=3 * g.dt, tau=3 * g.dt,
                 f0=1 / (10 * g.dt))
    ua, _ = oracle.run("adi", "fundamental", g, u0, 15, src)
    us, _ = oracle.run(scheme, "fundamental", g, u0, 15, src)
    assert yee.weighted_rel_l2(us, ua, g) < 1e-12
