"""Pins of the oracle's parameter-optimized 4-point difference (grid order 4
with a free outer weight b; the closing remark of Sec. III-A names
parameter-optimized operators without giving one), against things other than
the code under test:

* the difference: exact on quadratics for every b, on cubics only at the
  fourth-order b = -1/24, and its wall-folded matrices satisfy
  D_int = -D_half^T for every b;
* closed forms: PEC cavity modes stay exact eigenvectors with
  K(k) h = 2 (1 - 3b) sin(k h/2) + 2 b sin(3 k h/2), and every scheme evolves
  them as the 6x6 Cayley products with that K;
* the node-by-node dense assembly with the same weights against the
  vectorized operators and every scheme's dense formula; exact energy
  conservation;
* the least-squares choice of b: a brute-force scan of the discretized error
  integral finds the same minimum, the small-band limit is the Taylor
  (fourth-order) weight -1/24, and the optimized weight lowers the largest
  wavenumber error over its band."""
import numpy as np
import pytest

import oracle
import workloads as W
from oracle import dense, yee
from oracle.implicit import diff4_matrices
from oracle.source import Source

from . import _analytic as an

B_OPT = yee.optimized_outer(np.pi / 2)
OUTERS = [B_OPT, -0.07, -0.02]


def test_exact_on_quadratics_not_cubics():
    n, h = 14, 0.31
    x = np.arange(n + 1) * h
    mid = (np.arange(n) + 0.5) * h
    inner = slice(1, n - 1)
    for b in OUTERS + [-1.0 / 24.0]:
        w = yee.stencil4(b)
        for f, df, exact in ((lambda t: 0.7 * t ** 2 - 1.3 * t + 0.2, lambda t: 1.4 * t - 1.3, True),
                             (lambda t: 0.4 * t ** 3 - 0.2 * t, lambda t: 1.2 * t ** 2 - 0.2, b == -1.0 / 24.0)):
            e = np.zeros((1, 1, n + 1))
            e[0, 0, :] = f(x)
            got = yee.diff4_to_half(e, "x", h, w)[0, 0]
            err = np.abs(got[inner] - df(mid)[inner]).max()
            assert (err < 1e-12) == exact, (b, err)


@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_image_matrices_are_negative_transposes_for_any_outer_weight(n):
    for b in OUTERS:
        Dh, Di = diff4_matrices(n, 0.6, yee.stencil4(b))
        assert np.allclose(Di, -Dh.T, rtol=0, atol=1e-15)


@pytest.mark.parametrize("mnp", [(1, 1, 1), (3, 2, 4)])
def test_operators_on_cavity_mode(mnp):
    nx, ny, nz, dx, dy, dz = 9, 7, 8, 1e-3, 1.2e-3, 0.9e-3
    for b in OUTERS:
        g = yee.Grid(nx, ny, nz, dx, dy, dz, 1e-12, order=4, outer=b)
        a = np.random.default_rng(3).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
        A6, B6 = an.mode_matrices(nx, ny, nz, dx, dy, dz, *mnp, order=4, outer=b)
        u = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, a)
        for name, M6 in (("A", A6), ("B", B6)):
            ref = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, M6 @ a)
            got = yee.apply_operator(name, u, g)
            for x, y in zip(got, ref):
                assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max() + 1e-300


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_cavity_mode_evolution_matches_6x6_matrix_power(scheme):
    nx, ny, nz, dx, dy, dz = 10, 8, 9, 1e-3, 1.1e-3, 0.9e-3
    mnp = (2, 1, 3)
    dt = yee.cfl_dt(dx, dy, dz, 6.0)
    g = yee.Grid(nx, ny, nz, dx, dy, dz, dt, order=4, outer=B_OPT)
    a = np.random.default_rng(4).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(nx, ny, nz, dx, dy, dz, *mnp, order=4, outer=B_OPT)
    M = an.scheme_matrix(scheme, A6, B6, dt)
    N = 15
    amp = np.linalg.matrix_power(M, N) @ a
    if scheme == "lod2":
        Min, Mout = an.lod2_io(B6, dt)
        amp = Mout @ np.linalg.matrix_power(M, N) @ Min @ a
    ref = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, amp)
    u0 = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, a)
    for form in oracle.FORMS:
        u, _ = oracle.run(scheme, form, g, u0, N)
        assert yee.weighted_rel_l2(u, ref, g) < 1e-12


def _grid(seed, cfl=5.0):
    rng = np.random.default_rng(seed)
    nx, ny, nz, sp = 5, 4, 6, (1e-3, 1.2e-3, 0.8e-3)
    return yee.Grid(nx, ny, nz, *sp, yee.cfl_dt(*sp, cfl), rng.uniform(1, 12, (nz, ny, nx)),
                    rng.uniform(1, 3, (nz, ny, nx)), order=4, outer=B_OPT)


def test_dense_operators_equal_vectorized_and_skew_adjoint():
    g = _grid(1)
    ds = dense.DenseSystem(g)
    u = yee.clean(W.random_fields(g.nx, g.ny, g.nz, 2), g)
    Wm = np.diag(ds.w)
    for name in ("A", "B"):
        M = ds.op(name)
        got = ds.to_vec(yee.apply_operator(name, u, g))
        ref = M @ ds.to_vec(u)
        assert np.allclose(got, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
        assert np.abs(M.T @ Wm + Wm @ M).max() <= 1e-14 * np.abs(Wm @ M).max()


@pytest.mark.parametrize("scheme", ["adi", "lod1", "ss2", "lod2"])
@pytest.mark.parametrize("form", oracle.FORMS)
def test_scheme_matches_dense_formula(scheme, form):
    g = _grid(5)
    ds = dense.DenseSystem(g)
    u0 = W.random_fields(g.nx, g.ny, g.nz, 11)
    src = Source(1, 1, 2, amp=1e12, t0=2 * g.dt, tau=3 * g.dt, f0=1 / (8 * g.dt))
    x_ref, _ = dense.run_original(ds, scheme, ds.to_vec(u0), 8, src)
    u, _ = oracle.run(scheme, form, g, u0, 8, src)
    scale = np.sqrt(ds.w)
    err = np.linalg.norm((ds.to_vec(u) - x_ref) * scale) / np.linalg.norm(x_ref * scale)
    assert err < 1e-12, err


def test_energy_conserved_at_cfl_20():
    nx, ny, nz = 9, 8, 7
    g = yee.Grid(nx, ny, nz, 1e-3, 1e-3, 1e-3, yee.cfl_dt(1e-3, 1e-3, 1e-3, 20.0),
                 W.random_box_eps(nx, ny, nz, seed=9, nboxes=6), order=4, outer=B_OPT)
    _, tr = oracle.run("adi", "fundamental", g, W.random_fields(nx, ny, nz, 10), 25, None, 1)
    tr = np.array(tr)
    assert np.abs(tr - tr[0]).max() / tr[0] < 1e-12


def test_optimized_outer_weight():
    tm = np.pi / 2
    theta = np.linspace(0.0, tm, 20001)
    bs = np.linspace(-0.08, -0.02, 6001)                 # scan step 1e-5
    err = [np.trapezoid((yee.modified_wavenumber4(b, theta) - theta) ** 2, theta) for b in bs]
    assert abs(bs[int(np.argmin(err))] - B_OPT) <= 2e-5
    # a narrow band recovers the Taylor weight of the fourth-order difference
    assert abs(yee.optimized_outer(0.05) + 1.0 / 24.0) < 1e-5
    # the optimized weight lowers the largest wavenumber error over its band
    e_opt = np.abs(yee.modified_wavenumber4(B_OPT, theta) - theta).max()
    e_4 = np.abs(yee.modified_wavenumber4(-1.0 / 24.0, theta) - theta).max()
    assert e_opt < 0.5 * e_4
