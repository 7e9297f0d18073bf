"""Pins of the FP64 oracle against things other than itself.

* brute force: numpy.linalg.solve of every tridiagonal and every implicit stage;
* the dense matrix formulae of Sec. II (operators assembled node by node);
* closed forms: the PEC cavity modes (exact eigenvectors of the Yee operators)
  and the closed-form ADI dispersion relation;
* invariants: skew-adjointness of A and B, exact energy conservation of the
  Cayley sub-steps, the fundamental == original equivalence (Sec. II-A
  closing paragraph, Sec. II-B construction), the ADI <-> LOD link (Sec. II-E),
  the D'Yakonov and Douglas-Gunn splittings against Peaceman-Rachford (Sec. II-E),
  Crank-Nicolson (fundamental == classical, the closed-form Cayley phase);
* the temporal orders of Table I (2, 1, 2, 2).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import dense, yee
from oracle.implicit import solve_implicit
from oracle.source import Source
from oracle.tridiag import thomas

from . import _analytic as an


def small_grid(nx=4, ny=3, nz=5, cfl=4.0, seed=0, mu=True, spacing=(1e-3, 1.2e-3, 0.8e-3)):
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1, 12, (nz, ny, nx))
    mur = rng.uniform(1, 3, (nz, ny, nx)) if mu else None
    dt = yee.cfl_dt(*spacing, cfl)
    return yee.Grid(nx, ny, nz, *spacing, dt, eps, mur)


# --------------------------------------------------------------------------
# tridiagonal solver
# --------------------------------------------------------------------------

@pytest.mark.parametrize("beta", [1 / 24, 4 / 24 * 25, 400 / 24])
def test_thomas_matches_dense_solve(beta):
    rng = np.random.default_rng(1)
    n, lines = 17, 5
    a = -beta * rng.uniform(0.5, 1.5, (lines, n))
    c = -beta * rng.uniform(0.5, 1.5, (lines, n))
    b = 0.5 - a - c  # the fundamental scaling: 1/2 + sum of |off-diagonals|
    d = rng.standard_normal((lines, n))
    x = thomas(a, b, c, d)
    for L in range(lines):
        M = np.diag(b[L]) + np.diag(a[L, 1:], -1) + np.diag(c[L, :-1], 1)
        ref = np.linalg.solve(M, d[L])
        assert np.allclose(x[L], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())


# --------------------------------------------------------------------------
# operators
# --------------------------------------------------------------------------

def test_dense_operators_skew_adjoint_in_energy_norm():
    g = small_grid()
    ds = dense.DenseSystem(g)
    Wm = np.diag(ds.w)
    for M in (ds.A, ds.B):
        assert np.abs(M.T @ Wm + Wm @ M).max() <= 1e-14 * np.abs(Wm @ M).max()


@pytest.mark.parametrize("mnp", [(1, 1, 1), (2, 1, 3), (3, 2, 1)])
def test_operators_on_cavity_mode(mnp):
    nx, ny, nz, dx, dy, dz = 8, 6, 7, 1e-3, 1.3e-3, 0.9e-3
    g = yee.Grid(nx, ny, nz, dx, dy, dz, 1e-12)
    a = np.random.default_rng(2).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(nx, ny, nz, dx, dy, dz, *mnp)
    u = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, a)
    ds = dense.DenseSystem(g)
    for name, M6 in (("A", A6), ("B", B6)):
        ref = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, M6 @ a)
        got = yee.apply_operator(name, u, g)
        for x, y in zip(got, ref):
            assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1e-300) + 1e-300
        gd = ds.op(name) @ ds.to_vec(u)
        assert np.allclose(gd, ds.to_vec(ref), rtol=1e-12, atol=1e-12 * np.abs(gd).max())


# --------------------------------------------------------------------------
# implicit stages: line elimination vs dense solve
# --------------------------------------------------------------------------

@pytest.mark.parametrize("op", ["A", "B"])
@pytest.mark.parametrize("theta_scale", [0.5, 0.25, -0.25])
def test_implicit_stage_matches_dense(op, theta_scale):
    g = small_grid(seed=3)
    ds = dense.DenseSystem(g)
    theta = theta_scale * g.dt
    f = W.random_fields(g.nx, g.ny, g.nz, 7)
    got = solve_implicit(op, yee.PAIRS[op], yee.clean(f, g), theta, g)
    ref = np.linalg.solve(np.eye(ds.n) - theta * ds.op(op), ds.to_vec(f))
    assert np.allclose(ds.to_vec(got), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # static normal H untouched
    for n, c in enumerate(yee.COMPONENTS):
        if c[0] == "H":
            st = ~yee.dynamic_mask(c, g)
            assert np.array_equal(got[n][st], f[n][st])


# --------------------------------------------------------------------------
# whole schemes: component form vs dense matrix formula
# --------------------------------------------------------------------------

def _src(g):
    return Source(1, 1, 2, amp=1e12, t0=2 * g.dt, tau=3 * g.dt, f0=1 / (8 * g.dt))


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
@pytest.mark.parametrize("form", oracle.FORMS)
def test_scheme_matches_dense_formula(scheme, form):
    g = small_grid(seed=5)
    ds = dense.DenseSystem(g)
    u0 = W.random_fields(g.nx, g.ny, g.nz, 11)
    src = _src(g)
    x_ref, _ = dense.run_original(ds, scheme, ds.to_vec(u0), 12, src)
    u, _ = oracle.run(scheme, form, g, u0, 12, src)
    got = ds.to_vec(u)
    scale = np.sqrt(ds.w)
    err = np.linalg.norm((got - x_ref) * scale) / np.linalg.norm(x_ref * scale)
    assert err < 1e-12, err


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_dense_fundamental_equals_original(scheme):
    """The paper's algebra (proveADIi/a/c; the LOD auxiliary v) on matrices."""
    g = small_grid(seed=6, cfl=20.0)
    ds = dense.DenseSystem(g)
    x0 = ds.to_vec(W.random_fields(g.nx, g.ny, g.nz, 12))
    src = _src(g)
    xo, to = dense.run_original(ds, scheme, x0, 15, src)
    xf, tf = dense.run_fundamental(ds, scheme, x0, 15, src)
    scale = np.sqrt(ds.w)
    assert np.linalg.norm((xf - xo) * scale) / np.linalg.norm(xo * scale) < 1e-12
    assert np.allclose(to, tf, rtol=1e-12)


@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_fundamental_equals_conventional_larger_grid(scheme):
    nx, ny, nz = 12, 10, 11
    eps = W.random_box_eps(nx, ny, nz, seed=2, nboxes=8)
    g = yee.Grid(nx, ny, nz, 1e-3, 1e-3, 1e-3, yee.cfl_dt(1e-3, 1e-3, 1e-3, 10.0), eps)
    u0 = W.random_fields(nx, ny, nz, 3)
    src = Source(*W.interior_cell(nx, ny, nz, 4, margin=2), amp=1e12, t0=4 * g.dt,
                 tau=4 * g.dt, f0=1 / (10 * g.dt))
    uf, tf = oracle.run(scheme, "fundamental", g, u0, 30, src, 1)
    uc, tc = oracle.run(scheme, "conventional", g, u0, 30, src, 1)
    assert yee.weighted_rel_l2(uf, uc, g) < 1e-11
    assert np.allclose(tf, tc, rtol=1e-11)


# --------------------------------------------------------------------------
# invariants
# --------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", oracle.SCHEMES)
@pytest.mark.parametrize("cfl", [1.0, 5.0, 20.0])
def test_energy_invariant_conserved(scheme, cfl):
    nx, ny, nz = 9, 8, 7
    eps = W.random_box_eps(nx, ny, nz, seed=9, nboxes=6)
    g = yee.Grid(nx, ny, nz, 1e-3, 1e-3, 1e-3, yee.cfl_dt(1e-3, 1e-3, 1e-3, cfl), eps)
    u0 = W.random_fields(nx, ny, nz, 10)
    u, tr = oracle.run(scheme, "fundamental", g, u0, 40, None, 1)
    tr = np.array(tr)
    assert np.abs(tr - tr[0]).max() / tr[0] < 1e-12
    if scheme == "adi":
        # W(u^n) <= W((I + dt/2 B) u^n) = 4 * invariant: bounded for any CFL
        assert yee.energy(u, g) <= 4 * tr[-1] * (1 + 1e-12)


def test_adi_lod_link():
    """Sec. II-E: LOD1 fundamental iterations started from
    u^0 = (1/2 I + dt/4 B) v^0 give v^{n+1} (from (fastLODc)) = ADI fields."""
    from oracle import fundamental
    g = small_grid(nx=6, ny=5, nz=7, seed=12, cfl=8.0)
    phi0 = yee.clean(W.random_fields(g.nx, g.ny, g.nz, 13), g)
    bu = yee.apply_operator("B", phi0, g)
    U = [0.5 * a + 0.25 * g.dt * b for a, b in zip(phi0, bu)]
    adi = fundamental.FundamentalADI(phi0, g)
    for n in range(10):
        U = fundamental.lod_substep(U, "A", 0.5 * g.dt, g)
        Unew = fundamental.lod_substep(U, "B", 0.5 * g.dt, g)
        V = [a + b for a, b in zip(Unew, U)]  # v^{n+1} = u^{n+1} + u^{n+1/2}
        U = Unew
        adi.step()
        assert yee.weighted_rel_l2(V, adi.fields(), g) < 1e-13


# --------------------------------------------------------------------------
# D'Yakonov and Douglas-Gunn splittings (Sec. II-E)
# --------------------------------------------------------------------------

def _wrel(ds, a, b):
    scale = np.sqrt(ds.w)
    return np.linalg.norm((a - b) * scale) / np.linalg.norm(b * scale)


@pytest.mark.parametrize("scheme", oracle.SPLITTINGS)
@pytest.mark.parametrize("cfl", [2.0, 20.0])
def test_dense_splitting_original_equals_peaceman_rachford(scheme, cfl):
    """(orgDY) and the delta formulation give the Peaceman-Rachford fields of
    (clsADI): (I - dt/2 A)^-1 and (I + dt/2 A) commute, and the delta form is
    the same product written for the increment.  A wrong sign or a dropped
    operator in either formula breaks the equality."""
    g = small_grid(seed=21, cfl=cfl)
    ds = dense.DenseSystem(g)
    x0 = ds.to_vec(W.random_fields(g.nx, g.ny, g.nz, 22))
    x_pr, _ = dense.run_original(ds, "adi", x0, 12)
    x, mids = dense.run_splitting_original(ds, scheme, x0, 12)
    assert len(mids) == 12
    assert _wrel(ds, x, x_pr) < 1e-12


@pytest.mark.parametrize("scheme", oracle.SPLITTINGS)
def test_dense_splitting_fundamental_equals_original(scheme):
    """(fastDY) with its input reproduces (orgDY) step by step, including the
    intermediate u* = 2 v^{n+1/2}; (fasterADI) with the increments of (fastDGo)
    reproduces the delta formulation's du* and du at every step."""
    g = small_grid(seed=23, cfl=12.0)
    ds = dense.DenseSystem(g)
    x0 = ds.to_vec(W.random_fields(g.nx, g.ny, g.nz, 24))
    xo, mo = dense.run_splitting_original(ds, scheme, x0, 10)
    xf, mf = dense.run_splitting_fundamental(ds, scheme, x0, 10)
    assert _wrel(ds, xf, xo) < 1e-12
    for a, b in zip(mf, mo):
        if scheme == "dy":
            assert _wrel(ds, a, b) < 1e-12
        else:
            assert _wrel(ds, a[0], b[0]) < 1e-11 and _wrel(ds, a[1], b[1]) < 1e-11


def test_dyakonov_intermediate_is_original_adi_auxiliary():
    """u* of (orgDY) equals (I + dt/2 A) u^{n+1/2} of the original ADI
    (orgADIc), and differs from u^{n+1/2} itself."""
    g = small_grid(seed=25, cfl=6.0)
    ds = dense.DenseSystem(g)
    I, h = np.eye(ds.n), 0.5 * g.dt
    x0 = ds.to_vec(W.random_fields(g.nx, g.ny, g.nz, 26))
    _, mids = dense.run_splitting_original(ds, "dy", x0, 1)
    u_half = np.linalg.solve(I - h * ds.A, (I + h * ds.B) @ x0)
    assert _wrel(ds, mids[0], (I + h * ds.A) @ u_half) < 1e-12
    assert _wrel(ds, mids[0], u_half) > 1e-3


@pytest.mark.parametrize("scheme", oracle.SPLITTINGS)
@pytest.mark.parametrize("form", oracle.FORMS)
def test_splitting_component_form_matches_dense(scheme, form):
    g = small_grid(seed=27, cfl=8.0)
    ds = dense.DenseSystem(g)
    u0 = W.random_fields(g.nx, g.ny, g.nz, 28)
    x_ref, _ = dense.run_splitting_original(ds, scheme, ds.to_vec(u0), 9)
    u, _ = oracle.run(scheme, form, g, u0, 9)
    assert _wrel(ds, ds.to_vec(u), x_ref) < 1e-12


@pytest.mark.parametrize("scheme", oracle.SPLITTINGS)
def test_splitting_fields_equal_adi_larger_grid(scheme):
    nx, ny, nz = 12, 10, 11
    eps = W.random_box_eps(nx, ny, nz, seed=2, nboxes=8)
    g = yee.Grid(nx, ny, nz, 1e-3, 1e-3, 1e-3, yee.cfl_dt(1e-3, 1e-3, 1e-3, 10.0), eps)
    u0 = W.random_fields(nx, ny, nz, 3)
    ua, ta = oracle.run("adi", "conventional", g, u0, 25, None, 1)
    for form in oracle.FORMS:
        u, t = oracle.run(scheme, form, g, u0, 25, None, 1)
        assert yee.weighted_rel_l2(u, ua, g) < 1e-12
        assert np.allclose(t, ta, rtol=1e-12)
        assert np.abs(np.array(t) - t[0]).max() / t[0] < 1e-12   # conserved


@pytest.mark.parametrize("scheme", oracle.SPLITTINGS)
def test_splitting_with_source_equals_adi(scheme):
    """With a source, the fundamental D'Yakonov and Douglas-Gunn forms (the
    ADI convention: g in the auxiliary subtraction, g/2 in the unscaled
    variables of (fastDY)) give the fields of the original ADI with the same
    source, dense and component form; the original splittings take none."""
    g = small_grid(seed=29, cfl=6.0)
    ds = dense.DenseSystem(g)
    u0 = W.random_fields(g.nx, g.ny, g.nz, 30)
    src = _src(g)
    x_adi, _ = dense.run_original(ds, "adi", ds.to_vec(u0), 9, src)
    x, _ = dense.run_splitting_fundamental(ds, scheme, ds.to_vec(u0), 9, src)
    assert _wrel(ds, x, x_adi) < 1e-12
    u, _ = oracle.run(scheme, "fundamental", g, u0, 9, src)
    assert _wrel(ds, ds.to_vec(u), x_adi) < 1e-12
    with pytest.raises(ValueError):
        oracle.run(scheme, "conventional", g, u0, 2, src)


# --------------------------------------------------------------------------
# Crank-Nicolson without factorization (Sec. II-E)
# --------------------------------------------------------------------------

def test_sparse_assembly_equals_dense():
    g = small_grid(seed=31, cfl=8.0)
    d, s_ = dense.DenseSystem(g), dense.DenseSystem(g, sparse=True)
    assert np.array_equal(d.A, s_.A.toarray()) and np.array_equal(d.B, s_.B.toarray())


@pytest.mark.parametrize("cfl", [2.0, 20.0])
def test_cn_fundamental_equals_original_dense(cfl):
    """[1/2 I - dt/4 (A+B)] v = u, u' = v - u against the classical form, both
    written here with dense solves on the assembled matrices."""
    from oracle import crank_nicolson as cn
    g = small_grid(seed=33, cfl=cfl)
    ds = dense.DenseSystem(g)
    x0 = ds.to_vec(W.random_fields(g.nx, g.ny, g.nz, 34))
    I, K = np.eye(ds.n), ds.A + ds.B
    x_ref = x0.copy()
    for _ in range(8):
        x_ref = np.linalg.solve(I - 0.5 * g.dt * K, (I + 0.5 * g.dt * K) @ x_ref)
    xs = dense.DenseSystem(g, sparse=True)
    for form in oracle.FORMS:
        x, tr = cn.run(xs, x0, 8, form)
        assert _wrel(ds, x, x_ref) < 1e-12
        assert np.abs(np.array(tr) / tr[0] - 1).max() < 1e-12


@pytest.mark.parametrize("mnp", [(1, 1, 1), (2, 1, 3)])
@pytest.mark.parametrize("cfl", [1.0, 8.0])
def test_cn_cavity_mode_closed_form_phase(mnp, cfl):
    """On a PEC cavity mode the oracle's step is the 6x6 Cayley factor of
    dt (A + B)/2, whose rotation angle is 2 atan(w dt / 2) with w the Yee
    frequency (closed form, not from the oracle)."""
    nx, ny, nz, dx, dy, dz = 10, 8, 9, 1e-3, 1.1e-3, 0.9e-3
    dt = yee.cfl_dt(dx, dy, dz, cfl)
    g = yee.Grid(nx, ny, nz, dx, dy, dz, dt)
    a = np.random.default_rng(6).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(nx, ny, nz, dx, dy, dz, *mnp)
    C = an.cayley(A6 + B6, 0.5 * dt)
    ang = np.sort(np.abs(np.angle(np.linalg.eigvals(C))))
    phi = an.cn_phase(nx, ny, nz, dx, dy, dz, *mnp, dt)
    assert np.allclose(ang, [0, 0, phi, phi, phi, phi], atol=1e-10)
    N = 12
    u0 = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, a)
    ref = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, np.linalg.matrix_power(C, N) @ a)
    for form in oracle.FORMS:
        u, _ = oracle.run("cn", form, g, u0, N)
        assert yee.weighted_rel_l2(u, ref, g) < 1e-12


def test_cn_schur_complement_is_spd_and_equivalent():
    """The E-side reduction the library solves by CG: with theta = dt/2 and
    (A + B) = [[0, eps^-1 K], [-mu^-1 K^T, 0]] on the dynamic samples, the
    matrix S = eps + theta^2 K mu^-1 K^T is symmetric positive definite, and
    S v_E = 2 eps u_E + 2 theta K u_H with v_H = 2 u_H - theta mu^-1 K^T v_E
    solves [1/2 I - dt/4 (A + B)] v = u."""
    g = small_grid(seed=35, cfl=9.0)
    ds = dense.DenseSystem(g)
    X = ds.A + ds.B
    ie = np.array([c[0] == "E" for c, *_ in ds.nodes])
    ih = ~ie
    eps, mu = ds.w[ie], ds.w[ih]
    K = eps[:, None] * X[np.ix_(ie, ih)]          # eps^-1 K is the E-H block
    KT = -mu[:, None] * X[np.ix_(ih, ie)]         # -mu^-1 K^T is the H-E block
    assert np.allclose(K.T, KT, atol=1e-12 * np.abs(K).max())
    th = 0.5 * g.dt
    S = np.diag(eps) + th * th * K @ (KT / mu[:, None])
    assert np.allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(S).max())
    assert np.linalg.eigvalsh(S).min() > 0
    u = ds.to_vec(W.random_fields(g.nx, g.ny, g.nz, 36))
    uE, uH = u[ie], u[ih]
    vE = np.linalg.solve(S, 2 * eps * uE + 2 * th * K @ uH)
    vH = 2 * uH - th * (KT @ vE) / mu
    v = np.zeros_like(u)
    v[ie], v[ih] = vE, vH
    v_ref = np.linalg.solve(0.5 * np.eye(ds.n) - 0.25 * g.dt * X, u)
    assert _wrel(ds, v, v_ref) < 1e-12


def test_cn_temporal_order_two():
    nx, ny, nz, h = 8, 7, 6, 1e-3
    a = np.random.default_rng(7).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(nx, ny, nz, h, h, h, 1, 1, 1)
    T = 40 * yee.cfl_dt(h, h, h, 1.0)
    ref = an.exact(A6, B6, T) @ a
    w = np.r_[[an.EPS0] * 3, [an.MU0] * 3]
    errs = []
    for N in (640, 1280, 2560):
        x = np.linalg.matrix_power(an.cayley(A6 + B6, 0.5 * T / N), N) @ a
        errs.append(math.sqrt(np.sum(w * (x - ref) ** 2) / np.sum(w * ref ** 2)))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(s_ - 2) < 0.1 for s_ in slopes), (errs, slopes)


def test_cn_energy_conserved():
    nx, ny, nz = 9, 8, 7
    eps = W.random_box_eps(nx, ny, nz, seed=9, nboxes=6)
    g = yee.Grid(nx, ny, nz, 1e-3, 1e-3, 1e-3, yee.cfl_dt(1e-3, 1e-3, 1e-3, 20.0), eps)
    u0 = W.random_fields(nx, ny, nz, 10)
    u, tr = oracle.run("cn", "fundamental", g, u0, 30, None, 1)
    assert len(tr) == 31 and np.abs(np.array(tr) / tr[0] - 1).max() < 1e-12
    assert abs(tr[-1] / yee.energy(u, g) - 1) < 1e-13   # W over all samples


def test_cn_with_source_fundamental_equals_classical():
    """With a source (one term per step, at its middle): the fundamental form,
    which adds g/2 to u^n, against the classical form with g on its right
    side written here with dense solves."""
    from oracle import crank_nicolson as cn
    g = small_grid(seed=43, cfl=6.0)
    ds = dense.DenseSystem(g)
    x0 = ds.to_vec(W.random_fields(g.nx, g.ny, g.nz, 44))
    src = _src(g)
    I, K = np.eye(ds.n), ds.A + ds.B
    x_ref = x0.copy()
    for n in range(7):
        gv = ds.src_vec(src, src.g(0.5 * g.dt, (n + 0.5) * g.dt))
        x_ref = np.linalg.solve(I - 0.5 * g.dt * K, (I + 0.5 * g.dt * K) @ x_ref + gv)
    xs = dense.DenseSystem(g, sparse=True)
    for form in oracle.FORMS:
        x, _ = cn.run(xs, x0, 7, form, src)
        assert _wrel(ds, x, x_ref) < 1e-12


# --------------------------------------------------------------------------
# closed forms: cavity modes and dispersion
# --------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", oracle.SCHEMES)
def test_cavity_mode_evolution_matches_6x6_matrix_power(scheme):
    nx, ny, nz, dx, dy, dz = 10, 8, 9, 1e-3, 1.1e-3, 0.9e-3
    mnp = (2, 1, 3)
    dt = yee.cfl_dt(dx, dy, dz, 6.0)
    g = yee.Grid(nx, ny, nz, dx, dy, dz, dt)
    a = np.random.default_rng(4).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(nx, ny, nz, dx, dy, dz, *mnp)
    M = an.scheme_matrix(scheme, A6, B6, dt)
    N = 25
    amp = np.linalg.matrix_power(M, N) @ a
    if scheme == "lod2":
        Min, Mout = an.lod2_io(B6, dt)
        amp = Mout @ np.linalg.matrix_power(M, N) @ Min @ a
    ref = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, amp)
    u0 = an.mode_fields(nx, ny, nz, dx, dy, dz, *mnp, a)
    for form in oracle.FORMS:
        u, _ = oracle.run(scheme, form, g, u0, N)
        assert yee.weighted_rel_l2(u, ref, g) < 1e-12


@pytest.mark.parametrize("cfl", [1.0, 4.0, 20.0])
@pytest.mark.parametrize("mnp", [(1, 1, 0), (1, 1, 1), (2, 1, 1), (5, 3, 7)])
def test_adi_dispersion_closed_form(cfl, mnp):
    """Eigenvalues of the ADI amplification: {1, 1, e^{+-i w dt} (x2)} with the
    closed-form cos(w dt); as dt -> 0 the frequency tends to the Yee one."""
    n, h = 24, 1e-3
    dt = yee.cfl_dt(h, h, h, cfl)
    A6, B6 = an.mode_matrices(n, n, n, h, h, h, *mnp)
    M = an.scheme_matrix("adi", A6, B6, dt)
    ev = np.linalg.eigvals(M)
    assert np.allclose(np.abs(ev), 1.0, atol=1e-12)  # non-dissipative
    cosw = an.adi_dispersion_cos(n, n, n, h, h, h, *mnp, dt)
    re = np.sort(ev.real)
    assert abs(re[0] - cosw) < 1e-12 and abs(re[1] - cosw) < 1e-12
    assert np.all(re >= cosw - 1e-12)


def test_dispersion_worked_example_24cube():
    """24^3 cavity, 1 mm, CFL 4: ADI frequency of the (1,1,0) mode vs the Yee
    semi-discrete and the analytic resonance."""
    n, h = 24, 1e-3
    dt = yee.cfl_dt(h, h, h, 4.0)
    cosw = an.adi_dispersion_cos(n, n, n, h, h, h, 1, 1, 0, dt)
    f_adi = math.acos(cosw) / (2 * math.pi * dt)
    _, K = an.wavenumbers(n, n, n, h, h, h, 1, 1, 0)
    f_yee = an.C0 * math.sqrt(sum(k * k for k in K)) / (2 * math.pi)
    f_exact = an.C0 / 2 * math.sqrt(2) / (n * h)
    assert f_adi < f_yee < f_exact  # ADI slows the wave; Yee slows it less
    assert abs(f_exact - 8.83272e9) < 1e4
    assert abs(f_adi - 8.74373e9) < 1e4 and abs(f_yee - 8.82642e9) < 1e4


# --------------------------------------------------------------------------
# temporal orders (Table I, last row)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("scheme,order", [("adi", 2), ("lod1", 1), ("ss2", 2), ("lod2", 2)])
def test_temporal_order(scheme, order):
    """Global error at a fixed time T against the exact semi-discrete evolution
    expm(T (A + B)) of a cavity mode.  The oracle reproduces the 6x6 scheme
    matrices to 1e-12 (test above), so these orders are the oracle's orders."""
    nx, ny, nz, h = 8, 7, 6, 1e-3
    mnp = (1, 1, 1)
    a = np.random.default_rng(5).standard_normal(6) * np.r_[1, 1, 1, 1 / 377, 1 / 377, 1 / 377]
    A6, B6 = an.mode_matrices(nx, ny, nz, h, h, h, *mnp)
    T = 40 * yee.cfl_dt(h, h, h, 1.0)
    ref = an.exact(A6, B6, T) @ a
    w = np.r_[[an.EPS0] * 3, [an.MU0] * 3]
    errs = []
    for N in (640, 1280, 2560):
        dt = T / N
        M = an.scheme_matrix(scheme, A6, B6, dt)
        if scheme == "lod2":
            Min, Mout = an.lod2_io(B6, dt)
            x = Mout @ np.linalg.matrix_power(M, N) @ Min @ a
        else:
            x = np.linalg.matrix_power(M, N) @ a
        errs.append(math.sqrt(np.sum(w * (x - ref) ** 2) / np.sum(w * ref ** 2)))
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(abs(s - order) < 0.1 for s in slopes), (errs, slopes)
