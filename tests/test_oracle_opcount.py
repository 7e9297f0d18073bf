"""Table I of Sec. IV against the operation-counting form of the oracle.

`oracle.opcount` writes every procedure of the main iteration of ADI, LOD1/SS1,
SS2 and LOD2, original and new, per node with precomputed factors, and counts
the M/D and A/S its right-hand sides take.  These tests check
* the counts, for-loops and efficiency gains against the values Table I prints
  (tests/golden/table1_flops.json);
* that the counted expressions compute the schemes: their values at interior
  nodes of a random grid (random eps_r per cell, anisotropic cells) equal the
  right-hand sides formed from the operator form of eqs. (AMat), (bd) with
  oracle.yee.apply_operator."""
import json
import os

import numpy as np
import pytest

from oracle import opcount as oc
from oracle.yee import CIDX, COMPONENTS, PAIRS, Grid, apply_operator, cfl_dt

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_flops.json")
SCHEMES = ("ADI", "LOD1", "SS2", "LOD2")
KEYS = ("implicit_md", "implicit_as", "explicit_md", "explicit_as", "total_md", "total_as", "total")


@pytest.fixture(scope="module")
def table1():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def grid():
    rng = np.random.default_rng(21)
    nx, ny, nz = 6, 5, 7
    dx, dy, dz = 1.0e-3, 1.3e-3, 0.8e-3
    g = Grid(nx, ny, nz, dx, dy, dz, cfl_dt(dx, dy, dz, 2.0), eps_r=rng.uniform(1, 12, (nz, ny, nx)))
    return g, oc.random_arrays(g, rng)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("form", ["original", "new"])
def test_counts_match_table1(table1, grid, scheme, form):
    g, arrays = grid
    c = oc.step_counts(scheme, form, g, arrays, (3, 2, 3))
    want = table1[scheme][form]
    for k in KEYS:
        assert c[k] == want[k], (scheme, form, k, c[k], want[k])
    assert c["loops"] == table1[scheme]["loops"]


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("form", ["original", "new"])
def test_efficiency_gains_match_table1(table1, grid, scheme, form):
    g, arrays = grid
    ref = oc.step_counts("ADI", "original", g, arrays, (3, 2, 3))
    rhs, overall = oc.efficiency_gains(oc.step_counts(scheme, form, g, arrays, (3, 2, 3)), ref)
    want = table1[scheme][form]
    assert round(rhs, 2) == want["gain_rhs"]
    assert round(overall, 2) == want["gain_overall"]


def test_fundamental_procedure_is_21_flops(grid):
    """Every procedure of the new forms takes 21 flops per cell (Sec. IV)."""
    g, arrays = grid
    for X, Y in (("A", "B"), ("B", "A"), ("A", "A"), ("B", "B")):
        _, _, _, ti, tx = oc.procedure("new", X, Y, 0.5 * g.dt, arrays, (3, 2, 3), g)
        assert ti.md + ti.as_ + tx.md + tx.as_ == 21


def _vec(arrays, names):
    return [arrays[n] for n in names]


def _reference(form, X, Y, theta, arrays, g):
    """Right-hand sides of one procedure from the operator form: E line
    right-hand sides, H updates and (new LOD family) fields from the solution."""
    u = _vec(arrays, COMPONENTS)
    S = [arrays["S_" + c] for c in COMPONENTS[:3]] + [np.zeros(g.shape)] * 3
    XS = apply_operator(X, S, g)
    if form == "original":
        Yu = apply_operator(Y, u, g)
        w = [a + theta * b for a, b in zip(u, Yu)]
        Xw = apply_operator(X, w, g)
        rhs = {c: w[CIDX[c]] + theta * Xw[CIDX[c]] for c in COMPONENTS[:3]}
        hnew = {c: w[CIDX[c]] + theta * XS[CIDX[c]] for c in COMPONENTS[3:]}
        return rhs, hnew, {}
    if X != Y:   # new ADI: v = (E~ - e, h)
        v = [u[n] - arrays["e_" + COMPONENTS[n]] for n in range(3)] + u[3:]
        Xv = apply_operator(X, v, g)
        rhs = {c: v[CIDX[c]] + theta * Xv[CIDX[c]] for c in COMPONENTS[:3]}
        hnew = {c: u[CIDX[c]] + theta * XS[CIDX[c]] for c in COMPONENTS[3:]}
        return rhs, hnew, {}
    Xu = apply_operator(X, u, g)
    rhs = {c: u[CIDX[c]] + theta * Xu[CIDX[c]] for c in COMPONENTS[:3]}
    hnew = {c: u[CIDX[c]] + theta * XS[CIDX[c]] for c in COMPONENTS[3:]}
    enew = {c: S[CIDX[c]] - u[CIDX[c]] for c in COMPONENTS[:3]}
    return rhs, hnew, enew


@pytest.mark.parametrize("form", ["original", "new"])
@pytest.mark.parametrize("X,Y,frac", [("A", "B", 0.5), ("B", "A", 0.5), ("A", "A", 0.5), ("B", "B", 0.5),
                                      ("A", "A", 0.25)])
def test_counted_expressions_compute_the_schemes(grid, form, X, Y, frac):
    g, arrays = grid
    theta = frac * g.dt
    ref = _reference(form, X, Y, theta, arrays, g)
    for node in [(3, 2, 3), (1, 1, 1), (5, 3, 4), (2, 3, 1)]:
        got = oc.procedure(form, X, Y, theta, arrays, node, g)
        for part, want in zip(got[:3], ref):
            assert set(part) == set(want)
            for c, val in part.items():
                r = want[c][node]
                assert abs(val.v - r) <= 1e-12 * max(1.0, abs(r)), (form, X, Y, node, c, val.v, r)


def test_a_dropped_term_is_caught(grid):
    """The value check sees the cross term of the original ADI: without it the
    E right-hand side differs from the operator form."""
    g, arrays = grid
    theta = 0.5 * g.dt
    rhs, _, _ = _reference("original", "A", "B", theta, arrays, g)
    got, _, _, _, _ = oc.procedure("original", "A", "B", theta, arrays, (3, 2, 3), g)
    # the same right-hand side with the B-part of w left out of the H rows
    u = _vec(arrays, COMPONENTS)
    Yu = apply_operator("B", u, g)
    w = [a + theta * b for a, b in zip(u, Yu)]
    w_noH = w[:3] + u[3:]
    Xw = apply_operator("A", w_noH, g)
    for ce, _, _, _ in PAIRS["A"]:
        wrong = w_noH[CIDX[ce]][3, 2, 3] + theta * Xw[CIDX[ce]][3, 2, 3]
        assert abs(got[ce].v - rhs[ce][3, 2, 3]) <= 1e-12 * max(1.0, abs(rhs[ce][3, 2, 3]))
        assert abs(wrong - rhs[ce][3, 2, 3]) > 1e-6 * max(1.0, abs(rhs[ce][3, 2, 3]))
