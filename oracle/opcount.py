"""Operation counts of the main iterations, per grid cell and time step (Sec. IV, Table I).

Test infrastructure: only tests/ use this module.

The paper counts the multiplications/divisions (M/D) and additions/subtractions
(A/S) on the right-hand sides of every updating equation of one complete time
step.  Its conventions (Sec. IV, the paragraph before Table I):
* every multiplicative factor is precomputed and stored (here: per node, from
  eps at the E node, mu, theta and the spacings);
* one component of each kind per cell (equal numbers in all directions);
* "implicit" counts the right-hand sides of the E line systems (with the
  subtraction that recovers the field from the solved auxiliary variable,
  eqs. (fasterADIaa), (fastLODb), (fastLOD2b)), "explicit" the H updates;
* the tridiagonal solves are left out (about 5N flops for a system of order N).

Each procedure of a scheme is written out per node below, in the component form
its equations take on the Yee grid with the operators of eq. (AMat) and the
factors of eq. (bd), like terms collected under one factor, and evaluated with
`Counted` numbers that tally M/D and A/S.  The same expressions evaluated on
field values are compared, by the tests, with the right-hand sides formed from
the operator form with `oracle.yee.apply_operator`, so the counts belong to
expressions that compute the schemes.

Readings:
* Original (conventional) schemes, eqs. (clsADI), (orgLOD), (orgSS2), (orgLOD2):
  eliminating the implicit H rows gives the E line system
  (I - theta^2 X_EH X_HE) E' = [w + theta X w]_E with w = (I + theta Y) u
  (Y = the explicit operator: the other one for ADI, the same one for the LOD
  family); then H' = [w + theta X (E', 0)]_H.  With Y != X (ADI) the E
  right-hand side has four terms, one a mixed second difference of another E
  component through the mu of two H nodes; the count takes mu uniform (one
  precomputed factor), as the paper's counts of these schemes do.  With Y = X
  the terms in E_c collect into (1 - 2bd) E_c + bd (E_c[+1] + E_c[-1]).
* New (fundamental) schemes, eqs. (fasterADI) with (fasterADIaa)-(fasterADIddh),
  (fastLOD), (fastSS2), (fastLOD2): one difference under one factor per equation,
  e.g. e + b d_w h and h + d d_w E~.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .yee import MU0, PAIRS, Grid


@dataclass
class Tally:
    md: int = 0
    as_: int = 0


class Counted:
    """A value that counts the arithmetic done on it: +/- with another Counted
    is one A/S, * or / by a precomputed factor (a float) is one M/D."""
    __slots__ = ("v", "t")

    def __init__(self, v: float, t: Tally):
        self.v = float(v)
        self.t = t

    def __add__(self, o: "Counted") -> "Counted":
        assert isinstance(o, Counted)
        self.t.as_ += 1
        return Counted(self.v + o.v, self.t)

    def __sub__(self, o: "Counted") -> "Counted":
        assert isinstance(o, Counted)
        self.t.as_ += 1
        return Counted(self.v - o.v, self.t)

    def __mul__(self, f: float) -> "Counted":
        assert isinstance(f, float)
        self.t.md += 1
        return Counted(self.v * f, self.t)

    __rmul__ = __mul__


# Procedures of the main iteration of each scheme: (implicit operator X,
# explicit operator Y, theta as a fraction of dt).  Original ADI takes Y != X
# (eq. (clsADI)); the LOD family Y = X (eqs. (orgLOD), (orgSS2), (orgLOD2)).
# The new forms have the same procedures with matrix-operator-free right-hand
# sides (eqs. (fasterADI), (fastLOD), (fastSS2), (fastLOD2)).
PROCEDURES = {
    "ADI": (("A", "B", 0.5), ("B", "A", 0.5)),
    "LOD1": (("A", "A", 0.5), ("B", "B", 0.5)),
    "SS2": (("A", "A", 0.25), ("B", "B", 0.5), ("A", "A", 0.25)),
    "LOD2": (("A", "A", 0.5), ("B", "B", 0.5)),
}


def _pair_with_e(op: str, ce: str):
    return next(p for p in PAIRS[op] if p[0] == ce)


def _pair_with_h(op: str, ch: str):
    return next(p for p in PAIRS[op] if p[1] == ch)


class _Node:
    """Counted reads of named arrays around one node (k, j, i)."""

    def __init__(self, arrays: dict, node, t: Tally):
        self.a, self.n, self.t = arrays, node, t

    def __call__(self, name: str, **off) -> Counted:
        k, j, i = self.n
        k += off.get("z", 0)
        j += off.get("y", 0)
        i += off.get("x", 0)
        return Counted(self.a[name][k, j, i], self.t)


def _shift(w: str, s: int) -> dict:
    return {w: s}


def procedure(form: str, X: str, Y: str, theta: float, arrays: dict, node, g: Grid):
    """One procedure at one node: returns ({E comp: right-hand side}, {H comp:
    updated value}, {E comp: field from the solved variable (new forms)},
    implicit Tally, explicit Tally).

    arrays: 'Ex'.. 'Hz' the state entering the procedure (u; for the new ADI
    its E~ and the auxiliary h), 'e_Ex'.. the new ADI's e from the previous
    procedure, 'S_Ex'.. the solution of the E line systems."""
    ti, tx = Tally(), Tally()
    P, Q = _Node(arrays, node, ti), _Node(arrays, node, tx)
    k, j, i = node
    rhs, hnew, enew = {}, {}, {}
    for ce, ch, p, s in PAIRS[X]:
        eps = float(g.eps[k, j, i])
        hp = g.spacing(p)
        b = theta * s / (eps * hp)          # E row of X: b d_p H
        d = theta * s / (MU0 * hp)          # H row of X: d d_p E
        if form == "original" and X != Y:   # ADI, eq. (clsADI)
            _, ct, r, sy = _pair_with_e(Y, ce)        # E_c <- sY/eps d_r H_t in Y
            cm, _, r2, sy2 = _pair_with_h(Y, ch)      # H_q <- sY2/mu d_r2 E_m in Y
            bY = theta * sy / (eps * g.spacing(r))
            bdXY = theta * theta * s * sy2 / (eps * MU0 * hp * g.spacing(r2))
            # d_p (d_r2 E_m) through the H nodes n and n - e_p (r2 != p in ADI)
            cross = (P(cm, **_shift(r2, 1)) - P(cm)) - (P(cm, **{p: -1, r2: 1}) - P(cm, **_shift(p, -1)))
            rhs[ce] = P(ce) + bY * (P(ct) - P(ct, **_shift(r, -1))) + b * (P(ch) - P(ch, **_shift(p, -1))) + bdXY * cross
            dY = theta * sy2 / (MU0 * g.spacing(r2))
            hnew[ch] = Q(ch) + dY * (Q(cm, **_shift(r2, 1)) - Q(cm)) + d * (Q("S_" + ce, **_shift(p, 1)) - Q("S_" + ce))
        elif form == "original":            # LOD family, Y = X
            bd = theta * theta / (eps * MU0 * hp * hp)
            rhs[ce] = ((1.0 - 2.0 * bd) * P(ce) + (2.0 * b) * (P(ch) - P(ch, **_shift(p, -1)))
                       + bd * (P(ce, **_shift(p, 1)) + P(ce, **_shift(p, -1))))
            hnew[ch] = Q(ch) + d * ((Q(ce, **_shift(p, 1)) - Q(ce)) + (Q("S_" + ce, **_shift(p, 1)) - Q("S_" + ce)))
        elif X != Y:                        # new ADI, eqs. (fasterADIaa)-(fasterADIddh)
            rhs[ce] = (P(ce) - P("e_" + ce)) + b * (P(ch) - P(ch, **_shift(p, -1)))
            hnew[ch] = Q(ch) + d * (Q("S_" + ce, **_shift(p, 1)) - Q("S_" + ce))
        else:                               # new LOD family, eqs. (fastLOD), (fastSS2), (fastLOD2)
            rhs[ce] = P(ce) + b * (P(ch) - P(ch, **_shift(p, -1)))
            enew[ce] = P("S_" + ce) - P(ce)   # u = v - u, counted with the implicit side
            hnew[ch] = Q(ch) + d * (Q("S_" + ce, **_shift(p, 1)) - Q("S_" + ce))
    return rhs, hnew, enew, ti, tx


def step_counts(scheme: str, form: str, g: Grid, arrays: dict, node) -> dict:
    """M/D and A/S of one complete time step at one cell, split into implicit
    and explicit, with the number of component updating sweeps (for-loops) and
    of E line systems per cell."""
    ti, tx = Tally(), Tally()
    loops = systems = 0
    for X, Y, frac in PROCEDURES[scheme]:
        rhs, hnew, enew, a, b = procedure(form, X, Y, frac * g.dt, arrays, node, g)
        ti.md += a.md
        ti.as_ += a.as_
        tx.md += b.md
        tx.as_ += b.as_
        loops += len(rhs) + len(hnew)
        systems += len(rhs)
    return {"implicit_md": ti.md, "implicit_as": ti.as_, "explicit_md": tx.md, "explicit_as": tx.as_,
            "total_md": ti.md + tx.md, "total_as": ti.as_ + tx.as_,
            "total": ti.md + tx.md + ti.as_ + tx.as_, "loops": loops, "systems": systems}


def efficiency_gains(counts: dict, reference: dict, flops_per_row: int = 5) -> tuple[float, float]:
    """Gains over a reference scheme (the original ADI): on the right-hand
    sides alone, and with about flops_per_row flops per row of every
    tridiagonal system added to both (Sec. IV)."""
    rhs = reference["total"] / counts["total"]
    overall = ((reference["total"] + flops_per_row * reference["systems"])
               / (counts["total"] + flops_per_row * counts["systems"]))
    return rhs, overall


def random_arrays(g: Grid, rng: np.random.Generator) -> dict:
    """Random values for every array a procedure reads (interior use only)."""
    names = ["Ex", "Ey", "Ez", "Hx", "Hy", "Hz"]
    names += ["e_" + c for c in names[:3]] + ["S_" + c for c in names[:3]]
    return {n: rng.standard_normal(g.shape) for n in names}


__all__ = ["Counted", "Tally", "PROCEDURES", "procedure", "step_counts", "efficiency_gains", "random_arrays"]
