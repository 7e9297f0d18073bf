"""Original ("conventional") splitting formulae of Sec. II, applied literally.

Each sub-step is   (I - theta X) u' = (I + theta Y) u + g :
the right side is formed explicitly with the operator Y (a matrix operator on
the right-hand side -- what the fundamental schemes remove), then the implicit
side is solved pair by pair (``implicit.solve_implicit``).

* ADI, eq. (clsADI):   X = A, Y = B, theta = dt/2;  then X = B, Y = A.
* LOD1/SS1, (orgLOD):  X = Y = A, theta = dt/2;  then X = Y = B.
* SS2, (orgSS2):       A with dt/4, B with dt/2, A with dt/4 (X = Y).
* LOD2, (orgLOD2):     as LOD1 on the time levels n+1/4 -> n+3/4 -> n+5/4,
  with input processing (orgLOD2i) (theta = dt/4, operator B) and output
  processing (orgLOD2o) (theta = -dt/4, operator B).
"""
from __future__ import annotations

import numpy as np

from .implicit import solve_implicit
from .yee import CIDX, PAIRS, Grid, apply_operator


def substep(u, x_op: str, y_op: str, theta: float, g: Grid, src_val: float = 0.0,
            src_node=None):
    """One sub-step  (I - theta X) u' = (I + theta Y) u + g."""
    yu = apply_operator(y_op, u, g)
    f = [a + theta * b for a, b in zip(u, yu)]
    if src_node is not None and src_val != 0.0:
        f[CIDX["Ez"]] = f[CIDX["Ez"]].copy()
        f[CIDX["Ez"]][src_node] += src_val
    return solve_implicit(x_op, PAIRS[x_op], f, theta, g)


# (X, Y, theta / dt, source time in units of dt within the step)
MAIN = {
    "adi": (("A", "B", 0.5, 0.25), ("B", "A", 0.5, 0.75)),
    "lod1": (("A", "A", 0.5, 0.25), ("B", "B", 0.5, 0.75)),
    "ss2": (("A", "A", 0.25, 0.125), ("B", "B", 0.5, 0.5), ("A", "A", 0.25, 0.875)),
    "lod2": (("A", "A", 0.5, 0.5), ("B", "B", 0.5, 1.0)),
}


def step(scheme: str, u, g: Grid, n: int, source=None):
    """Main iteration n of a scheme (for LOD2 the state is on the n+1/4 levels)."""
    node = (source.k, source.j, source.i) if source is not None else None
    for x_op, y_op, th, tf in MAIN[scheme]:
        theta = th * g.dt
        val = source.g(theta, (n + tf) * g.dt) if source is not None else 0.0
        u = substep(u, x_op, y_op, theta, g, val, node)
    return u


def input_processing(scheme: str, u, g: Grid):
    if scheme == "lod2":  # (orgLOD2i)
        return substep(u, "B", "B", 0.25 * g.dt, g)
    return [np.array(a, copy=True) for a in u]


def output_processing(scheme: str, u, g: Grid):
    if scheme == "lod2":  # (orgLOD2o): (I + dt/4 B) u^{n+1} = (I - dt/4 B) u^{n+5/4}
        return substep(u, "B", "B", -0.25 * g.dt, g)
    return [np.array(a, copy=True) for a in u]


def invariant(scheme: str, u, g: Grid) -> float:
    """The energy each scheme conserves without sources, evaluated on its main-
    iteration state: W(u) for LOD1, SS2 and LOD2 (on the n+1/4 levels);
    W((1/2 I + dt/4 B) u) = W((I + dt/2 B) u)/4 for ADI."""
    from .yee import energy
    if scheme == "adi":
        bu = apply_operator("B", u, g)
        return energy([0.5 * a + 0.25 * g.dt * b for a, b in zip(u, bu)], g)
    return energy(u, g)


def splitting_step(scheme: str, u, g: Grid):
    """One step of the original D'Yakonov (orgDY) or delta-formulation
    Douglas-Gunn splitting of Sec. II-E, operators applied as written:
      "dy":  (I - dt/2 A) u* = (I + dt/2 A)(I + dt/2 B) u^n ;  (I - dt/2 B) u^{n+1} = u*
      "dg":  (I - dt/2 A) du* = dt (A + B) u^n ;  (I - dt/2 B) du = du* ;  u^{n+1} = u^n + du
    """
    h = 0.5 * g.dt
    if scheme == "dy":
        bu = apply_operator("B", u, g)
        w = [a + h * b for a, b in zip(u, bu)]
        aw = apply_operator("A", w, g)
        f = [a + h * b for a, b in zip(w, aw)]
        ustar = solve_implicit("A", PAIRS["A"], f, h, g)
        return solve_implicit("B", PAIRS["B"], ustar, h, g)
    if scheme == "dg":
        au = apply_operator("A", u, g)
        bu = apply_operator("B", u, g)
        f = [g.dt * (a + b) for a, b in zip(au, bu)]
        dstar = solve_implicit("A", PAIRS["A"], f, h, g)
        du = solve_implicit("B", PAIRS["B"], dstar, h, g)
        return [a + b for a, b in zip(u, du)]
    raise ValueError(scheme)
