"""Fundamental schemes in the paper's component form (Sec. III).

Every implicit update has the matrix-operator-free form of eqs. (fasterADIb),
(fastLODa), (fastSS2a), (fastLOD2a):

    (1/2 I - theta/2 X) v = u ,

which, for a pair (E, H, w, s) of X and b = theta/eps, d = theta/mu (eq. (bd)
with theta = dt/2), is the implicit line equation plus an explicit H update

    1/2 e - (b d / 2) d_w^2 e = E + s b d_w H            (e.g. (fastLOD2.1))
    H <- H + s d d_w e                                     ((fastestLOD2ex1/2))
    E <- e - E                                             ((fastLOD2.bbE))

LOD family (LOD1 = SS1, SS2, LOD2): the state u holds the fields E, H; each
sub-step applies the three updates above to the three pairs of X.  Sec. III-B
prints them for LOD2; LOD1/SS1 and SS2 follow "by similar arguments" with
theta = dt/2 (LOD1) or dt/4, dt/2, dt/4 (SS2).

ADI (Sec. III-A): the state is (E~, e, h) in the scaling u~ = 2u of (uTldCol):
    e^n = E~^n - e^{n-1/2}                                 (fasterADIaa)
    1/2 E~^{n+1/2} - (bd/2) d^2 E~^{n+1/2} = e^n + b d h^n     (A pairs)
    h^{n+1/2} = h^n + d d E~^{n+1/2}                        (fasterADIbbh)
    e^{n+1/2} = E~^{n+1/2} - e^n                            (fasterADIcc)
    1/2 E~^{n+1} - (bd/2) d^2 E~^{n+1} = e^{n+1/2} - b d h^{n+1/2}  (B pairs)
    h^{n+1} = h^{n+1/2} - d d E~^{n+1}                      (fasterADIddh)
with input v^{-1/2} = (I - dt/2 B) u^0 (fastADIi), u~^0 = 2 u^0, the first
magnetic auxiliary h^0 = H~^0 - h^{-1/2} (fasterADIaah), and output
u = u~/2 (fasterADIo), where H~^{n+1} = 2 h^{n+1/2} - d d E~^{n+1}
(fasterADIddd) = h^{n+1/2} + h^{n+1}.

Sources (convention of ``source``): a sub-step with nonhomogeneous term g
solves (1/2 I - theta/2 X) v = u + g/2 and sets u' = v - u (LOD family); in
ADI the term enters the auxiliary subtraction, e <- E~ - e + g (the auxiliary
v equals 2u in the u~ scaling).
"""
from __future__ import annotations

import numpy as np

from .implicit import line_operator_solve, solve_implicit
from .yee import CIDX, PAIRS, Grid, apply_operator, d_half, d_int, dynamic_mask, energy

E_COMPS = ("Ex", "Ey", "Ez")
H_COMPS = ("Hx", "Hy", "Hz")


def _implicit(op: str, e_rhs_src, h_src, theta: float, g: Grid):
    """Solve the three implicit line equations of operator `op`:
    1/2 V - (bd/2) d_w^2 V = e_rhs_src[E] + s b d_w h_src[H]  -> dict E comp -> V."""
    out = {}
    for ce, ch, w, s in PAIRS[op]:
        b = theta / g.eps
        rhs = e_rhs_src[ce] + s * b * d_int(h_src[ch], w, g)
        out[ce] = line_operator_solve(rhs, ce, ch, w, 0.5 * theta * theta, 0.5, g)
    return out


def _h_update(op: str, h: dict, v: dict, theta: float, g: Grid, sign: float = 1.0):
    """H <- H + s d d_w V for the three pairs of `op` (dynamic H nodes only)."""
    for ce, ch, w, s in PAIRS[op]:
        d = theta / g.mu
        h[ch] = h[ch] + sign * s * d * d_half(v[ce], w, g) * dynamic_mask(ch, g)


# ----------------------------------------------------------------------------
# LOD family
# ----------------------------------------------------------------------------

def lod_substep(u, op: str, theta: float, g: Grid, src_val: float = 0.0, src_node=None):
    """(1/2 I - theta/2 X) v = u + g/2 ;  u' = v - u  in component form."""
    E = {c: u[CIDX[c]] for c in E_COMPS}
    H = {c: np.array(u[CIDX[c]], copy=True) for c in H_COMPS}
    rhs_e = dict(E)
    if src_node is not None and src_val != 0.0:
        rhs_e["Ez"] = E["Ez"].copy()
        rhs_e["Ez"][src_node] += 0.5 * src_val
    v = _implicit(op, rhs_e, H, theta, g)          # implicit updating
    _h_update(op, H, v, theta, g)                   # explicit, h absorbed into H
    E_new = {c: (v[c] - E[c]) * dynamic_mask(c, g) for c in E_COMPS}  # E = e - E
    return [E_new["Ex"], E_new["Ey"], E_new["Ez"], H["Hx"], H["Hy"], H["Hz"]]


LOD_MAIN = {
    "lod1": (("A", 0.5, 0.25), ("B", 0.5, 0.75)),
    "ss2": (("A", 0.25, 0.125), ("B", 0.5, 0.5), ("A", 0.25, 0.875)),
    "lod2": (("A", 0.5, 0.5), ("B", 0.5, 1.0)),
}


def lod_step(scheme: str, u, g: Grid, n: int, source=None):
    node = (source.k, source.j, source.i) if source is not None else None
    for op, th, tf in LOD_MAIN[scheme]:
        theta = th * g.dt
        val = source.g(theta, (n + tf) * g.dt) if source is not None else 0.0
        u = lod_substep(u, op, theta, g, val, node)
    return u


def lod2_input(u, g: Grid):
    """(fastLOD2i): (1/2 I - dt/8 B) v^{1/4} = u^0 ; u^{1/4} = v^{1/4} - u^0."""
    return lod_substep(u, "B", 0.25 * g.dt, g)


def lod2_output(u, g: Grid):
    """(fastLOD2o): (1/2 I + dt/8 B) v^{n+1} = u^{n+5/4} ; u^{n+1} = v^{n+1} - u^{n+5/4}."""
    return lod_substep(u, "B", -0.25 * g.dt, g)


# ----------------------------------------------------------------------------
# ADI in the paper's (E~, e, h) variables
# ----------------------------------------------------------------------------

class FundamentalADI:
    """State of the fundamental ADI iteration (fasterADI) with combined h updates."""

    def __init__(self, u0, g: Grid):
        self.g = g
        half = 0.5 * g.dt
        bu = apply_operator("B", u0, g)
        vm = [a - half * b for a, b in zip(u0, bu)]            # (fastADIi)
        self.Et = {c: 2.0 * u0[CIDX[c]] for c in E_COMPS}       # (uTldCol)
        Ht0 = {c: 2.0 * u0[CIDX[c]] for c in H_COMPS}
        self.e = {c: vm[CIDX[c]] for c in E_COMPS}              # e^{-1/2}
        # first magnetic auxiliary from (fasterADIaah) at n = 0
        self.h = {c: Ht0[c] - vm[CIDX[c]] for c in H_COMPS}     # h^0
        self.h_half = None
        self.n = 0
        self.u0 = [np.array(a, copy=True) for a in u0]

    def step(self, source=None):
        g, n = self.g, self.n
        theta = 0.5 * g.dt
        node = (source.k, source.j, source.i) if source is not None else None
        # (fasterADIaa): e^n = E~^n - e^{n-1/2}  (+ g of sub-step A)
        self.e = {c: self.Et[c] - self.e[c] for c in E_COMPS}
        if node is not None:
            self.e["Ez"][node] += source.g(theta, (n + 0.25) * g.dt)
        # implicit A, then (fasterADIbbh)
        vt = _implicit("A", self.e, self.h, theta, g)
        self.Et.update(vt)
        _h_update("A", self.h, vt, theta, g)
        self.h_half = {c: self.h[c].copy() for c in H_COMPS}
        # (fasterADIcc): e^{n+1/2} = E~^{n+1/2} - e^n  (+ g of sub-step B)
        self.e = {c: self.Et[c] - self.e[c] for c in E_COMPS}
        if node is not None:
            self.e["Ez"][node] += source.g(theta, (n + 0.75) * g.dt)
        # implicit B (s = -1 carried by the pairs), then (fasterADIddh)
        vt = _implicit("B", self.e, self.h, theta, g)
        self.Et.update(vt)
        _h_update("B", self.h, vt, theta, g)
        self.n += 1

    def fields(self):
        """(fasterADIo): u = u~/2 with H~ = h^{n-1/2} + h^n (fasterADIddd)."""
        if self.h_half is None:  # no step taken yet: u^0 itself
            return [np.array(a, copy=True) for a in self.u0]
        E = [0.5 * self.Et[c] for c in E_COMPS]
        H = [0.5 * (self.h_half[c] + self.h[c]) for c in H_COMPS]
        return E + H

    def invariant(self) -> float:
        """W(v^n)/4 with v^n = (E~^n - e^{n-1/2}, h^n): the conserved energy,
        equal to W((I + dt/2 B) u^n)/4."""
        v = [self.Et[c] - self.e[c] for c in E_COMPS] + [self.h[c] for c in H_COMPS]
        return 0.25 * energy(v, self.g)


# ----------------------------------------------------------------------------
# D'Yakonov and Douglas-Gunn in fundamental form (Sec. II-E), no sources
# ----------------------------------------------------------------------------

def solve_half(op: str, r, theta: float, g: Grid):
    """y with (1/2 I - theta/2 X) y = r for all six components, i.e. the stage
    (I - theta X) y = 2 r (static normal H keeps 2 r, wall E stays 0)."""
    return solve_implicit(op, PAIRS[op], [2.0 * a for a in r], theta, g)


def _src_add(v, source, val):
    """v with val added at the Ez sample of the source (a copy of that component)."""
    if source is None or val == 0.0:
        return v
    v = list(v)
    v[CIDX["Ez"]] = v[CIDX["Ez"]].copy()
    v[CIDX["Ez"]][source.k, source.j, source.i] += val
    return v


def dyakonov(u0, g: Grid, steps: int, record=None, source=None):
    """Eq. (fastDY) with input v^{-1/2} = (1/2 I - dt/4 B) u^0; returns u^steps.
    `record(n, u)` is called with u^n for n = 0..steps when given.  A source
    term g of a sub-step enters the auxiliary subtraction as g/2 (the ADI
    convention in these unscaled variables)."""
    half = 0.5 * g.dt
    bu = apply_operator("B", u0, g)
    v = [0.5 * a - 0.5 * half * b for a, b in zip(u0, bu)]   # v^{-1/2}
    u = [np.array(a, copy=True) for a in u0]
    if record:
        record(0, u)
    for n in range(steps):
        gA = source.g(half, (n + 0.25) * g.dt) if source is not None else 0.0
        gB = source.g(half, (n + 0.75) * g.dt) if source is not None else 0.0
        v = _src_add([a - b for a, b in zip(u, v)], source, 0.5 * gA)    # v^n = u^n - v^{n-1/2}
        uh = solve_half("A", v, half, g)                                  # u^{n+1/2}
        v = _src_add([a - b for a, b in zip(uh, v)], source, 0.5 * gB)   # v^{n+1/2}
        u = solve_half("B", v, half, g)                                   # u^{n+1}
        if record:
            record(n + 1, u)
    return u


def douglas_gunn(u0, g: Grid, steps: int, record=None, source=None):
    """The ADI iteration (fasterADI) from (fastADIi), (uTldCol), with the field
    advanced by the increment of (fastDGo): u^{n+1} = u^n + (u~^{n+1} - u~^n)/2.
    A source term g enters the auxiliary subtraction as in ADI."""
    half = 0.5 * g.dt
    bu = apply_operator("B", u0, g)
    v = [a - half * b for a, b in zip(u0, bu)]                # v^{-1/2}
    ut = [2.0 * a for a in u0]                                # u~^0
    u = [np.array(a, copy=True) for a in u0]
    if record:
        record(0, u)
    for n in range(steps):
        gA = source.g(half, (n + 0.25) * g.dt) if source is not None else 0.0
        gB = source.g(half, (n + 0.75) * g.dt) if source is not None else 0.0
        v = _src_add([a - b for a, b in zip(ut, v)], source, gA)
        uth = solve_half("A", v, half, g)                     # u~^{n+1/2}
        v = _src_add([a - b for a, b in zip(uth, v)], source, gB)
        utn = solve_half("B", v, half, g)                     # u~^{n+1}
        u = [a + 0.5 * (b - c) for a, b, c in zip(u, utn, ut)]
        ut = utn
        if record:
            record(n + 1, u)
    return u
