"""Yee-grid Maxwell operators A and B of eq. (AMat), coefficients (bd), masks, energy.

Sec. III (opening) of the paper splits Maxwell's curl equations for a lossless
isotropic medium into two 6x6 operator matrices,

    A: Ex <- (1/eps) d_y Hz,  Ey <- (1/eps) d_z Hx,  Ez <- (1/eps) d_x Hy,
       Hx <- (1/mu)  d_z Ey,  Hy <- (1/mu)  d_x Ez,  Hz <- (1/mu)  d_y Ex,
    B: Ex <- -(1/eps) d_z Hy, Ey <- -(1/eps) d_x Hz, Ez <- -(1/eps) d_y Hx,
       Hx <- -(1/mu)  d_y Ez, Hy <- -(1/mu)  d_z Ex, Hz <- -(1/mu)  d_x Ey,

with d_w the second-order central difference on Yee cells (Sec. III-A, last
paragraph; Sec. III-B, "second-order central-differencing operators on Yee
cells").  Each operator couples the six components in three disjoint (E, H)
pairs, each pair along one axis w with a sign s:

    A: (Ex, Hz, y, +1), (Ey, Hx, z, +1), (Ez, Hy, x, +1)
    B: (Ex, Hy, z, -1), (Ey, Hz, x, -1), (Ez, Hx, y, -1)

Readings where the paper is silent:
* PEC on all six faces: tangential E on a wall is 0; normal H on a wall is
  static (its driving differences are tangential E on that wall).
* eps and mu at staggered nodes: the component stored at node index [k, j, i]
  uses the cell value eps_r[k, j, i] (indices clamped to the last cell for the
  H entries on the far walls).  Every dynamic E node has an in-range index.
* SI units; the constants below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
C0 = 1.0 / math.sqrt(EPS0 * MU0)

COMPONENTS = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
CIDX = {c: n for n, c in enumerate(COMPONENTS)}
AXIS = {"x": 2, "y": 1, "z": 0}  # array axis of each spatial direction ([k, j, i])

# (E component, H component, line axis, sign) for the three pairs of A and of B,
# read off eq. (AMat).
PAIRS = {
    "A": (("Ex", "Hz", "y", +1), ("Ey", "Hx", "z", +1), ("Ez", "Hy", "x", +1)),
    "B": (("Ex", "Hy", "z", -1), ("Ey", "Hz", "x", -1), ("Ez", "Hx", "y", -1)),
}


def cfl_dt(dx: float, dy: float, dz: float, cfl_number: float) -> float:
    """cfl_number times the vacuum Yee limit 1/(c0 sqrt(dx^-2+dy^-2+dz^-2))."""
    return cfl_number / (C0 * math.sqrt(dx ** -2 + dy ** -2 + dz ** -2))


@dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    dt: float
    eps_r: np.ndarray | None = None  # (nz, ny, nx) relative permittivity per cell
    mu_r: np.ndarray | None = None   # (nz, ny, nx) relative permeability per cell
    _cache: dict = field(default_factory=dict, repr=False)

    def __post_init__(self):
        if self.eps_r is None:
            self.eps_r = np.ones((self.nz, self.ny, self.nx))
        if self.mu_r is None:
            self.mu_r = np.ones((self.nz, self.ny, self.nx))
        self.eps_r = np.asarray(self.eps_r, dtype=np.float64)
        self.mu_r = np.asarray(self.mu_r, dtype=np.float64)
        assert self.eps_r.shape == (self.nz, self.ny, self.nx)
        assert self.mu_r.shape == (self.nz, self.ny, self.nx)

    @property
    def shape(self):
        return (self.nz + 1, self.ny + 1, self.nx + 1)

    def spacing(self, w: str) -> float:
        return {"x": self.dx, "y": self.dy, "z": self.dz}[w]

    def _node_values(self, cell: np.ndarray) -> np.ndarray:
        k = np.minimum(np.arange(self.nz + 1), self.nz - 1)
        j = np.minimum(np.arange(self.ny + 1), self.ny - 1)
        i = np.minimum(np.arange(self.nx + 1), self.nx - 1)
        return cell[np.ix_(k, j, i)]

    @property
    def eps(self) -> np.ndarray:
        """Absolute permittivity at every node index (owned-index reading)."""
        if "eps" not in self._cache:
            self._cache["eps"] = EPS0 * self._node_values(self.eps_r)
        return self._cache["eps"]

    @property
    def mu(self) -> np.ndarray:
        if "mu" not in self._cache:
            self._cache["mu"] = MU0 * self._node_values(self.mu_r)
        return self._cache["mu"]

    def material(self, comp: str) -> np.ndarray:
        return self.eps if comp[0] == "E" else self.mu


def dynamic_mask(comp: str, g: Grid) -> np.ndarray:
    """True at the nodes whose value the time stepping changes.

    E: inside the box and not on a wall it is tangential to.
    H: inside the box and not on a wall it is normal to.
    """
    m = np.zeros(g.shape, dtype=bool)
    nx, ny, nz = g.nx, g.ny, g.nz
    if comp == "Ex":
        m[1:nz, 1:ny, 0:nx] = True
    elif comp == "Ey":
        m[1:nz, 0:ny, 1:nx] = True
    elif comp == "Ez":
        m[0:nz, 1:ny, 1:nx] = True
    elif comp == "Hx":
        m[0:nz, 0:ny, 1:nx] = True
    elif comp == "Hy":
        m[0:nz, 1:ny, 0:nx] = True
    elif comp == "Hz":
        m[1:nz, 0:ny, 0:nx] = True
    else:
        raise ValueError(comp)
    return m


def diff_to_integer(f: np.ndarray, w: str, h: float) -> np.ndarray:
    """Central difference of a field sampled at half-integer positions along w
    (stored index j <-> j+1/2), evaluated at the integer positions j:
    (f[j] - f[j-1]) / h.  Entry j = 0 is left 0 (a wall for every E that uses it)."""
    ax = AXIS[w]
    out = np.zeros_like(f)
    n = f.shape[ax]
    dst = [slice(None)] * 3
    a = [slice(None)] * 3
    b = [slice(None)] * 3
    dst[ax] = slice(1, n)
    a[ax] = slice(1, n)
    b[ax] = slice(0, n - 1)
    out[tuple(dst)] = (f[tuple(a)] - f[tuple(b)]) / h
    return out


def diff_to_half(f: np.ndarray, w: str, h: float) -> np.ndarray:
    """Central difference of a field sampled at integer positions along w,
    evaluated at the half-integer positions j+1/2 (stored at index j):
    (f[j+1] - f[j]) / h.  The last entry (outside the box) is left 0."""
    ax = AXIS[w]
    out = np.zeros_like(f)
    n = f.shape[ax]
    dst = [slice(None)] * 3
    a = [slice(None)] * 3
    b = [slice(None)] * 3
    dst[ax] = slice(0, n - 1)
    a[ax] = slice(1, n)
    b[ax] = slice(0, n - 1)
    out[tuple(dst)] = (f[tuple(a)] - f[tuple(b)]) / h
    return out


def apply_operator(op: str, u, g: Grid):
    """X u for X = A or B of eq. (AMat); returns a list of six arrays, zero at
    every non-dynamic node."""
    out = [np.zeros(g.shape) for _ in COMPONENTS]
    for ce, ch, w, s in PAIRS[op]:
        h = g.spacing(w)
        e, hh = u[CIDX[ce]], u[CIDX[ch]]
        out[CIDX[ce]] = s * diff_to_integer(hh, w, h) / g.eps * dynamic_mask(ce, g)
        out[CIDX[ch]] = s * diff_to_half(e, w, h) / g.mu * dynamic_mask(ch, g)
    return out


def energy(u, g: Grid) -> float:
    """Discrete electromagnetic energy  sum eps |E|^2 + mu |H|^2  over all nodes
    (cell volume omitted, uniform).  The paper defines no energy; this is the
    weighted norm in which A and B are skew-adjoint."""
    tot = 0.0
    for n, c in enumerate(COMPONENTS):
        tot += float(np.sum(g.material(c) * u[n] * u[n]))
    return tot


def weighted_rel_l2(u, ref, g: Grid) -> float:
    """Energy-weighted relative L2 difference ||u - ref||_W / ||ref||_W."""
    num = energy([a - b for a, b in zip(u, ref)], g)
    den = energy(ref, g)
    return math.sqrt(num / den) if den > 0 else math.sqrt(num)


def clean(u, g: Grid):
    """Copy of u with every non-dynamic E node set to 0 (the PEC walls)."""
    out = []
    for n, c in enumerate(COMPONENTS):
        a = np.array(u[n], dtype=np.float64, copy=True)
        if c[0] == "E":
            a[~dynamic_mask(c, g)] = 0.0
        out.append(a)
    return out
