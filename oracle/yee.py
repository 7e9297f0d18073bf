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
    order: int = 2                   # accuracy order of the staggered first differences (2 or 4)
    outer: float = -1.0 / 24.0       # order 4: outer weight b of the 4-point difference (stencil4)
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
        assert self.order in (2, 4)

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

    @property
    def w4(self) -> np.ndarray:
        """Weights of the 4-point staggered difference (order 4)."""
        return stencil4(self.outer)


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


# ----------------------------------------------------------------------------
# Fourth-order staggered first differences.  The closing remark of Sec. III-A
# leaves the difference operators open (higher order, optimized, compact); the
# updating equations keep their form with any d_w.  This is the fourth-order
# one: at a point midway between samples spaced h,
#     d_w f = (f[-3/2] - 27 f[-1/2] + 27 f[+1/2] - f[+3/2]) / (24 h),
# exact for cubics.  Reading where the paper is silent: near a PEC wall the
# stencil reaches across the wall to image samples -- the E tangential to the
# wall odd about it (E[-j] = -E[j], E = 0 on the wall), the H tangential to it
# even (H[-1/2 - j] = H[1/2 + j]) -- so that, as for the second-order
# differences, d_int = -d_half^T on the dynamic samples and A, B stay
# skew-adjoint in the energy norm.  Every sine/cosine PEC cavity mode is then
# an eigenvector, with d_w sin(k x) = K4 cos(k x), K4 = (27 sin(k h / 2) -
# sin(3 k h / 2)) / (12 h).
# ----------------------------------------------------------------------------
W4 = np.array([1.0, -27.0, 27.0, -1.0]) / 24.0


# The same remark names parameter-optimized operators.  Reading: the 4-point
# staggered difference with a free outer weight b,
#     d_w f = [(1 - 3b)(f[+1/2] - f[-1/2]) + b (f[+3/2] - f[-3/2])] / h,
# exact on quadratics for every b (consistency fixes the inner weight), fourth
# order only at b = -1/24 (W4), with the same image folding at the walls (so
# d_int = -d_half^T still holds) and the modified wavenumber
#     K(k) h = 2 (1 - 3b) sin(k h / 2) + 2 b sin(3 k h / 2).
def stencil4(outer: float) -> np.ndarray:
    """Weights of the samples at -3/2, -1/2, +1/2, +3/2 for outer weight b."""
    inner = 1.0 - 3.0 * outer
    return np.array([-outer, -inner, inner, outer])


def modified_wavenumber4(outer: float, theta):
    """K(k) h of the 4-point difference at theta = k h."""
    return 2.0 * (1.0 - 3.0 * outer) * np.sin(theta / 2.0) + 2.0 * outer * np.sin(1.5 * theta)


def optimized_outer(theta_max: float) -> float:
    """Reading of the parameter-optimized operator: the outer weight b that
    minimizes the squared error of the modified wavenumber, integral over
    theta in [0, theta_max] of (K(k) h - theta)^2, a least-squares problem in
    b: K h - theta = e0 + b g with e0 = 2 sin(theta/2) - theta and
    g = 2 sin(3 theta/2) - 6 sin(theta/2), so b = -<e0, g> / <g, g>."""
    from scipy.integrate import quad

    def e0(t):
        return 2.0 * np.sin(t / 2.0) - t

    def g(t):
        return 2.0 * np.sin(1.5 * t) - 6.0 * np.sin(t / 2.0)
    num = quad(lambda t: e0(t) * g(t), 0.0, theta_max, epsabs=0.0, epsrel=1e-13, limit=200)[0]
    den = quad(lambda t: g(t) * g(t), 0.0, theta_max, epsabs=0.0, epsrel=1e-13, limit=200)[0]
    return -num / den


def diff4_to_half(f: np.ndarray, w: str, h: float, wts: np.ndarray = W4) -> np.ndarray:
    """Fourth-order difference of the E samples (integer positions 0..n along
    w, tangential to the walls at 0 and n) at the half-integer positions
    j+1/2 (stored at j, j = 0..n-1), with odd images across the walls.  The
    last entry (outside the box) is 0."""
    ax = AXIS[w]
    a = np.moveaxis(f, ax, -1)
    n = a.shape[-1] - 1
    ext = np.zeros(a.shape[:-1] + (n + 3,))     # positions -1 .. n+1
    ext[..., 1:n + 2] = a
    ext[..., 0] = -a[..., 1]
    ext[..., n + 2] = -a[..., n - 1]
    out = np.zeros_like(a)
    for j in range(n):                           # E at j-1, j, j+1, j+2 -> ext index +1
        out[..., j] = (wts[0] * ext[..., j] + wts[1] * ext[..., j + 1] + wts[2] * ext[..., j + 2]
                       + wts[3] * ext[..., j + 3]) / h
    return np.moveaxis(out, -1, ax)


def diff4_to_integer(f: np.ndarray, w: str, h: float, wts: np.ndarray = W4) -> np.ndarray:
    """Fourth-order difference of the H samples (positions j+1/2 stored at j,
    j = 0..n-1) at the integer positions j = 1..n-1, with even images across
    the walls.  Entries 0 and n (walls) are 0."""
    ax = AXIS[w]
    a = np.moveaxis(f, ax, -1)
    n = a.shape[-1] - 1
    ext = np.zeros(a.shape[:-1] + (n + 2,))     # stored -1 .. n
    ext[..., 1:n + 1] = a[..., 0:n]
    ext[..., 0] = a[..., 0]
    ext[..., n + 1] = a[..., n - 1]
    out = np.zeros_like(a)
    for j in range(1, n):                        # H stored j-2, j-1, j, j+1 -> ext index +1
        out[..., j] = (wts[0] * ext[..., j - 1] + wts[1] * ext[..., j] + wts[2] * ext[..., j + 1]
                       + wts[3] * ext[..., j + 2]) / h
    return np.moveaxis(out, -1, ax)


def d_int(f: np.ndarray, w: str, g: Grid) -> np.ndarray:
    """The grid's first difference of H samples along w at the E positions."""
    return diff4_to_integer(f, w, g.spacing(w), g.w4) if g.order == 4 else diff_to_integer(f, w, g.spacing(w))


def d_half(f: np.ndarray, w: str, g: Grid) -> np.ndarray:
    """The grid's first difference of E samples along w at the H positions."""
    return diff4_to_half(f, w, g.spacing(w), g.w4) if g.order == 4 else diff_to_half(f, w, g.spacing(w))


def apply_operator(op: str, u, g: Grid):
    """X u for X = A or B of eq. (AMat); returns a list of six arrays, zero at
    every non-dynamic node."""
    out = [np.zeros(g.shape) for _ in COMPONENTS]
    for ce, ch, w, s in PAIRS[op]:
        e, hh = u[CIDX[ce]], u[CIDX[ch]]
        out[CIDX[ce]] = s * d_int(hh, w, g) / g.eps * dynamic_mask(ce, g)
        out[CIDX[ch]] = s * d_half(e, w, g) / g.mu * dynamic_mask(ch, g)
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
