"""Dense-matrix schemes on tiny grids, with A and B assembled node by node.

The operators of eq. (AMat) are assembled here directly from Maxwell's curl
equations on the Yee grid -- one explicit loop over the dynamic nodes, each row
written from the positions of the two neighbouring samples -- without using the
vectorized difference code of ``yee``.  The vector u holds the dynamic nodes
only (static normal H is carried aside; wall E is 0).

Schemes are then the plain matrix formulae of Sec. II:
  original:    (clsADI), (orgLOD), (orgSS2), (orgLOD2)+(orgLOD2i)+(orgLOD2o)
  fundamental: (fasterADI)+(fastADIi)+(fasterADIo), (fastLOD), (fastSS2),
               (fastLOD2)+(fastLOD2i)+(fastLOD2o)
Every solve is ``numpy.linalg.solve`` on the dense system.

Grids of order 4 (the fourth-order staggered differences of ``yee``) are
assembled the same way, row by row, each row taking the four partner samples
along the pair's axis, folded onto their images across a PEC wall.
"""
from __future__ import annotations

import numpy as np

from .yee import COMPONENTS, CIDX, EPS0, MU0, PAIRS, Grid, dynamic_mask


class DenseSystem:
    def __init__(self, g: Grid, sparse: bool = False):
        self.g = g
        self.index = {}
        self.nodes = []
        for c in COMPONENTS:
            m = dynamic_mask(c, g)
            for k, j, i in zip(*np.nonzero(m)):
                self.index[(c, int(k), int(j), int(i))] = len(self.nodes)
                self.nodes.append((c, int(k), int(j), int(i)))
        self.n = len(self.nodes)
        if sparse:   # same assembly into (row, col, value) lists (larger grids)
            self.A, self.B = [], []
        else:
            self.A = np.zeros((self.n, self.n))
            self.B = np.zeros((self.n, self.n))
        if g.order == 4:
            self._assemble4()
        else:
            self._assemble()
        if sparse:
            from scipy.sparse import csr_matrix
            self.A, self.B = ([csr_matrix((np.array([t[2] for t in M]), ([t[0] for t in M], [t[1] for t in M])),
                                          shape=(self.n, self.n)) for M in (self.A, self.B)])
        self.w = np.array([self._material(c, k, j, i) for c, k, j, i in self.nodes])

    def _material(self, c, k, j, i):
        g = self.g
        kk, jj, ii = min(k, g.nz - 1), min(j, g.ny - 1), min(i, g.nx - 1)
        if c[0] == "E":
            return EPS0 * g.eps_r[kk, jj, ii]
        return MU0 * g.mu_r[kk, jj, ii]

    def _add(self, M, row, comp, k, j, i, val):
        col = self.index.get((comp, k, j, i))
        if col is None:
            # only wall E (which is 0) may be referenced outside the dynamic set
            assert comp[0] == "E", (comp, k, j, i)
            return
        if isinstance(M, list):
            M.append((row, col, val))   # duplicates are summed by csr_matrix
        else:
            M[row, col] += val

    def _assemble(self):
        g = self.g
        dx, dy, dz = g.dx, g.dy, g.dz
        A, B = self.A, self.B
        for r, (c, k, j, i) in enumerate(self.nodes):
            inv = 1.0 / self._material(c, k, j, i)
            if c == "Ex":   # at (i+1/2, j, k)
                # A: (1/eps) dHz/dy ; Hz at (i+1/2, j+-1/2, k)
                self._add(A, r, "Hz", k, j, i, inv / dy)
                self._add(A, r, "Hz", k, j - 1, i, -inv / dy)
                # B: -(1/eps) dHy/dz ; Hy at (i+1/2, j, k+-1/2)
                self._add(B, r, "Hy", k, j, i, -inv / dz)
                self._add(B, r, "Hy", k - 1, j, i, inv / dz)
            elif c == "Ey":  # at (i, j+1/2, k)
                self._add(A, r, "Hx", k, j, i, inv / dz)       # dHx/dz, Hx at (i, j+1/2, k+-1/2)
                self._add(A, r, "Hx", k - 1, j, i, -inv / dz)
                self._add(B, r, "Hz", k, j, i, -inv / dx)      # -dHz/dx, Hz at (i+-1/2, j+1/2, k)
                self._add(B, r, "Hz", k, j, i - 1, inv / dx)
            elif c == "Ez":  # at (i, j, k+1/2)
                self._add(A, r, "Hy", k, j, i, inv / dx)       # dHy/dx, Hy at (i+-1/2, j, k+1/2)
                self._add(A, r, "Hy", k, j, i - 1, -inv / dx)
                self._add(B, r, "Hx", k, j, i, -inv / dy)      # -dHx/dy, Hx at (i, j+-1/2, k+1/2)
                self._add(B, r, "Hx", k, j - 1, i, inv / dy)
            elif c == "Hx":  # at (i, j+1/2, k+1/2)
                self._add(A, r, "Ey", k + 1, j, i, inv / dz)   # dEy/dz, Ey at (i, j+1/2, k+1/2+-1/2)
                self._add(A, r, "Ey", k, j, i, -inv / dz)
                self._add(B, r, "Ez", k, j + 1, i, -inv / dy)  # -dEz/dy, Ez at (i, j+1/2+-1/2, k+1/2)
                self._add(B, r, "Ez", k, j, i, inv / dy)
            elif c == "Hy":  # at (i+1/2, j, k+1/2)
                self._add(A, r, "Ez", k, j, i + 1, inv / dx)   # dEz/dx
                self._add(A, r, "Ez", k, j, i, -inv / dx)
                self._add(B, r, "Ex", k + 1, j, i, -inv / dz)  # -dEx/dz
                self._add(B, r, "Ex", k, j, i, inv / dz)
            elif c == "Hz":  # at (i+1/2, j+1/2, k)
                self._add(A, r, "Ex", k, j + 1, i, inv / dy)   # dEx/dy
                self._add(A, r, "Ex", k, j, i, -inv / dy)
                self._add(B, r, "Ey", k, j, i + 1, -inv / dx)  # -dEy/dx
                self._add(B, r, "Ey", k, j, i, inv / dx)

    def _assemble4(self):
        """A and B with the fourth-order differences: for the pair (E, H, w, s)
        of an operator, an E row at integer position p along w takes the H
        samples at p - 3/2 .. p + 3/2 (stored p-2 .. p+1) with the grid's 4-point weights / h
        times s/eps; an H row at p + 1/2 takes the E samples at p-1 .. p+2 times
        s/mu.  Across a wall an H sample is its even image, an E sample its odd
        image (a wall E itself is 0)."""
        g = self.g
        W = g.w4
        cells = {"x": g.nx, "y": g.ny, "z": g.nz}
        for r, (c, k, j, i) in enumerate(self.nodes):
            inv = 1.0 / self._material(c, k, j, i)
            for name in ("A", "B"):
                M = self.op(name)
                for ce, ch, w, s in PAIRS[name]:
                    if c not in (ce, ch):
                        continue
                    n, h = cells[w], g.spacing(w)
                    pos = {"x": i, "y": j, "z": k}[w]

                    def at(q):
                        return (q, j, i) if w == "z" else ((k, q, i) if w == "y" else (k, j, q))
                    for t in range(4):
                        if c == ce:
                            q = pos - 2 + t                       # H stored index
                            if q < 0:
                                q = -1 - q
                            elif q > n - 1:
                                q = 2 * n - 1 - q
                            self._add(M, r, ch, *at(q), s * inv * W[t] / h)
                        else:
                            q, sgn = pos - 1 + t, 1.0             # E position
                            if q < 0:
                                q, sgn = -q, -1.0
                            elif q > n:
                                q, sgn = 2 * n - q, -1.0
                            self._add(M, r, ce, *at(q), sgn * s * inv * W[t] / h)

    # -- conversions --------------------------------------------------------
    def to_vec(self, u) -> np.ndarray:
        return np.array([u[CIDX[c]][k, j, i] for c, k, j, i in self.nodes])

    def from_vec(self, x: np.ndarray, template) -> list:
        out = [np.array(a, dtype=np.float64, copy=True) for a in template]
        for n, c in enumerate(COMPONENTS):
            if c[0] == "E":
                out[n][~dynamic_mask(c, self.g)] = 0.0
        for v, (c, k, j, i) in zip(x, self.nodes):
            out[CIDX[c]][k, j, i] = v
        return out

    def op(self, name: str) -> np.ndarray:
        return {"A": self.A, "B": self.B}[name]

    def src_vec(self, source, val: float) -> np.ndarray:
        gvec = np.zeros(self.n)
        if source is not None and val != 0.0:
            gvec[self.index[("Ez", source.k, source.j, source.i)]] = val
        return gvec

    def energy(self, x: np.ndarray) -> float:
        return float(np.sum(self.w * x * x))


# ----------------------------------------------------------------------------
# matrix schemes
# ----------------------------------------------------------------------------

_ORIG = {  # (X, Y, theta/dt, source time within the step)
    "adi": (("A", "B", 0.5, 0.25), ("B", "A", 0.5, 0.75)),
    "lod1": (("A", "A", 0.5, 0.25), ("B", "B", 0.5, 0.75)),
    "ss2": (("A", "A", 0.25, 0.125), ("B", "B", 0.5, 0.5), ("A", "A", 0.25, 0.875)),
    "lod2": (("A", "A", 0.5, 0.5), ("B", "B", 0.5, 1.0)),
}


def run_original(ds: DenseSystem, scheme: str, x0: np.ndarray, steps: int, source=None):
    """Original splitting formulae; returns (x at step `steps`, invariant trace)."""
    g, I = ds.g, np.eye(ds.n)
    x = x0.copy()
    if scheme == "lod2":  # (orgLOD2i)
        th = 0.25 * g.dt
        x = np.linalg.solve(I - th * ds.B, (I + th * ds.B) @ x)
    trace = [_invariant_orig(ds, scheme, x)]
    for n in range(steps):
        for xo, yo, tf, tt in _ORIG[scheme]:
            th = tf * g.dt
            rhs = (I + th * ds.op(yo)) @ x
            if source is not None:
                rhs = rhs + ds.src_vec(source, source.g(th, (n + tt) * g.dt))
            x = np.linalg.solve(I - th * ds.op(xo), rhs)
        trace.append(_invariant_orig(ds, scheme, x))
    if scheme == "lod2":  # (orgLOD2o)
        th = 0.25 * g.dt
        x = np.linalg.solve(I + th * ds.B, (I - th * ds.B) @ x)
    return x, trace


def _invariant_orig(ds, scheme, x):
    if scheme == "adi":
        return 0.25 * ds.energy(x + 0.5 * ds.g.dt * (ds.B @ x))
    return ds.energy(x)


def run_fundamental(ds: DenseSystem, scheme: str, x0: np.ndarray, steps: int, source=None):
    """Fundamental matrix iterations; returns (x at step `steps`, invariant trace)."""
    g, I = ds.g, np.eye(ds.n)
    dt = g.dt
    if scheme == "adi":
        # (fastADIi), (uTldCol); iteration (fasterADI); output (fasterADIo)
        v = (I - 0.5 * dt * ds.B) @ x0          # v^{-1/2}
        ut = 2.0 * x0
        trace = [0.25 * ds.energy(ut - v)]
        for n in range(steps):
            v = ut - v + ds.src_vec(source, source.g(0.5 * dt, (n + 0.25) * dt) if source else 0.0)
            ut = np.linalg.solve(0.5 * I - 0.25 * dt * ds.A, v)
            v = ut - v + ds.src_vec(source, source.g(0.5 * dt, (n + 0.75) * dt) if source else 0.0)
            ut = np.linalg.solve(0.5 * I - 0.25 * dt * ds.B, v)
            trace.append(0.25 * ds.energy(ut - v))
        return 0.5 * ut, trace
    u = x0.copy()
    if scheme == "lod2":  # (fastLOD2i)
        vq = np.linalg.solve(0.5 * I - dt / 8 * ds.B, u)
        u = vq - u
    trace = [ds.energy(u)]
    for n in range(steps):
        for xo, _, tf, tt in _ORIG[scheme]:
            th = tf * dt
            gval = source.g(th, (n + tt) * dt) if source is not None else 0.0
            v = np.linalg.solve(0.5 * I - 0.5 * th * ds.op(xo), u + 0.5 * ds.src_vec(source, gval))
            u = v - u
        trace.append(ds.energy(u))
    if scheme == "lod2":  # (fastLOD2o)
        v = np.linalg.solve(0.5 * I + dt / 8 * ds.B, u)
        u = v - u
    return u, trace


# ----------------------------------------------------------------------------
# further splittings of Sec. II-E: D'Yakonov and Douglas-Gunn (no sources)
# ----------------------------------------------------------------------------

def run_splitting_original(ds: DenseSystem, scheme: str, x0: np.ndarray, steps: int):
    """Original splitting formulae of Sec. II-E on matrices.

    "dy", eq. (orgDY):  (I - dt/2 A) u* = (I + dt/2 A)(I + dt/2 B) u^n ,
                        (I - dt/2 B) u^{n+1} = u* ;
    "dg", the delta formulation (before (fastDGo)):
                        (I - dt/2 A) du* = dt (A + B) u^n ,
                        (I - dt/2 B) du = du* ,   u^{n+1} = u^n + du .
    Returns (u^steps, per-step intermediates): u* for "dy", (du*, du) for "dg".
    """
    I, h = np.eye(ds.n), 0.5 * ds.g.dt
    x = x0.copy()
    mids = []
    for _ in range(steps):
        if scheme == "dy":
            ustar = np.linalg.solve(I - h * ds.A, (I + h * ds.A) @ ((I + h * ds.B) @ x))
            x = np.linalg.solve(I - h * ds.B, ustar)
            mids.append(ustar)
        elif scheme == "dg":
            dstar = np.linalg.solve(I - h * ds.A, ds.g.dt * ((ds.A + ds.B) @ x))
            du = np.linalg.solve(I - h * ds.B, dstar)
            x = x + du
            mids.append((dstar, du))
        else:
            raise ValueError(scheme)
    return x, mids


def run_splitting_fundamental(ds: DenseSystem, scheme: str, x0: np.ndarray, steps: int, source=None):
    """Fundamental forms of the same splittings (Sec. II-E).

    "dy", eq. (fastDY) with its input v^{-1/2} = (1/2 I - dt/4 B) u^0:
        v^n = u^n - v^{n-1/2};  (1/2 I - dt/4 A) u^{n+1/2} = v^n;
        v^{n+1/2} = u^{n+1/2} - v^n;  (1/2 I - dt/4 B) u^{n+1} = v^{n+1/2};
      intermediate u* = 2 v^{n+1/2}.
    "dg", the ADI iteration (fasterADI) with (fastADIi) and (uTldCol), and the
      increments of (fastDGo): du* = u~^{n+1/2} - u~^n, du = (u~^{n+1} - u~^n)/2,
      accumulated as u^{n+1} = u^n + du.
    A source enters as in ADI (the convention of ``source``): the term g of each
    sub-step is added to the auxiliary subtraction, as g in the u~ scaling of
    (fasterADI) and as g/2 in the unscaled variables of (fastDY).
    Returns the same as ``run_splitting_original``.
    """
    g, I = ds.g, np.eye(ds.n)
    q = 0.25 * g.dt
    mids = []
    if scheme == "dy":
        v = (0.5 * I - q * ds.B) @ x0            # v^{-1/2}
        u = x0.copy()
        for n in range(steps):
            gA = ds.src_vec(source, source.g(0.5 * g.dt, (n + 0.25) * g.dt)) if source else 0.0
            gB = ds.src_vec(source, source.g(0.5 * g.dt, (n + 0.75) * g.dt)) if source else 0.0
            v = u - v + 0.5 * gA                 # v^n
            uh = np.linalg.solve(0.5 * I - q * ds.A, v)
            v = uh - v + 0.5 * gB                # v^{n+1/2}
            u = np.linalg.solve(0.5 * I - q * ds.B, v)
            mids.append(2.0 * v)
        return u, mids
    if scheme == "dg":
        v = (I - 0.5 * g.dt * ds.B) @ x0         # v^{-1/2}, (fastADIi)
        ut = 2.0 * x0                            # u~^0, (uTldCol)
        u = x0.copy()
        for n in range(steps):
            gA = ds.src_vec(source, source.g(0.5 * g.dt, (n + 0.25) * g.dt)) if source else 0.0
            gB = ds.src_vec(source, source.g(0.5 * g.dt, (n + 0.75) * g.dt)) if source else 0.0
            v = ut - v + gA
            uth = np.linalg.solve(0.5 * I - q * ds.A, v)
            dstar = uth - ut
            v = uth - v + gB
            utn = np.linalg.solve(0.5 * I - q * ds.B, v)
            du = 0.5 * (utn - ut)
            u = u + du
            ut = utn
            mids.append((dstar, du))
        return u, mids
    raise ValueError(scheme)
