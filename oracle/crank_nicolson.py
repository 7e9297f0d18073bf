"""Crank-Nicolson without factorization (Sec. II-E, closing part).

Original form, the classical scheme with both operators on each side:

    [I - dt/2 (A + B)] u^{n+1} = [I + dt/2 (A + B)] u^n ;

fundamental form, with the matrix-operator-free right side:

    [1/2 I - dt/4 (A + B)] u^{n+1/2} = u^n ,   u^{n+1} = u^{n+1/2} - u^n .

A and B are the operators of eq. (AMat), assembled node by node by
``dense.DenseSystem`` (sparse storage for grids beyond a few hundred nodes).
Each form's matrix is factorized once by a sparse direct LU
(``scipy.sparse.linalg.splu``); a step is one solve.  The paper gives the
scheme without a nonhomogeneous term; a source, if given, follows the
convention of ``source`` (one term per step, at its middle).  Without one,
being the Cayley transform of an operator that is skew-adjoint in the energy
norm, a step conserves W(u) = sum eps E^2 + mu H^2 exactly.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from .dense import DenseSystem
from .yee import Grid, clean, energy


def run(ds: DenseSystem, x0: np.ndarray, steps: int, form: str = "fundamental", source=None):
    """Advance the dynamic-node vector x0 by `steps` steps; returns (x, W trace).

    A source adds, by the convention of ``source``, g = theta amp p(t) with
    theta = dt/2 at the middle t = (n + 1/2) dt of step n: to the right side of
    the classical form, and as g/2 to u^n in the fundamental form (whose
    u^{n+1} = u^{n+1/2} - u^n is unchanged)."""
    n, dt = ds.n, ds.g.dt
    I = sp.identity(n, format="csc")
    K = sp.csc_matrix(ds.A + ds.B)
    x = np.array(x0, dtype=np.float64, copy=True)
    trace = [ds.energy(x)]
    if form == "fundamental":
        lu = splu(sp.csc_matrix(0.5 * I - 0.25 * dt * K))
        for n in range(steps):
            gv = ds.src_vec(source, source.g(0.5 * dt, (n + 0.5) * dt)) if source is not None else 0.0
            xh = lu.solve(x + 0.5 * gv)   # u^{n+1/2}
            x = xh - x                    # u^{n+1}
            trace.append(ds.energy(x))
    elif form == "conventional":
        lu = splu(sp.csc_matrix(I - 0.5 * dt * K))
        rhs_op = sp.csr_matrix(I + 0.5 * dt * K)
        for n in range(steps):
            gv = ds.src_vec(source, source.g(0.5 * dt, (n + 0.5) * dt)) if source is not None else 0.0
            x = lu.solve(rhs_op @ x + gv)
            trace.append(ds.energy(x))
    else:
        raise ValueError(form)
    return x, trace


def run_fields(g: Grid, fields, steps: int, form: str = "fundamental", energy_every: int = 0, source=None):
    """Six node arrays in, six out (wall-tangential E treated as 0, static
    normal H passed through); trace at steps 0, e, 2e, ... (e = energy_every)."""
    u = clean(fields, g)
    ds = DenseSystem(g, sparse=True)
    x0 = ds.to_vec(u)
    x, tr = run(ds, x0, steps, form, source)
    # the trace is W over all samples: the static normal H on the walls, which
    # the dynamic-node vector leaves out, adds a constant
    static = energy(u, g) - ds.energy(x0)
    trace = [t + static for t in tr[::energy_every]] if energy_every else []
    return ds.from_vec(x, u), trace
