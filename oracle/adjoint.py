"""Reference gradient of a probe objective with respect to eps_r (tiny grids).

Objective: J = sum_{n=1..N} dt * (Ex^2 + Ey^2 + Ez^2) of the ADI field at the
probe node (the E samples stored at the probe cell's node index).

The ADI field follows the original splitting formula (clsADI) with the point
source convention of ``source``:
    phi^{n+1/2} = (I - th A)^{-1} [(I + th B) phi^n + g_A],
    phi^{n+1}   = (I - th B)^{-1} [(I + th A) phi^{n+1/2} + g_B],   th = dt/2,
which the fundamental ADI reproduces exactly (Sec. II-A).  eps enters only
the E rows of A and B (1/eps), so dA/deps_i = -(1/eps_i) e_i e_i^T A, and the
gradient follows by reverse-mode differentiation of the two linear solves per
step, written out on the dense matrices of ``dense``.  The gradient is with
respect to eps_r of each cell: the cell's value enters the Ex, Ey, Ez samples
stored at its node index.
"""
from __future__ import annotations

import numpy as np

from .dense import DenseSystem
from .yee import EPS0, Grid


def _probe_rows(ds: DenseSystem, probe):
    i, j, k = probe
    return [ds.index[(c, k, j, i)] for c in ("Ex", "Ey", "Ez") if (c, k, j, i) in ds.index]


def objective(g: Grid, u0, steps: int, source, probe):
    """J for the given grid (dense ADI, FP64)."""
    ds = DenseSystem(g)
    return _forward(ds, ds.to_vec(u0), steps, source, probe)[0]


def _forward(ds, x0, steps, source, probe):
    g, I = ds.g, np.eye(ds.n)
    th = 0.5 * g.dt
    rows = _probe_rows(ds, probe)
    LA, LB = I - th * ds.A, I - th * ds.B
    RA, RB = I + th * ds.A, I + th * ds.B
    phis = [x0.copy()]
    halves = []
    J = 0.0
    x = x0.copy()
    for n in range(steps):
        ga = ds.src_vec(source, source.g(th, (n + 0.25) * g.dt)) if source is not None else 0.0
        gb = ds.src_vec(source, source.g(th, (n + 0.75) * g.dt)) if source is not None else 0.0
        xh = np.linalg.solve(LA, RB @ x + ga)
        x = np.linalg.solve(LB, RA @ xh + gb)
        halves.append(xh)
        phis.append(x)
        J += g.dt * float(np.sum(x[rows] ** 2))
    return J, phis, halves


def gradient(g: Grid, u0, steps: int, source, probe):
    """(J, dJ/deps_r per cell as an (nz, ny, nx) array)."""
    ds = DenseSystem(g)
    I = np.eye(ds.n)
    th = 0.5 * g.dt
    rows = _probe_rows(ds, probe)
    J, phis, halves = _forward(ds, ds.to_vec(u0), steps, source, probe)
    LA, LB = I - th * ds.A, I - th * ds.B
    RA, RB = I + th * ds.A, I + th * ds.B
    eps_abs = ds.w.copy()            # eps at E rows (mu at H rows, unused)
    is_e = np.array([c[0] == "E" for c, *_ in ds.nodes])
    grad_node = np.zeros(ds.n)       # dJ/d eps (absolute) per E row
    lam = np.zeros(ds.n)             # adjoint of phi^{n+1}
    for n in range(steps - 1, -1, -1):
        phi1, phih, phi0 = phis[n + 1], halves[n], phis[n]
        lam = lam.copy()
        lam[rows] += 2.0 * g.dt * phi1[rows]
        # phi^{n+1} = LB^{-1} (RA phih + gB):  z = LB^{-T} lam
        z = np.linalg.solve(LB.T, lam)
        # d/deps_i of (RA phih - LB phi1) = th (dA phih + dB phi1), dX = -(1/eps_i) e_i e_i^T X
        grad_node += -(th / eps_abs) * z * (ds.A @ phih + ds.B @ phi1) * is_e
        lam_h = RA.T @ z
        # phih = LA^{-1} (RB phi0 + gA):  w = LA^{-T} lam_h
        w = np.linalg.solve(LA.T, lam_h)
        grad_node += -(th / eps_abs) * w * (ds.B @ phi0 + ds.A @ phih) * is_e
        lam = RB.T @ w
    grad = np.zeros((g.nz, g.ny, g.nx))
    for val, (c, k, j, i) in zip(grad_node, ds.nodes):
        if c[0] == "E" and val != 0.0:
            grad[k, j, i] += EPS0 * val
    return J, grad
