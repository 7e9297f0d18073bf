"""Closed-form pins that do not come from the oracle.

PEC cavity modes on the Yee grid.  For integer mode numbers (m, n, p) the fields

    Ex = a1 cos(kx x) sin(ky y) sin(kz z)   Hx = a4 sin(kx x) cos(ky y) cos(kz z)
    Ey = a2 sin(kx x) cos(ky y) sin(kz z)   Hy = a5 cos(kx x) sin(ky y) cos(kz z)
    Ez = a3 sin(kx x) sin(ky y) cos(kz z)   Hz = a6 cos(kx x) cos(ky y) sin(kz z)

(k_w = m_w pi / L_w), sampled at the Yee positions, satisfy the PEC walls, and
the staggered central difference maps each profile to another one of the set:
  d_w sin(k_w w) = K_w cos(k_w w),  d_w cos(k_w w) = -K_w sin(k_w w),
  K_w = (2/dw) sin(k_w dw / 2)
(order 2).  The fourth-order staggered difference (1, -27, 27, -1)/(24 dw) maps
them the same way with K_w = (27 sin(k_w dw / 2) - sin(3 k_w dw / 2)) / (12 dw)
(order 4), since the odd/even images across the PEC walls continue the sines
and cosines.
Hence the operators A and B of eq. (AMat) act on the six amplitudes as exact
6x6 matrices (below), every scheme acts on them as a product of 6x6 Cayley
factors, and the exact semi-discrete solution is expm(t (A + B)).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sl

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
C0 = 1.0 / math.sqrt(EPS0 * MU0)


def wavenumbers(nx, ny, nz, dx, dy, dz, m, n, p, order=2, outer=None):
    """outer: order 4 with the outer weight b of the 4-point difference
    [(1 - 3b)(f[+1/2] - f[-1/2]) + b (f[+3/2] - f[-3/2])] / dw, which maps the
    profiles with K_w = (2/dw) ((1 - 3b) sin(k_w dw/2) + b sin(3 k_w dw/2))."""
    k = (m * math.pi / (nx * dx), n * math.pi / (ny * dy), p * math.pi / (nz * dz))
    if order == 4 and outer is not None:
        K = tuple(2.0 / h * ((1.0 - 3.0 * outer) * math.sin(kw * h / 2.0) + outer * math.sin(1.5 * kw * h))
                  for kw, h in zip(k, (dx, dy, dz)))
    elif order == 4:
        K = tuple((27.0 * math.sin(kw * h / 2.0) - math.sin(1.5 * kw * h)) / (12.0 * h)
                  for kw, h in zip(k, (dx, dy, dz)))
    else:
        K = tuple(2.0 / h * math.sin(kw * h / 2.0) for kw, h in zip(k, (dx, dy, dz)))
    return k, K


def mode_matrices(nx, ny, nz, dx, dy, dz, m, n, p, eps=EPS0, mu=MU0, order=2, outer=None):
    """6x6 matrices of A and B on the amplitudes (a1..a6) of the (m, n, p) mode."""
    _, (Kx, Ky, Kz) = wavenumbers(nx, ny, nz, dx, dy, dz, m, n, p, order, outer)
    A = np.zeros((6, 6))
    B = np.zeros((6, 6))
    # A: Ex<-(1/eps) dy Hz, Ey<-(1/eps) dz Hx, Ez<-(1/eps) dx Hy, Hx<-(1/mu) dz Ey, ...
    A[0, 5] = -Ky / eps
    A[1, 3] = -Kz / eps
    A[2, 4] = -Kx / eps
    A[3, 1] = Kz / mu
    A[4, 2] = Kx / mu
    A[5, 0] = Ky / mu
    # B: Ex<- -(1/eps) dz Hy, Ey<- -(1/eps) dx Hz, Ez<- -(1/eps) dy Hx, ...
    B[0, 4] = Kz / eps
    B[1, 5] = Kx / eps
    B[2, 3] = Ky / eps
    B[3, 2] = -Ky / mu
    B[4, 0] = -Kz / mu
    B[5, 1] = -Kx / mu
    return A, B


def _extent(comp, nx, ny, nz):
    m = np.ones((nz + 1, ny + 1, nx + 1), dtype=bool)
    if comp in ("Ex", "Hy", "Hz"):
        m[:, :, nx] = False
    if comp in ("Ey", "Hx", "Hz"):
        m[:, ny, :] = False
    if comp in ("Ez", "Hx", "Hy"):
        m[nz, :, :] = False
    return m


def mode_fields(nx, ny, nz, dx, dy, dz, m, n, p, amps):
    """The six node arrays [k, j, i] of the mode with amplitudes `amps`."""
    (kx, ky, kz), _ = wavenumbers(nx, ny, nz, dx, dy, dz, m, n, p)
    k = np.arange(nz + 1)[:, None, None]
    j = np.arange(ny + 1)[None, :, None]
    i = np.arange(nx + 1)[None, None, :]

    def X(h):
        return kx * (i + h) * dx

    def Y(h):
        return ky * (j + h) * dy

    def Z(h):
        return kz * (k + h) * dz

    prof = [
        np.cos(X(.5)) * np.sin(Y(0)) * np.sin(Z(0)),
        np.sin(X(0)) * np.cos(Y(.5)) * np.sin(Z(0)),
        np.sin(X(0)) * np.sin(Y(0)) * np.cos(Z(.5)),
        np.sin(X(0)) * np.cos(Y(.5)) * np.cos(Z(.5)),
        np.cos(X(.5)) * np.sin(Y(0)) * np.cos(Z(.5)),
        np.cos(X(.5)) * np.cos(Y(.5)) * np.sin(Z(0)),
    ]
    out = []
    for c, a, f in zip(("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"), amps, prof):
        v = a * f * _extent(c, nx, ny, nz)
        # sin() at the far wall is ~1e-16, not 0: zero the wall-tangential E exactly
        if c == "Ex":
            v[:, [0, ny], :] = 0.0
            v[[0, nz], :, :] = 0.0
        elif c == "Ey":
            v[:, :, [0, nx]] = 0.0
            v[[0, nz], :, :] = 0.0
        elif c == "Ez":
            v[:, :, [0, nx]] = 0.0
            v[:, [0, ny], :] = 0.0
        out.append(v)
    return out


def cayley(X, theta):
    I = np.eye(X.shape[0])
    return np.linalg.solve(I - theta * X, I + theta * X)


def scheme_matrix(scheme, A, B, dt):
    """One main iteration of each scheme on the 6 amplitudes (original form)."""
    I = np.eye(6)
    h = dt / 2
    if scheme == "adi":
        half = np.linalg.solve(I - h * A, I + h * B)
        return np.linalg.solve(I - h * B, (I + h * A) @ half)
    if scheme in ("lod1", "lod2"):
        return cayley(B, h) @ cayley(A, h)
    if scheme == "ss2":
        return cayley(A, dt / 4) @ cayley(B, dt / 2) @ cayley(A, dt / 4)
    raise ValueError(scheme)


def lod2_io(B, dt):
    """LOD2 input (orgLOD2i) and output (orgLOD2o) matrices."""
    return cayley(B, dt / 4), cayley(B, -dt / 4)


def exact(A, B, t):
    return sl.expm(t * (A + B))


def adi_dispersion_cos(nx, ny, nz, dx, dy, dz, m, n, p, dt, c=C0, order=2):
    """Closed form cos(w~ dt) of the ADI amplification on mode (m, n, p):
    (cx cy + cy cz + cz cx - 1)/2 with c_w = (1 - s_w^2)/(1 + s_w^2),
    s_w = (c dt / 2) K_w (order 2: (c dt / dw) sin(k_w dw / 2))."""
    _, K = wavenumbers(nx, ny, nz, dx, dy, dz, m, n, p, order)
    s = [c * dt / 2 * Kw for Kw in K]
    cw = [(1 - x * x) / (1 + x * x) for x in s]
    return (cw[0] * cw[1] + cw[1] * cw[2] + cw[2] * cw[0] - 1) / 2


def cn_phase(nx, ny, nz, dx, dy, dz, m, n, p, dt, c=C0):
    """Phase per step of Crank-Nicolson on mode (m, n, p): the Cayley factor of
    dt (A + B)/2 maps the eigenvalues +-i w of A + B, w = c |K| (the Yee
    frequency), to e^{+-i phi} with phi = 2 atan(w dt / 2)."""
    _, K = wavenumbers(nx, ny, nz, dx, dy, dz, m, n, p)
    w = c * math.sqrt(sum(k * k for k in K))
    return 2.0 * math.atan(0.5 * w * dt)
