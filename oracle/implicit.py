"""Implicit line systems of one (E, H) pair, eliminated to a tridiagonal E system.

For a pair (E, H) of operator X along axis w with sign s (see ``yee.PAIRS``),
X acts as  E <- (s/eps) d_w H,  H <- (s/mu) d_w E.  An implicit equation

    (alpha I - (kappa_t) X) [E'; H'] = [f_E; f_H]

is solved by eliminating H' = (f_H + kappa_t (s/mu) d_w E') / alpha, which
leaves along every grid line of axis w the tridiagonal system

    alpha E' - (kappa_t^2 / alpha) (1/eps) d_w( (1/mu) d_w E' )
        = f_E + (kappa_t / alpha) (s/eps) d_w f_H .

Two instances appear in the paper:
* the original splitting formulae, (I - theta X) u' = rhs  (alpha = 1,
  kappa_t = theta), e.g. the implicit halves of (clsADI), (orgLOD), (orgSS2),
  (orgLOD2);
* the fundamental implicit updates, (1/2 I - theta/2 X) v = u (alpha = 1/2,
  kappa_t = theta/2), printed componentwise in Sec. III-A as
  1/2 E~ - (b d / 2) d_w^2 E~ = e + s b d_w h  with b = theta/eps, d = theta/mu
  (eq. (bd) has theta = dt/2).

d_w^2 is read as the composite d_w((1/mu) d_w .) of the two staggered first
differences (E -> H -> E), so with constant mu it is the 3-point second
difference scaled by b d.  The unknowns are the dynamic E nodes of each line,
with E' = 0 on both PEC walls at the line ends.

With the fourth-order differences of ``yee`` (grid order 4) the composite
couples each E node to three neighbours on either side: the line system is
assembled from the two difference matrices (images folded in) and solved
densely per line.
"""
from __future__ import annotations

import numpy as np

from .tridiag import thomas
from .yee import AXIS, CIDX, W4, Grid, d_half, d_int, dynamic_mask


def diff4_matrices(n: int, h: float, wts: np.ndarray = W4):
    """Matrices of the fourth-order differences on one line of n cells:
    Dh (n x (n-1)) maps the E unknowns j = 1..n-1 to the H samples j+1/2
    (j = 0..n-1); Di ((n-1) x n) maps the H samples to the E unknowns.  Images:
    E odd about the walls (E = 0 on them), H even."""
    Dh = np.zeros((n, n - 1))
    for hh in range(n):
        for t in range(4):                  # E position hh - 1 + t
            p, sgn = hh - 1 + t, 1.0
            if p < 0:
                p, sgn = -p, -1.0
            elif p > n:
                p, sgn = 2 * n - p, -1.0
            if 1 <= p <= n - 1:
                Dh[hh, p - 1] += sgn * wts[t] / h
    Di = np.zeros((n - 1, n))
    for j in range(1, n):
        for t in range(4):                  # H stored j - 2 + t
            q = j - 2 + t
            if q < 0:
                q = -1 - q
            elif q > n - 1:
                q = 2 * n - 1 - q
            Di[j - 1, q] += wts[t] / h
    return Dh, Di


def line_operator_solve(rhs_e: np.ndarray, ce: str, ch: str, w: str, coef: float,
                        alpha: float, g: Grid) -> np.ndarray:
    """Solve  alpha V - coef (1/eps) d_w((1/mu) d_w V) = rhs_e  on every line of
    axis w, for V at the nodes of E component `ce` (paired H component `ch`
    supplies the mu nodes).  Returns V on the full node array, 0 at every
    non-dynamic node of `ce`.
    """
    ax = AXIS[w]
    h = g.spacing(w)
    eps = np.moveaxis(g.eps, ax, -1)
    mu = np.moveaxis(g.mu, ax, -1)
    r = np.moveaxis(rhs_e, ax, -1)
    n = r.shape[-1] - 1  # cells along w; unknowns j = 1 .. n-1
    if n < 2:
        return np.zeros_like(rhs_e)
    if g.order == 4:
        # alpha V - coef (1/eps) Di (1/mu) Dh V, one dense system per line
        Dh, Di = diff4_matrices(n, h, g.w4)
        e_j = eps[..., 1:n]
        mu_h = mu[..., 0:n]
        K = np.einsum("jh,...h,hk->...jk", Di, 1.0 / mu_h, Dh)
        M = alpha * np.eye(n - 1) - coef * K / e_j[..., :, None]
        v = np.zeros_like(r)
        v[..., 1:n] = np.linalg.solve(M, r[..., 1:n, None])[..., 0]
        return np.moveaxis(v, -1, ax) * dynamic_mask(ce, g)
    e_j = eps[..., 1:n]
    mu_lo = mu[..., 0:n - 1]  # H node j-1/2 (stored at j-1)
    mu_hi = mu[..., 1:n]      # H node j+1/2 (stored at j)
    lo = -coef / (e_j * mu_lo * h * h)
    hi = -coef / (e_j * mu_hi * h * h)
    diag = alpha - lo - hi
    x = thomas(lo, diag, hi, r[..., 1:n])
    v = np.zeros_like(r)
    v[..., 1:n] = x
    v = np.moveaxis(v, -1, ax)
    return v * dynamic_mask(ce, g)


def pair_schur_rhs(f_e: np.ndarray, f_h: np.ndarray, w: str, s: int, kappa_t: float,
                   alpha: float, eps: np.ndarray, g: Grid) -> np.ndarray:
    """f_E + (kappa_t/alpha) (s/eps) d_w f_H  (right side after eliminating H)."""
    return f_e + (kappa_t / alpha) * s * d_int(f_h, w, g) / eps


def solve_implicit(op: str, pairs, f, theta: float, g: Grid):
    """Solve (I - theta X) u' = f for the six components (X = A or B, given by
    its pairs).  Non-dynamic nodes keep f (static normal H) or 0 (wall E)."""
    out = [np.array(a, copy=True) for a in f]
    for ce, ch, w, s in pairs:
        f_e, f_h = f[CIDX[ce]], f[CIDX[ch]]
        rhs = pair_schur_rhs(f_e, f_h, w, s, theta, 1.0, g.eps, g)
        e_new = line_operator_solve(rhs, ce, ch, w, theta * theta, 1.0, g)
        dyn_h = dynamic_mask(ch, g)
        h_new = np.where(dyn_h, f_h + theta * s * d_half(e_new, w, g) / g.mu, f_h)
        out[CIDX[ce]] = e_new
        out[CIDX[ch]] = h_new
    return out
