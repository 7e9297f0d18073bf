"""Pin of the reference gradient (oracle/adjoint.py) against central finite
differences of the FP64 objective (brute force)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, yee
from oracle.source import Source


def _case(seed=0):
    nx, ny, nz = 4, 3, 5
    rng = np.random.default_rng(seed)
    eps = rng.uniform(1, 12, (nz, ny, nx))
    dt = yee.cfl_dt(1e-3, 1e-3, 1e-3, 5.0)
    g = yee.Grid(nx, ny, nz, 1e-3, 1e-3, 1e-3, dt, eps)
    u0 = W.random_fields(nx, ny, nz, seed + 1)
    src = Source(1, 1, 2, amp=1e12, t0=2 * dt, tau=3 * dt, f0=1 / (8 * dt))
    return g, u0, src, (2, 1, 3)


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_fd(seed):
    g, u0, src, probe = _case(seed)
    J, grad = adjoint.gradient(g, u0, 8, src, probe)
    assert J > 0
    h = 1e-5
    cells = [(0, 0, 0), (3, 1, 2), (2, 2, 1), (1, 0, 3), (4, 2, 3)]
    for (k, j, i) in cells:
        e = g.eps_r.copy()
        e[k, j, i] += h
        gp = yee.Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.dt, e)
        e = g.eps_r.copy()
        e[k, j, i] -= h
        gm = yee.Grid(g.nx, g.ny, g.nz, g.dx, g.dy, g.dz, g.dt, e)
        fd = (adjoint.objective(gp, u0, 8, src, probe) - adjoint.objective(gm, u0, 8, src, probe)) / (2 * h)
        assert abs(fd - grad[k, j, i]) <= 1e-6 * np.abs(grad).max() + 1e-7 * abs(fd), ((k, j, i), fd, grad[k, j, i])


def test_gradient_zero_outside_dependence():
    """Cells whose E samples are all walls (last cell layer owns only far-wall
    nodes for some components) still get a finite, consistent gradient; the
    objective is unchanged by eps of a cell with no dynamic E sample."""
    g, u0, src, probe = _case(3)
    J, grad = adjoint.gradient(g, u0, 4, src, probe)
    assert np.all(np.isfinite(grad))


@pytest.mark.parametrize("op", ["A", "B"])
@pytest.mark.parametrize("theta_scale", [0.3, 2.5])
def test_cayley_transpose_is_reverse_step_in_scaled_variables(op, theta_scale):
    """The identity the adjoint rests on: with M = diag(eps, mu) and X = A or B
    of eq. (AMat), C(theta) = (I - theta X)^-1 (I + theta X) satisfies
    C(theta)^T = M C(-theta) M^-1 (X = M^-1 K with K skew-symmetric), checked
    on assembled matrices of a random medium; and the dot-product identity
    <C d, w> = <d, C^T w> holds for the matrix the reverse sweep applies."""
    from oracle.dense import DenseSystem
    nx, ny, nz = 4, 3, 5
    rng = np.random.default_rng(7)
    eps = rng.uniform(1, 12, (nz, ny, nx))
    mu = rng.uniform(1, 3, (nz, ny, nx))
    dt = yee.cfl_dt(1e-3, 1e-3, 1e-3, 5.0)
    g = yee.Grid(nx, ny, nz, 1e-3, 1.3e-3, 0.8e-3, dt, eps, mu)
    ds = DenseSystem(g)
    X = ds.A if op == "A" else ds.B
    I = np.eye(ds.n)
    th = theta_scale * dt
    C = lambda t: np.linalg.solve(I - t * X, I + t * X)
    Mw = np.diag(ds.w)
    Mi = np.diag(1.0 / ds.w)
    lhs = C(th).T
    rhs = Mw @ C(-th) @ Mi
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(lhs).max()
    # K = M X is skew-symmetric (the structural fact behind the identity)
    K = Mw @ X
    assert np.abs(K + K.T).max() <= 1e-12 * np.abs(K).max()
    d, w = rng.standard_normal(ds.n), rng.standard_normal(ds.n)
    assert abs((C(th) @ d) @ w - d @ (rhs @ w)) <= 1e-11 * np.linalg.norm(d) * np.linalg.norm(w)
