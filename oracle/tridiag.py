"""Thomas algorithm (tridiagonal LU without pivoting), vectorized over lines.

Sec. IV of the paper prices a tridiagonal system of order N at about 5N flops
"using precomputed bidiagonally factorized elements", i.e. Gaussian elimination
specialised to three diagonals.  Every implicit system of the method is
strictly diagonally dominant (diagonal 1 + 2 beta against off-diagonals beta,
or 1/2 + 2 beta against beta in the fundamental scaling), so no pivoting is
needed.
"""
from __future__ import annotations

import numpy as np


def thomas(a: np.ndarray, b: np.ndarray, c: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Solve a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j along the LAST axis.

    All four arrays have the same shape (..., n); a[..., 0] and c[..., n-1] are
    ignored (the unknowns outside the line are 0).  Leading axes are
    independent lines.  FP64.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[-1]
    cp = np.empty_like(d)
    dp = np.empty_like(d)
    cp[..., 0] = c[..., 0] / b[..., 0]
    dp[..., 0] = d[..., 0] / b[..., 0]
    for j in range(1, n):
        den = b[..., j] - a[..., j] * cp[..., j - 1]
        cp[..., j] = c[..., j] / den
        dp[..., j] = (d[..., j] - a[..., j] * dp[..., j - 1]) / den
    x = np.empty_like(d)
    x[..., n - 1] = dp[..., n - 1]
    for j in range(n - 2, -1, -1):
        x[..., j] = dp[..., j] - cp[..., j] * x[..., j + 1]
    return x
