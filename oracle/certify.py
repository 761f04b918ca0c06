"""A-posteriori certificate of computed eigenpairs of the symmetric pattern
matrix (the residual of the eigen-iteration's convergence test, taken
explicitly), for graphs too large for the oracle's own solve.

For a unit vector x, theta = x^T A x and r = A x - theta x, symmetric A has
an eigenvalue within ||r|| of theta.  If moreover the interval
(theta - delta, theta + delta) holds only one eigenvalue lambda, the
Kato-Temple inequality bounds |theta - lambda| <= ||r||^2 / delta.  Here delta
is taken from the other computed values: the distance to the nearest other
theta_j minus that pair's own residual (a reading: it assumes no eigenvalue
outside the computed set lies between them, which the certificate cannot
check).
"""
from __future__ import annotations

import numpy as np

from .ops import spmm


def certify(row_ptr: np.ndarray, col_idx: np.ndarray, X: np.ndarray, threads: int = 1):
    """X: (n, k) candidate eigenvectors (any scaling).  Returns the Rayleigh
    quotients theta, the residual norms ||A x - theta x|| / ||x||, and the
    Kato-Temple bounds (inf where the gap is not positive)."""
    X = np.asarray(X, dtype=np.float64)
    AX = spmm(row_ptr, col_idx, X, threads=threads)
    xx = np.sum(X * X, axis=0)
    theta = np.sum(X * AX, axis=0) / xx
    R = AX - X * theta
    resid = np.sqrt(np.sum(R * R, axis=0) / xx)
    k = theta.shape[0]
    kt = np.full(k, np.inf)
    for i in range(k):
        others = [abs(theta[i] - theta[j]) - resid[j] for j in range(k) if j != i]
        delta = min(others) if others else np.inf
        if delta > resid[i]:
            kt[i] = resid[i] ** 2 / delta
    return theta, resid, kt
