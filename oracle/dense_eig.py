"""Dense symmetric eigendecomposition by cyclic Jacobi (brute-force spectra check).

Golub & Van Loan's cyclic-by-row Jacobi method, run in C (``oracle.c``).  Used
only to check spectra of small graphs (n <= 512) independently of the
Krylov-Schur iteration.
"""
from __future__ import annotations

import numpy as np

from . import lib, ptr


def jacobi_eigh(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 100):
    """Eigenvalues (ascending) and eigenvectors (columns) of symmetric A."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    n = A.shape[0]
    assert A.shape == (n, n)
    V = np.empty((n, n), dtype=np.float64)
    sweeps = lib().oracle_jacobi(n, ptr(A), ptr(V), tol, max_sweeps)
    w = np.diag(A).copy()
    order = np.argsort(w, kind="stable")
    return w[order], V[:, order], int(sweeps)
