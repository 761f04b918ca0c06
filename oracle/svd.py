"""Largest singular values of a directed graph's pattern matrix (oracle).

The paper computes the SVD of its directed billion-node page graph with the
same block Krylov-Schur eigensolver (its scalability section), which needs
products with A and with A^T.  Here the singular values of A are read as
the square roots of the largest eigenvalues of the symmetric positive
semidefinite A^T A, computed by the oracle's Krylov-Schur with the operator
X -> A^T (A X) (two pattern products, FP64): sigma_i = sqrt(lambda_i), the
right singular vectors are the eigenvectors.  (Reading: A^T A rather than a
Golub-Kahan bidiagonalisation; for the largest singular values squaring the
condition number costs nothing.)
"""
from __future__ import annotations

import numpy as np

from .krylov_schur import krylov_schur
from .ops import spmm


def svds(rp, ci, rpt, cit, n: int, nsv: int, b: int, m: int, tol: float, X0: np.ndarray,
         threads: int = 1, **kw):
    """(A, A^T) as two CSRs.  Returns (sigma, V, result) with sigma descending,
    V the right singular vectors (n x nsv) and the Krylov-Schur result of
    A^T A (its evals are sigma^2)."""
    def op(X):
        return spmm(rpt, cit, spmm(rp, ci, X, threads=threads), threads=threads)
    r = krylov_schur(op, n, nsv, b, m, tol, X0, **kw)
    sigma = np.sqrt(np.maximum(r.evals, 0.0))
    return sigma, r.evecs, r
