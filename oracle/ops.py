"""Sparse and dense subspace operations, FP64.

- ``spmm``: Y = A X for the 0/1 pattern matrix (the sparse matrix
  multiplication section: every nonzero (i, j) adds row j of X to row i of Y).
- ``gram``: C = alpha * V^T W, the MvTransMv operation of the table of dense
  operations the eigensolver needs.
- ``block_update``: W <- beta * W + alpha * V C, the MvTimesMatAddMv operation
  of the same table.
- ``col_norms``: the MvNorm operation.

X, Y, V, W are (n, cols) float64 arrays; the library matmul is used as a step.
"""
from __future__ import annotations

import numpy as np

from . import lib, ptr


def spmm(row_ptr: np.ndarray, col_idx: np.ndarray, X: np.ndarray, threads: int = 1) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float64)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    n, b = X.shape
    assert row_ptr.shape[0] == n + 1
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    Y = np.empty((n, b), dtype=np.float64)
    lib().oracle_spmm(n, ptr(rp), ptr(ci), ptr(X), b, ptr(Y), threads)
    return Y[:, 0] if squeeze else Y


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def gram(V: np.ndarray, W: np.ndarray, alpha: float = 1.0) -> np.ndarray:
    return alpha * (V.T @ W)


def block_update(W: np.ndarray, V: np.ndarray, C: np.ndarray, alpha: float = 1.0,
                 beta: float = 1.0) -> np.ndarray:
    return beta * W + alpha * (V @ C)


def col_norms(X: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum(X * X, axis=0))
