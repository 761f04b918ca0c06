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


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16: the nearest number with 8 significant bits in FP32's
    exponent range (normal exponents -126..127, subnormal spacing 2^-133),
    ties to the even last bit, one rounding from the input's exact value;
    results past the largest finite value become infinite.  Zeros keep their
    sign; NaN and infinities pass through.  Returns float64."""
    x = np.asarray(x, dtype=np.float64)
    out = x.copy()
    fin = np.isfinite(x) & (x != 0.0)
    ax = np.abs(x[fin])
    _, E = np.frexp(ax)                      # ax = f * 2^E, f in [0.5, 1)
    e = np.maximum(E - 1, -126)              # exponent of the leading bit, clamped
    q = np.ldexp(ax, 7 - e)                  # exact: ax in units of the last kept bit
    y = np.ldexp(np.rint(q), e - 7)          # rint rounds half to even
    y[y >= 2.0 ** 128] = np.inf
    out[fin] = np.copysign(y, x[fin])
    return out


def spmm_rows_from_edges(n: int, src: np.ndarray, dst: np.ndarray, X: np.ndarray,
                         rows: np.ndarray) -> np.ndarray:
    """Rows `rows` (sorted, distinct) of A X, with A the symmetrised,
    deduplicated, loop-free pattern of the edge stream, without building A.
    Each row sums its neighbours' X rows in ascending neighbour order."""
    rows = np.asarray(rows, dtype=np.int64)
    s = np.asarray(src)
    d = np.asarray(dst)
    mark = np.zeros(n, dtype=bool)
    mark[rows] = True
    m1 = mark[s]
    m2 = mark[d]
    u = np.concatenate([s[m1], d[m2]]).astype(np.int64)
    v = np.concatenate([d[m1], s[m2]]).astype(np.int64)
    keep = u != v
    key = np.unique(u[keep] * np.int64(n) + v[keep])
    ru = key // n
    cv = key - ru * n
    Y = np.zeros((rows.shape[0], X.shape[1]))
    np.add.at(Y, np.searchsorted(rows, ru), np.asarray(X, dtype=np.float64)[cv])
    return Y
