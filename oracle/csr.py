"""Graph -> pattern-only CSR (the sparse matrix format section).

The paper stores a graph's adjacency as a sparse matrix with no value array;
for an undirected graph the matrix is symmetric.  The oracle's CSR is the
plain definition: row i lists the distinct neighbours j != i of vertex i in
ascending order, ``row_ptr`` (int64, n+1 entries) holds the row offsets and
``col_idx`` (int32) the column indices.  A sample stream is symmetrised (each
pair (u, v) contributes (u, v) and (v, u)), self-loops are dropped and repeats
are merged.
"""
from __future__ import annotations

import numpy as np


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray):
    s = np.concatenate([np.asarray(src, dtype=np.int64), np.asarray(dst, dtype=np.int64)])
    d = np.concatenate([np.asarray(dst, dtype=np.int64), np.asarray(src, dtype=np.int64)])
    keep = s != d
    key = np.unique(s[keep] * np.int64(n) + d[keep])  # sorted by (row, col), repeats merged
    rows = key // n
    cols = (key - rows * n).astype(np.int32)
    deg = np.bincount(rows, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    return row_ptr, cols


def degrees(row_ptr: np.ndarray) -> np.ndarray:
    return np.diff(row_ptr)
