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


def csr_build(n: int, src: np.ndarray, dst: np.ndarray, threads: int = 1):
    """The same CSR as csr_from_edges, built by the C loop (counting, per-row
    sort and merge), for graphs too large for a global sort of the pairs."""
    from . import lib, ptr
    s = np.ascontiguousarray(src, dtype=np.int32)
    d = np.ascontiguousarray(dst, dtype=np.int32)
    assert s.shape == d.shape
    if s.size and (min(s.min(), d.min()) < 0 or max(s.max(), d.max()) >= n):
        raise ValueError("vertex id out of range")
    row_ptr = np.empty(n + 1, dtype=np.int64)
    col = np.empty(max(2 * s.size, 1), dtype=np.int32)
    nnz = lib().oracle_csr_build(n, s.size, ptr(s), ptr(d), ptr(row_ptr), ptr(col), threads)
    if nnz < 0:
        raise MemoryError("oracle_csr_build: allocation failed")
    return row_ptr, col[:nnz]


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


def csr_directed(n: int, src: np.ndarray, dst: np.ndarray):
    """Pattern CSR of a directed graph: row u lists the distinct v != u with
    an arc (u, v), ascending (no symmetrising).  The transpose is
    csr_directed(n, dst, src)."""
    s = np.asarray(src, dtype=np.int64)
    d = np.asarray(dst, dtype=np.int64)
    keep = s != d
    key = np.unique(s[keep] * np.int64(n) + d[keep])
    rows = key // n
    cols = (key - rows * n).astype(np.int32)
    deg = np.bincount(rows, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    return row_ptr, cols


def degrees(row_ptr: np.ndarray) -> np.ndarray:
    return np.diff(row_ptr)
