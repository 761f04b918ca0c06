"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

Only input generation lives here (edge streams of synthetic graphs, dense
random blocks).  Nothing in this module computes any step of the eigensolver:
no CSR construction, no products, no orthogonalisation.  All randomness is
Philox4x32-10 (Salmon et al., SC 2011) keyed by a 64-bit seed, so every value
is a pure function of (seed, index).

The paper measures on real graphs (its evaluation section, the graph table)
that are not available here; the families below stand in for them:
R-MAT (the paper's own synthetic graphs are R-MAT), Chung-Lu with Pareto
expected degrees, and a stochastic block model; plus closed-form graphs whose
spectra are known exactly.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libfesynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c with gcc (OpenMP) into libfesynth.so next to it."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                               os.path.join(_HERE, "gen.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i64, i32, u64, u32, f64 = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_double)
        lib.synth_philox4x32_10.argtypes = [P, P, P]
        lib.synth_permutation.argtypes = [i64, u64, P]
        lib.synth_rmat.argtypes = [i32, i64, f64, f64, f64, u64, P, P, P]
        lib.synth_chung_lu_weights.argtypes = [i64, f64, f64, u64, P]
        lib.synth_chung_lu.argtypes = [i64, i64, P, u64, P, P]
        lib.synth_sbm.argtypes = [i64, i32, f64, i64, u64, P, P]
        lib.synth_normal.argtypes = [i64, u64, u32, P]
        lib.synth_small_int.argtypes = [i64, u64, u32, i32, i32, P]
        for f in (lib.synth_philox4x32_10, lib.synth_permutation, lib.synth_rmat,
                  lib.synth_chung_lu_weights, lib.synth_chung_lu, lib.synth_sbm,
                  lib.synth_normal, lib.synth_small_int):
            f.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _L().synth_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def permutation(n: int, seed: int) -> np.ndarray:
    perm = np.empty(n, dtype=np.int32)
    _L().synth_permutation(n, seed, _p(perm))
    return perm


def rmat_edges(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
               c: float = 0.19, seed: int = 1, relabel: bool = True):
    """Raw R-MAT sample stream: (src, dst) int32 arrays of edge_factor * 2^scale edges.

    With relabel=True both ends pass through a seeded random permutation of the
    2^scale vertices (seed + 1), which removes R-MAT's id/degree correlation.
    """
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    perm = permutation(n, seed + 1) if relabel else None
    _L().synth_rmat(scale, m, a, b, c, seed, _p(perm), _p(src), _p(dst))
    return n, src, dst


def chung_lu_edges(n: int, alpha: float = 2.1, mean_deg: float = 16.0, seed: int = 1):
    """Chung-Lu sample stream with Pareto(alpha) expected degrees scaled to mean_deg.

    round(n * mean_deg / 2) endpoint pairs; self-loops and repeats are left in.
    """
    w = np.empty(n, dtype=np.float64)
    _L().synth_chung_lu_weights(n, alpha, mean_deg, seed, _p(w))
    m = int(round(n * mean_deg / 2.0))
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _L().synth_chung_lu(n, m, _p(w), seed, _p(src), _p(dst))
    return n, src, dst


def sbm_edges(n: int, blocks: int, rho: float, mean_deg: float, seed: int = 1):
    """Stochastic block model sample stream (equal blocks, in-block fraction rho)."""
    m = int(round(n * mean_deg / 2.0))
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _L().synth_sbm(n, blocks, rho, m, seed, _p(src), _p(dst))
    return n, src, dst


def normal(shape, seed: int, stream: int = 0) -> np.ndarray:
    """N(0,1) float64 array (Box-Muller over Philox draws)."""
    count = int(np.prod(shape))
    out = np.empty(count, dtype=np.float64)
    _L().synth_normal(count, seed, stream, _p(out))
    return out.reshape(shape)


def small_ints(shape, seed: int, stream: int = 0, lo: int = -8, hi: int = 8) -> np.ndarray:
    """Integers uniform in [lo, hi] as float64 (sums stay exact in every dtype)."""
    count = int(np.prod(shape))
    out = np.empty(count, dtype=np.float64)
    _L().synth_small_int(count, seed, stream, lo, hi, _p(out))
    return out.reshape(shape)


# ---------------------------------------------------------------- closed forms

def _pairs(src, dst, n):
    return n, np.asarray(src, dtype=np.int32), np.asarray(dst, dtype=np.int32)


def complete_graph(n: int):
    i, j = np.triu_indices(n, 1)
    return _pairs(i, j, n)


def cycle_graph(n: int):
    i = np.arange(n)
    return _pairs(i, (i + 1) % n, n)


def path_graph(n: int):
    i = np.arange(n - 1)
    return _pairs(i, i + 1, n)


def star_graph(n: int):
    """Centre 0 joined to leaves 1..n-1."""
    return _pairs(np.zeros(n - 1, dtype=np.int64), np.arange(1, n), n)


def complete_bipartite(p: int, q: int):
    i, j = np.meshgrid(np.arange(p), p + np.arange(q), indexing="ij")
    return _pairs(i.ravel(), j.ravel(), p + q)


def hypercube(d: int):
    n = 1 << d
    v = np.arange(n)
    src, dst = [], []
    for bit in range(d):
        u = v ^ (1 << bit)
        keep = v < u
        src.append(v[keep])
        dst.append(u[keep])
    return _pairs(np.concatenate(src), np.concatenate(dst), n)


# ----------------------------------------------------- learned-start graph set

def learned_start_graph(seed: int, min_log2n: int = 14, max_log2n: int = 18):
    """One graph of the learned-start training/evaluation family.

    With equal odds: Chung-Lu with Pareto exponent alpha ~ U[2.0, 2.8], or a
    stochastic block model with k ~ U{4..16} equal blocks and in-block
    fraction rho ~ U[0.6, 0.9]; n = 2^U{min_log2n..max_log2n}; target mean
    degree ~ U[8, 32].  The recipe is drawn from numpy's PCG64 seeded with
    `seed`; the edges from Philox with the same seed.  Returns
    (n, src, dst, description).
    """
    rng = np.random.default_rng(seed)
    kind = "chung_lu" if rng.random() < 0.5 else "sbm"
    n = 1 << int(rng.integers(min_log2n, max_log2n + 1))
    mean = float(rng.uniform(8.0, 32.0))
    if kind == "chung_lu":
        alpha = float(rng.uniform(2.0, 2.8))
        n, s, d = chung_lu_edges(n, alpha=alpha, mean_deg=mean, seed=seed)
        desc = f"chung_lu n={n} alpha={alpha:.2f} mean={mean:.1f}"
    else:
        k = int(rng.integers(4, 17))
        rho = float(rng.uniform(0.6, 0.9))
        n, s, d = sbm_edges(n, k, rho, mean, seed=seed)
        desc = f"sbm n={n} k={k} rho={rho:.2f} mean={mean:.1f}"
    return n, s, d, desc


def learned_start_features(n: int, seed: int) -> np.ndarray:
    """The network's per-vertex random inputs: (n, 15) N(0,1) draws (stream 7)."""
    return normal((n, 15), seed=seed, stream=7)
