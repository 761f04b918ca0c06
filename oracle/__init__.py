"""CPU oracle for the block Krylov-Schur hot path.

TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import anything here.  The GPU library shares no code
with this package (no kernels, headers, helpers or constants), and this package
never imports the GPU library.

Everything is plain FP64: a C loop for the sparse product and the dense
Jacobi check (``oracle.c``), numpy for the rest.  Each function cites the
passage of the paper it follows.  Where the paper is silent the documented
reading is implemented (the list of readings is kept with the design notes).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, brute force or invariants, except the learned-start
network's training quality, which has nothing to pin it (parity unpinned).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc into liboracle.so (OpenMP used only to split rows)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                               os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        L.oracle_spmm.argtypes = [ctypes.c_int64, P, P, P, ctypes.c_int32, P, ctypes.c_int32]
        L.oracle_spmm.restype = None
        L.oracle_jacobi.argtypes = [ctypes.c_int32, P, P, ctypes.c_double, ctypes.c_int32]
        L.oracle_jacobi.restype = ctypes.c_int32
        L.oracle_csr_build.argtypes = [ctypes.c_int64, ctypes.c_int64, P, P, P, P, ctypes.c_int32]
        L.oracle_csr_build.restype = ctypes.c_int64
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int32
        _lib = L
    return _lib


def ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


from .csr import csr_from_edges, csr_build, csr_directed, degrees  # noqa: E402
from .ops import (spmm, gram, block_update, col_norms, max_threads, round_bf16,  # noqa: E402
                  spmm_rows_from_edges)
from .dense_eig import jacobi_eigh  # noqa: E402
from .rng import philox4x32_10, refill_column  # noqa: E402
from .krylov_schur import krylov_schur, KSResult, restart_keep, ritz_scale, EPS23  # noqa: E402
from .certify import certify  # noqa: E402
from .svd import svds  # noqa: E402
