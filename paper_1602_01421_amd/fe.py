"""Thin ctypes binding of libfe.so (names follow the C ABI in include/fe.h).

Only argument marshalling happens here: every step of the sparse product,
the Gram/update kernels and the Krylov-Schur iteration runs in the HIP
library.  PyTorch supplies device memory (tensors) and streams.  If the
library is not built, every entry point raises FeError.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfe.so")

FE_OK, FE_EINVAL, FE_ENOMEM, FE_EDEVICE, FE_ENOCONV, FE_EBREAKDOWN, FE_EUNSUPPORTED = range(7)
FE_F64, FE_F32, FE_BF16 = 0, 1, 2
FE_SYMMETRIZE, FE_DEDUPE, FE_DROP_SELF, FE_RELABEL_BY_DEGREE = 0x1, 0x2, 0x4, 0x8
FE_GRAPH_DEFAULT = FE_SYMMETRIZE | FE_DEDUPE | FE_DROP_SELF

EXPORTED = ("fe_last_error", "fe_version", "fe_csr_build", "fe_csr_from_csr", "fe_csr_info",
            "fe_csr_perm", "fe_csr_export", "fe_csr_free", "fe_spmm", "fe_spmm_gather_bound",
            "fe_spmm_gather_bound_sets", "fe_gather_rows", "fe_gram", "fe_gram_noalloc",
            "fe_block_update", "fe_block_update_gram", "fe_krylov_schur", "fe_ks_workspace_bytes",
            "fe_svds",
            "fe_dense_symeig", "fe_gnn_param_count",
            "fe_gnn_create", "fe_gnn_free", "fe_gnn_get_params", "fe_gnn_set_params",
            "fe_gnn_forward", "fe_gnn_backward", "fe_gnn_adam")


class FeError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fe status {status}: {msg}")
        self.status = status


class KsOpts(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_int32), ("which", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("start", ctypes.c_void_p), ("hip_stream", ctypes.c_void_p),
                ("eta", ctypes.c_double), ("profile", ctypes.c_int32),
                ("verbose", ctypes.c_int32), ("mixed", ctypes.c_int32),
                ("mixed_switch", ctypes.c_double), ("start_check", ctypes.c_int32),
                ("start_drop", ctypes.c_double), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_uint64), ("keep", ctypes.c_int32)]


class KsReport(ctypes.Structure):
    _fields_ = [("restarts", ctypes.c_int32), ("spmm_calls", ctypes.c_int32),
                ("spmm_cols", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("refills", ctypes.c_int32), ("gram_calls", ctypes.c_int32),
                ("update_calls", ctypes.c_int32), ("switch_restart", ctypes.c_int32),
                ("spmm_calls_low", ctypes.c_int32),
                ("rho", ctypes.c_double * 64), ("ritz", ctypes.c_double * 64),
                ("resid", ctypes.c_double * 64),
                ("t_spmm", ctypes.c_double), ("t_gram", ctypes.c_double),
                ("t_update", ctypes.c_double), ("t_other_dev", ctypes.c_double),
                ("bytes_spmm", ctypes.c_double), ("bytes_gram", ctypes.c_double),
                ("bytes_update", ctypes.c_double),
                ("t_host", ctypes.c_double), ("t_total", ctypes.c_double),
                ("start_fallback", ctypes.c_int32), ("device_allocs", ctypes.c_int32)]


_lib = None


def lib():
    """Load libfe.so (raises FeError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FeError(FE_EDEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, u32, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_uint32, ctypes.c_double)
        L.fe_last_error.restype = ctypes.c_char_p
        L.fe_version.restype = i32
        sig = {
            "fe_csr_build": [i64, i64, P, P, u32, ctypes.POINTER(P)],
            "fe_csr_from_csr": [i64, P, P, u32, ctypes.POINTER(P)],
            "fe_csr_info": [P, P, P, P],
            "fe_csr_perm": [P, P],
            "fe_csr_export": [P, P, P],
            "fe_spmm": [P, P, P, i32, i32, P],
            "fe_spmm_gather_bound": [P, P, P, i32, i32, P],
            "fe_gather_rows": [P, i64, P, i64, i32, i32, P, P],
            "fe_gram": [P, i32, i64, P, i64, i32, i32, f64, P, P],
            "fe_gram_noalloc": [P, i32, i64, P, i64, i32, i32, f64, P, P],
            "fe_block_update": [P, i64, i32, P, i32, i64, P, f64, f64, i32, P],
            "fe_block_update_gram": [P, i64, i32, P, i32, i64, P, P, i32, P],
            "fe_krylov_schur": [P, i32, i32, i32, f64, ctypes.POINTER(KsOpts), P, P,
                                ctypes.POINTER(KsReport)],
            "fe_dense_symeig": [i32, P, P, P],
            "fe_ks_workspace_bytes": [P, i32, i32, i32, ctypes.POINTER(KsOpts),
                                      ctypes.POINTER(ctypes.c_uint64)],
            "fe_svds": [P, P, i32, i32, i32, f64, ctypes.POINTER(KsOpts), P, P,
                        ctypes.POINTER(KsReport)],
            "fe_gnn_create": [ctypes.c_uint64, i32, ctypes.POINTER(P)],
            "fe_gnn_get_params": [P, P],
            "fe_gnn_set_params": [P, P],
            "fe_gnn_forward": [P, P, P, P, i32, P],
            "fe_gnn_backward": [P, P, P, P, ctypes.POINTER(ctypes.c_double), P, P],
            "fe_gnn_adam": [P, f64, f64, P],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.fe_csr_free.argtypes = [P]
        L.fe_csr_free.restype = None
        L.fe_gnn_free.argtypes = [P]
        L.fe_gnn_free.restype = None
        L.fe_gnn_param_count.argtypes = []
        L.fe_gnn_param_count.restype = i64
        L.fe_spmm_gather_bound_sets.argtypes = []
        L.fe_spmm_gather_bound_sets.restype = i32
        _lib = L
    return _lib


def _check(st: int, allow=()):
    if st != FE_OK and st not in allow:
        raise FeError(st, lib().fe_last_error().decode())
    return st


def _np_ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def _dt_of(t) -> int:
    import torch
    m = {torch.float64: FE_F64, torch.float32: FE_F32, torch.bfloat16: FE_BF16}
    if t.dtype not in m:
        raise FeError(FE_EINVAL, f"unsupported dtype {t.dtype}")
    return m[t.dtype]


def torch_dtype(dt: int):
    import torch
    return {FE_F64: torch.float64, FE_F32: torch.float32, FE_BF16: torch.bfloat16}[dt]


def _dev_ptr(t):
    if not t.is_cuda:
        raise FeError(FE_EINVAL, "tensor must live on the GPU")
    if not t.is_contiguous():
        raise FeError(FE_EINVAL, "tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


def version() -> int:
    return int(lib().fe_version())


class Csr:
    """Owning wrapper of an fe_csr handle."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        n, nnz, md = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().fe_csr_info(self._h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(md)))
        self.n, self.nnz, self.max_deg = n.value, nnz.value, md.value

    @property
    def handle(self):
        return self._h

    def perm(self) -> np.ndarray:
        p = np.empty(self.n, dtype=np.int32)
        _check(lib().fe_csr_perm(self._h, _np_ptr(p)))
        return p

    def export(self):
        rp = np.empty(self.n + 1, dtype=np.int64)
        ci = np.empty(max(self.nnz, 1), dtype=np.int32)
        _check(lib().fe_csr_export(self._h, _np_ptr(rp), _np_ptr(ci)))
        return rp, ci[: self.nnz]

    def close(self):
        if self._h:
            lib().fe_csr_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fe_csr_build(n: int, src: np.ndarray, dst: np.ndarray, flags: int = FE_GRAPH_DEFAULT) -> Csr:
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    if src.shape != dst.shape:
        raise FeError(FE_EINVAL, "src/dst length mismatch")
    h = ctypes.c_void_p()
    _check(lib().fe_csr_build(n, src.shape[0], _np_ptr(src), _np_ptr(dst), flags, ctypes.byref(h)))
    return Csr(h)


def fe_csr_from_csr(n: int, row_ptr: np.ndarray, col_idx: np.ndarray, flags: int = 0) -> Csr:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().fe_csr_from_csr(n, _np_ptr(rp), _np_ptr(ci), flags, ctypes.byref(h)))
    return Csr(h)


def fe_spmm(A: Csr, X, Y=None, stream=None):
    """Y = A X for a device tensor X of shape (n, b); returns Y."""
    import torch
    if X.dim() != 2 or X.shape[0] != A.n:
        raise FeError(FE_EINVAL, f"X must be ({A.n}, b)")
    if Y is None:
        Y = torch.empty_like(X)
    _check(lib().fe_spmm(A.handle, _dev_ptr(X), _dev_ptr(Y), X.shape[1], _dt_of(X), _stream(stream)))
    return Y


def fe_spmm_gather_bound(A: Csr, X, out=None, stream=None):
    """The product's gathers without its rows (its memory ceiling on A): X (n, b)
    device tensor; out: FP64 device buffer of fe_spmm_gather_bound_sets()
    workgroup sums (allocated if None); returns out."""
    import torch
    if X.dim() != 2 or X.shape[0] != A.n:
        raise FeError(FE_EINVAL, f"X must be ({A.n}, b)")
    sets = lib().fe_spmm_gather_bound_sets()
    if out is None:
        out = torch.empty(sets, dtype=torch.float64, device=X.device)
    if out.dtype != torch.float64 or out.numel() < sets:
        raise FeError(FE_EINVAL, f"out must hold {sets} float64")
    _check(lib().fe_spmm_gather_bound(A.handle, _dev_ptr(X), _dev_ptr(out), X.shape[1], _dt_of(X),
                                      _stream(stream)))
    return out


def fe_gather_rows(idx, X, out=None, stream=None):
    """The product's gathers over an index stream: X row idx[e] for every e, in
    order (idx: 1-D int32 device tensor; X: (n, b) device tensor); out as for
    fe_spmm_gather_bound; returns out."""
    import torch
    if X.dim() != 2 or idx.dim() != 1 or idx.dtype != torch.int32:
        raise FeError(FE_EINVAL, "idx must be 1-D int32 and X (n, b)")
    sets = lib().fe_spmm_gather_bound_sets()
    if out is None:
        out = torch.empty(sets, dtype=torch.float64, device=X.device)
    if out.dtype != torch.float64 or out.numel() < sets:
        raise FeError(FE_EINVAL, f"out must hold {sets} float64")
    _check(lib().fe_gather_rows(_dev_ptr(idx), idx.numel(), _dev_ptr(X), X.shape[0], X.shape[1],
                                _dt_of(X), _dev_ptr(out), _stream(stream)))
    return out


def fe_gram(V, W, alpha: float = 1.0, C=None, stream=None):
    """C = alpha V^T W.  V: (nblk, n, b) device tensor (packed blocks), W: (n, b)."""
    import torch
    nblk, n, b = V.shape
    if W.shape != (n, b) or W.dtype != V.dtype:
        raise FeError(FE_EINVAL, "W must be (n, b) with V's dtype")
    if C is None:
        C = torch.empty((nblk * b, b), dtype=torch.float64, device=V.device)
    _check(lib().fe_gram(_dev_ptr(V), nblk, n * b, _dev_ptr(W), n, b, _dt_of(V), alpha,
                         _dev_ptr(C), _stream(stream)))
    return C


def fe_gram_noalloc(V, W, C, alpha: float = 1.0, stream=None):
    """C = alpha V^T W into the caller's C ((nblk*b, b) FP64), with the
    library's static partials array: the C call allocates nothing."""
    import torch
    nblk, n, b = V.shape
    if W.shape != (n, b) or W.dtype != V.dtype:
        raise FeError(FE_EINVAL, "W must be (n, b) with V's dtype")
    if C.shape != (nblk * b, b) or C.dtype != torch.float64:
        raise FeError(FE_EINVAL, "C must be (nblk*b, b) float64")
    _check(lib().fe_gram_noalloc(_dev_ptr(V), nblk, n * b, _dev_ptr(W), n, b, _dt_of(V), alpha,
                                 _dev_ptr(C), _stream(stream)))
    return C


def fe_block_update_gram(W, V, C, Cout=None, stream=None):
    """W <- W - V C, then Cout = [V W]^T W ((k+b, b) FP64) in one pass over V."""
    import torch
    n, b = W.shape
    nblk = V.shape[0]
    if V.dim() != 3 or V.shape[1:] != (n, b) or V.dtype != W.dtype:
        raise FeError(FE_EINVAL, "V must be (nblk, n, b) with W's dtype")
    if C.shape != (nblk * b, b) or C.dtype != torch.float64:
        raise FeError(FE_EINVAL, "C must be (k, b) float64")
    if Cout is None:
        Cout = torch.empty((nblk * b + b, b), dtype=torch.float64, device=W.device)
    _check(lib().fe_block_update_gram(_dev_ptr(W), n, b, _dev_ptr(V), nblk, n * b, _dev_ptr(C),
                                      _dev_ptr(Cout), _dt_of(W), _stream(stream)))
    return Cout


def fe_block_update(W, V, C, alpha: float = 1.0, beta: float = 1.0, stream=None):
    """W <- beta W + alpha V C.  V: (nblk, n, b) (or W itself for in-place), C: (k, b) FP64."""
    n, b = W.shape
    if V.dim() == 2:
        nblk = 1
    else:
        nblk = V.shape[0]
        if V.shape[1:] != (n, b):
            raise FeError(FE_EINVAL, "V blocks must be (n, b)")
    if C.shape != (nblk * b, b) or C.dtype != __import__("torch").float64:
        raise FeError(FE_EINVAL, "C must be (k, b) float64")
    _check(lib().fe_block_update(_dev_ptr(W), n, b, _dev_ptr(V), nblk, n * b, _dev_ptr(C), alpha,
                                 beta, _dt_of(W), _stream(stream)))
    return W


@dataclass
class KsResult:
    evals: np.ndarray
    evecs: object
    status: int
    restarts: int
    spmm_calls: int
    spmm_cols: int
    converged: int
    refills: int
    gram_calls: int
    update_calls: int
    switch_restart: int
    spmm_calls_low: int
    rho: np.ndarray
    ritz: np.ndarray
    resid: np.ndarray
    t_spmm: float
    t_gram: float
    t_update: float
    t_other_dev: float
    bytes_spmm: float
    bytes_gram: float
    bytes_update: float
    t_host: float
    t_total: float
    start_fallback: int = -1
    device_allocs: int = 0


def _ks_opts(dtype, mixed, start):
    import torch
    if dtype is None:
        dtype = torch.float64
    o = KsOpts()
    o.dt = {torch.float64: FE_F64, torch.float32: FE_F32, torch.bfloat16: FE_BF16}[dtype]
    o.mixed = int(mixed)
    if start is not None:
        o.start = _dev_ptr(start).value
    return o, dtype


def fe_ks_workspace_bytes(A: Csr, nev: int, block: int, m: int, dtype=None, mixed: bool = False,
                          start=None) -> int:
    """Device bytes fe_krylov_schur needs for these arguments (its workspace)."""
    o, _ = _ks_opts(dtype, mixed, start)
    out = ctypes.c_uint64()
    _check(lib().fe_ks_workspace_bytes(A.handle, nev, block, m, ctypes.byref(o), ctypes.byref(out)))
    return out.value


def fe_krylov_schur(A: Csr, nev: int, block: int, m: int, tol: float, dtype=None, start=None,
                    seed: int = 0, max_restarts: int = 0, eta: float = 0.0, stream=None,
                    want_vectors: bool = True, profile: bool = False,
                    verbose: bool = False, mixed: bool = False,
                    mixed_switch: float = 0.0, start_check: int = 0,
                    start_drop: float = 0.0, workspace=None, keep: int = 0) -> KsResult:
    """Block Krylov-Schur for the nev largest-magnitude eigenpairs (see fe.h).
    workspace: optional device tensor of at least fe_ks_workspace_bytes bytes."""
    import torch
    if dtype is None:
        dtype = torch.float64
    dt = {torch.float64: FE_F64, torch.float32: FE_F32, torch.bfloat16: FE_BF16}[dtype]
    o = KsOpts()
    o.dt = dt
    o.which = 0
    o.max_restarts = max_restarts
    o.seed = seed
    o.eta = eta
    o.profile = int(profile)
    o.verbose = int(verbose)
    o.mixed = int(mixed)
    o.mixed_switch = mixed_switch
    o.start_check = start_check
    o.start_drop = start_drop
    o.keep = keep
    o.hip_stream = _stream(stream).value
    if start is not None:
        if start.shape != (A.n, block) or start.dtype != dtype:
            raise FeError(FE_EINVAL, "start must be (n, block) in the solve dtype")
        o.start = _dev_ptr(start).value
    if workspace is not None:
        o.workspace = _dev_ptr(workspace).value
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    evals = np.zeros(nev, dtype=np.float64)
    evecs = torch.empty((A.n, nev), dtype=dtype, device="cuda") if want_vectors else None
    rep = KsReport()
    st = lib().fe_krylov_schur(A.handle, nev, block, m, tol, ctypes.byref(o), _np_ptr(evals),
                               _dev_ptr(evecs) if evecs is not None else None, ctypes.byref(rep))
    _check(st, allow=(FE_ENOCONV,))
    return KsResult(evals=evals, evecs=evecs, status=st, restarts=rep.restarts,
                    spmm_calls=rep.spmm_calls, spmm_cols=rep.spmm_cols,
                    converged=rep.converged, refills=rep.refills, gram_calls=rep.gram_calls,
                    update_calls=rep.update_calls, switch_restart=rep.switch_restart,
                    spmm_calls_low=rep.spmm_calls_low, rho=np.array(rep.rho[:nev]),
                    ritz=np.array(rep.ritz[:nev]),
                    resid=np.array(rep.resid[:nev]), t_spmm=rep.t_spmm, t_gram=rep.t_gram,
                    t_update=rep.t_update, t_other_dev=rep.t_other_dev,
                    bytes_spmm=rep.bytes_spmm, bytes_gram=rep.bytes_gram,
                    bytes_update=rep.bytes_update, t_host=rep.t_host,
                    t_total=rep.t_total, start_fallback=rep.start_fallback,
                    device_allocs=rep.device_allocs)


def fe_svds(A: Csr, At: Csr, nsv: int, block: int, m: int, tol: float, dtype=None, start=None,
            seed: int = 0, max_restarts: int = 0, stream=None, want_vectors: bool = True,
            profile: bool = False) -> KsResult:
    """Largest singular values of a pattern matrix from handles of A and A^T
    (see fe.h).  Returns a KsResult whose evals are the singular values
    (descending) and whose evecs are the right singular vectors."""
    import torch
    if dtype is None:
        dtype = torch.float64
    o = KsOpts()
    o.dt = {torch.float64: FE_F64, torch.float32: FE_F32, torch.bfloat16: FE_BF16}[dtype]
    o.seed = seed
    o.max_restarts = max_restarts
    o.profile = int(profile)
    o.hip_stream = _stream(stream).value
    if start is not None:
        if start.shape != (A.n, block) or start.dtype != dtype:
            raise FeError(FE_EINVAL, "start must be (n, block) in the solve dtype")
        o.start = _dev_ptr(start).value
    sv = np.zeros(nsv, dtype=np.float64)
    vecs = torch.empty((A.n, nsv), dtype=dtype, device="cuda") if want_vectors else None
    rep = KsReport()
    st = lib().fe_svds(A.handle, At.handle, nsv, block, m, tol, ctypes.byref(o), _np_ptr(sv),
                       _dev_ptr(vecs) if vecs is not None else None, ctypes.byref(rep))
    _check(st, allow=(FE_ENOCONV,))
    return KsResult(evals=sv, evecs=vecs, status=st, restarts=rep.restarts,
                    spmm_calls=rep.spmm_calls, spmm_cols=rep.spmm_cols,
                    converged=rep.converged, refills=rep.refills, gram_calls=rep.gram_calls,
                    update_calls=rep.update_calls, switch_restart=rep.switch_restart,
                    spmm_calls_low=rep.spmm_calls_low, rho=np.array(rep.rho[:nsv]),
                    ritz=np.array(rep.ritz[:nsv]), resid=np.array(rep.resid[:nsv]),
                    t_spmm=rep.t_spmm, t_gram=rep.t_gram, t_update=rep.t_update,
                    t_other_dev=rep.t_other_dev, bytes_spmm=rep.bytes_spmm,
                    bytes_gram=rep.bytes_gram, bytes_update=rep.bytes_update, t_host=rep.t_host,
                    t_total=rep.t_total, start_fallback=rep.start_fallback,
                    device_allocs=rep.device_allocs)


def fe_dense_symeig(a: np.ndarray):
    """Host eigendecomposition of a small symmetric matrix: (w, z), unordered."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    n = a.shape[0]
    w = np.empty(n)
    z = np.empty((n, n))
    _check(lib().fe_dense_symeig(n, _np_ptr(a), _np_ptr(w), _np_ptr(z)))
    return w, z


# ------------------------------------------------------------ learned start
GNN_SHAPES = [("W0", (16, 64)), ("U0", (16, 64)), ("b0", (64,)),
              ("W1", (64, 64)), ("U1", (64, 64)), ("b1", (64,)),
              ("W2", (64, 64)), ("U2", (64, 64)), ("b2", (64,)), ("P", (64, 8))]


def gnn_unflatten(flat: np.ndarray) -> dict:
    out, at = {}, 0
    for name, shp in GNN_SHAPES:
        size = int(np.prod(shp))
        out[name] = np.asarray(flat[at:at + size], dtype=np.float64).reshape(shp)
        at += size
    return out


def gnn_flatten(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float32).ravel()
                           for name, _ in GNN_SHAPES])


class Gnn:
    """Owning wrapper of an fe_gnn (learned start-block network)."""

    def __init__(self, seed: int = 0, compute: str = "bf16"):
        h = ctypes.c_void_p()
        dt = {"bf16": FE_BF16, "f32": FE_F32}[compute]
        _check(lib().fe_gnn_create(seed, dt, ctypes.byref(h)))
        self._h = h
        self.count = int(lib().fe_gnn_param_count())

    def get_params(self) -> np.ndarray:
        out = np.empty(self.count, dtype=np.float32)
        _check(lib().fe_gnn_get_params(self._h, _np_ptr(out)))
        return out

    def set_params(self, flat: np.ndarray):
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        assert flat.shape == (self.count,)
        _check(lib().fe_gnn_set_params(self._h, _np_ptr(flat)))

    def forward(self, A: Csr, z, X=None, block: int = 8, stream=None):
        """Start block X (n x block, original vertex order) for random features z
        (n x 15, FP32 device); block < 8 folds the 8 outputs (column c sums
        outputs c, c + block, ...)."""
        import torch
        if X is None:
            X = torch.empty((A.n, block), dtype=torch.float32, device="cuda")
        _check(lib().fe_gnn_forward(self._h, A.handle, _dev_ptr(z), _dev_ptr(X), block,
                                    _stream(stream)))
        return X

    def backward(self, A: Csr, z, V, want_grads: bool = False, stream=None):
        """Forward + loss + backward; returns (loss, grads or None)."""
        loss = ctypes.c_double()
        g = np.empty(self.count, dtype=np.float32) if want_grads else None
        _check(lib().fe_gnn_backward(self._h, A.handle, _dev_ptr(z), _dev_ptr(V),
                                     ctypes.byref(loss), _np_ptr(g) if g is not None else None,
                                     _stream(stream)))
        return loss.value, g

    def adam(self, lr: float = 1e-3, clip: float = 0.0, stream=None):
        """One Adam step; clip > 0 scales the gradients to global norm <= clip first."""
        _check(lib().fe_gnn_adam(self._h, lr, clip, _stream(stream)))

    def close(self):
        if self._h:
            lib().fe_gnn_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
