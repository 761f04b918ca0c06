"""Pins for the oracle's readings and helpers that no closed-form spectrum
covers (no GPU): the bfloat16 rounding used as the checker of every BF16
test, the restart size, the network's degree feature, and the two block-QR
thresholds (refill and the Cholesky-QR guard).
"""
import math
import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

import fe_synth as S
import oracle as O
from oracle import gnn as G
import importlib
K = importlib.import_module("oracle.krylov_schur")


# ------------------------------------------------------------ bfloat16 RNE
def _bf16_chunk_mismatches(start: int, count: int) -> int:
    import torch
    u = np.arange(start, start + count, dtype=np.uint64).astype(np.uint32)
    f = u.view(np.float32)
    with np.errstate(invalid="ignore"):
        a = O.round_bf16(f)
    b = torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()
    same = (a == b) | (np.isnan(a) & np.isnan(b))
    # signed zeros: a == b treats -0 == +0, so compare the sign bit as well
    # (not for NaN: its sign carries no value, and torch's cast drops it)
    same &= (np.signbit(a) == np.signbit(b)) | np.isnan(a)
    return int((~same).sum())


def test_round_bf16_every_fp32_bit_pattern_matches_torch():
    """All 2^32 FP32 bit patterns against torch's CPU float -> bfloat16 cast
    (round to nearest, ties to even; NaN stays NaN, infinities and signed
    zeros are kept), in chunks over freshly started worker processes (no
    fork of a process whose threads may hold locks)."""
    chunk = 1 << 24
    starts = list(range(0, 1 << 32, chunk))
    workers = max(1, min(8, os.cpu_count() or 1))
    ctx = multiprocessing.get_context("spawn")
    with ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        bad = sum(ex.map(_bf16_chunk_mismatches, starts, [chunk] * len(starts)))
    assert bad == 0


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0),
    (1.0 + 2.0 ** -8, 1.0),                  # tie, kept last bit even (0) -> down
    (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),  # tie, last kept bit odd -> up to even
    (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # just above the tie -> up
    (1.0 + 2.0 ** -8 - 2.0 ** -20, 1.0),     # just below the tie -> down
    (-(1.0 + 3 * 2.0 ** -8), -(1.0 + 2.0 ** -6)),
    (3.4028234663852886e38, math.inf),       # FP32 max rounds past the BF16 max
    (3.3895313892515355e38, 3.3895313892515355e38),  # the BF16 max itself
    (2.0 ** -133, 2.0 ** -133),              # subnormal, exact in BF16
    (1.5 * 2.0 ** -149, 0.0),                # below half the smallest BF16 subnormal
    (1.5 * 2.0 ** -133, 2.0 ** -132),        # subnormal tie -> even
    (1.0 + 2.0 ** -8 + 2.0 ** -30, 1.0 + 2.0 ** -7),  # FP64 input just above a tie: one
                                             # rounding goes up (via FP32 it would tie down)
])
def test_round_bf16_hand_cases(x, want):
    assert O.round_bf16(np.array([x]))[0] == want


def test_round_bf16_specials():
    with np.errstate(invalid="ignore"):
        r = O.round_bf16(np.array([np.nan, np.inf, -np.inf, 0.0, -0.0]))
    assert np.isnan(r[0]) and r[1] == np.inf and r[2] == -np.inf
    assert r[3] == 0.0 and not np.signbit(r[3]) and r[4] == 0.0 and np.signbit(r[4])


# ------------------------------------------------------------ restart size
@pytest.mark.parametrize("m,b,nev,p", [(32, 4, 8, 20), (48, 4, 8, 28), (48, 8, 8, 32), (64, 8, 8, 40)])
def test_restart_keep_reading_values(m, b, nev, p):
    assert O.restart_keep(m, b, nev) == p


def test_restart_keep_invariants():
    for b in (1, 2, 4, 8, 16):
        for m in range(2 * b, 257, b):
            for nev in range(1, m - b + 1):
                p = O.restart_keep(m, b, nev)
                assert (m - p) % b == 0 and nev <= p < m


# ----------------------------------------------------- network degree input
def test_features_first_column_is_log1p_degree():
    # star with 5 leaves plus one isolated vertex: degrees 5, 1 x 5, 0
    n, s, d = S.star_graph(6)
    rp, ci = O.csr_from_edges(n + 1, s, d)
    z = np.arange((n + 1) * 15, dtype=np.float64).reshape(n + 1, 15)
    F = G.features(rp, z)
    assert F.shape == (n + 1, 16)
    assert F[0, 0] == pytest.approx(math.log(6.0), rel=1e-15)
    assert np.allclose(F[1:n, 0], math.log(2.0), rtol=1e-15)
    assert F[n, 0] == 0.0
    assert np.array_equal(F[:, 1:], z)


# ------------------------------------------------------ block QR thresholds
def _pair(ratio: float, n: int = 500, seed: int = 7):
    """Two columns: w0, and w0 plus a perpendicular part `ratio` times its norm."""
    rng = np.random.default_rng(seed)
    w0 = rng.standard_normal(n)
    r = rng.standard_normal(n)
    r -= w0 * (w0 @ r) / (w0 @ w0)
    r *= ratio * np.linalg.norm(w0) / np.linalg.norm(r)
    return np.stack([w0, w0 + r], axis=1)


@pytest.mark.parametrize("ratio", [1e-7, 1e-9, 3e-10])
def test_block_qr_keeps_near_dependent_columns(ratio):
    """Above the refill threshold a column is kept, exactly: Q orthonormal and
    Q R reproduces W to rounding (a refill would lose the ratio-sized part)."""
    W = _pair(ratio)
    nb = np.linalg.norm(W, axis=0)
    Q, R, nref = K._block_qr(np.zeros((W.shape[0], 0)), W.copy(), nb, 1e-10, 1, 1)
    assert nref == 0
    assert np.abs(Q.T @ Q - np.eye(2)).max() < 1e-13
    assert np.abs(Q @ R - W).max() < 1e-14 * np.abs(W).max()


def test_block_qr_refills_below_threshold():
    W = _pair(1e-13)
    nb = np.linalg.norm(W, axis=0)
    Q, R, nref = K._block_qr(np.zeros((W.shape[0], 0)), W.copy(), nb, 1e-10, 1, 1)
    assert nref == 1
    assert np.all(R[1, :] == 0.0)
    assert np.abs(Q.T @ Q - np.eye(2)).max() < 1e-13
    assert np.abs(Q[:, 0] * R[0, 0] - W[:, 0]).max() < 1e-14 * np.abs(W).max()


def test_block_qr_non_finite_column_is_dependent():
    rng = np.random.default_rng(3)
    W = rng.standard_normal((300, 3))
    W[:, 1] = np.nan
    nb = np.sqrt(np.sum(W * W, axis=0))
    Q, R, nref = K._block_qr(np.zeros((300, 0)), W.copy(), nb, 1e-10, 5, 0)
    assert nref == 1 and np.all(np.isfinite(Q)) and np.all(R[1, :] == 0.0)
    assert np.abs(Q.T @ Q - np.eye(3)).max() < 1e-13


@pytest.mark.parametrize("name", ["complete", "bipartite", "hypercube", "star"])
def test_refills_keep_tight_tolerance(name):
    """Closed forms whose Krylov space is exhausted (exact breakdown, refills)
    still meet tol 1e-12 in the explicit residual: a refill at eta = 1e-10
    discards only rounding-level parts."""
    g, lam, nev = {
        "complete": (S.complete_graph(40), np.array([39.0] + [-1.0] * 39), 5),
        "bipartite": (S.complete_bipartite(12, 20), np.array([math.sqrt(240), -math.sqrt(240), 0.0]), 2),
        "hypercube": (S.hypercube(6), np.array([6.0 - 2 * k for k in range(7)]), 5),
        "star": (S.star_graph(60), np.array([math.sqrt(59), -math.sqrt(59)] + [0.0] * 58), 2),
    }[name]
    n, s, d = g
    rp, ci = O.csr_from_edges(n, s, d)
    r = O.krylov_schur(lambda X: O.spmm(rp, ci, X), n, nev, 4, 24, 1e-12,
                       S.normal((n, 4), seed=3))
    assert r.converged and r.refills > 0
    assert r.resid.max() <= 1e-12
    assert all(np.min(np.abs(lam - t)) <= 1e-12 * max(1.0, abs(t)) for t in r.evals)


# ------------------------------------------------- C CSR build, certificate
def test_csr_build_matches_definition():
    n, s, d = S.chung_lu_edges(5000, seed=12)
    s = np.concatenate([s, s[:700], np.arange(60)])  # repeats and self-loops
    d = np.concatenate([d, d[:700], np.arange(60)])
    rp, ci = O.csr_from_edges(n, s, d)
    for threads in (1, 4):
        rp2, ci2 = O.csr_build(n, s, d, threads=threads)
        assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)
    for g in (S.star_graph(300), S.complete_graph(30), S.rmat_edges(12, seed=4)):
        rp, ci = O.csr_from_edges(*g)
        rp2, ci2 = O.csr_build(*g, threads=3)
        assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)


def test_certificate_bounds_hold_on_known_spectra():
    """Path graph P_n (eigenvalues 2 cos(pi k/(n+1)), eigenvectors
    sin(pi j k/(n+1))): perturbed eigenvectors give Rayleigh quotients whose
    true errors lie within both the residual bound and the Kato-Temple bound."""
    n = 400
    g = S.path_graph(n)
    rp, ci = O.csr_from_edges(*g)
    ks = np.array([1, 2, 3, 200])
    j = np.arange(1, n + 1)[:, None]
    lam = 2 * np.cos(np.pi * ks / (n + 1))
    V = np.sin(np.pi * j * ks[None, :] / (n + 1))
    rng = np.random.default_rng(1)
    X = V + 1e-6 * rng.standard_normal(V.shape) * np.linalg.norm(V, axis=0) / np.sqrt(n)
    theta, resid, kt = O.certify(rp, ci, X)
    err = np.abs(theta - lam)   # the top gaps are ~2e-4, well above the residuals
    assert np.all(np.isfinite(kt))
    assert np.all(err <= resid) and np.all(err <= kt) and np.all(kt < resid)
    theta0, resid0, _ = O.certify(rp, ci, V)   # exact eigenvectors
    assert np.allclose(theta0, lam, atol=1e-13) and resid0.max() < 1e-13


# --------------------------------------------------- directed graphs, SVD
def _dense_directed(n, rp, ci):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = 1.0
    return A


def test_csr_directed_definition_and_transpose():
    n, s, d = S.rmat_edges(9, seed=5)
    rp, ci = O.csr_directed(n, s, d)
    rpt, cit = O.csr_directed(n, d, s)
    A = _dense_directed(n, rp, ci)
    assert np.array_equal(A.T, _dense_directed(n, rpt, cit))
    assert np.all(np.diag(A) == 0)
    want = np.zeros((n, n))
    keep = s != d
    want[s[keep], d[keep]] = 1.0
    assert np.array_equal(A, want)
    assert not np.array_equal(A, A.T)  # R-MAT arcs are directed


@pytest.mark.parametrize("seed", [1, 2])
def test_svds_matches_dense_svd(seed):
    """Directed R-MAT, n = 512: the oracle's A^T A Krylov-Schur against
    numpy's dense SVD (LAPACK, an independent routine)."""
    n, s, d = S.rmat_edges(9, seed=seed)
    rp, ci = O.csr_directed(n, s, d)
    rpt, cit = O.csr_directed(n, d, s)
    sig, V, r = O.svds(rp, ci, rpt, cit, n, 6, 4, 32, 1e-12, S.normal((n, 4), seed=3))
    assert r.converged
    want = np.linalg.svd(_dense_directed(n, rp, ci), compute_uv=False)[:6]
    assert np.allclose(sig, want, rtol=1e-10)
    A = _dense_directed(n, rp, ci)
    assert np.allclose(A.T @ (A @ V), V * sig ** 2, atol=1e-8 * sig[0] ** 2)


def test_svds_closed_forms():
    # out-star: one row with p ones -> sigma_1 = sqrt(p); complete bipartite
    # arcs K_{p -> q} -> sigma_1 = sqrt(p q); the rest 0
    p = 40
    src = np.zeros(p, dtype=np.int32)
    dst = np.arange(1, p + 1, dtype=np.int32)
    n = p + 1
    rp, ci = O.csr_directed(n, src, dst)
    rpt, cit = O.csr_directed(n, dst, src)
    sig, _, r = O.svds(rp, ci, rpt, cit, n, 1, 4, 16, 1e-12, S.normal((n, 4), seed=1))
    assert abs(sig[0] - np.sqrt(p)) < 1e-12
    P, Q = 7, 9
    src = np.repeat(np.arange(P), Q).astype(np.int32)
    dst = (P + np.tile(np.arange(Q), P)).astype(np.int32)
    n = P + Q
    rp, ci = O.csr_directed(n, src, dst)
    rpt, cit = O.csr_directed(n, dst, src)
    sig, _, r = O.svds(rp, ci, rpt, cit, n, 1, 2, 8, 1e-12, S.normal((n, 2), seed=2))
    assert abs(sig[0] - np.sqrt(P * Q)) < 1e-12
