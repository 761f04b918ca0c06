"""Pins for the CPU oracle (no GPU).

The paper prints no worked numerical example, so the oracle is pinned by
closed-form spectra, brute force on tiny inputs, library routines on special
cases (numpy/scipy, used here only as independent checks) and invariants.
The planted-mistake tests at the end show that plausible slips in the oracle
are caught by these pins.
"""
import numpy as np
import pytest

import fe_synth as S
import oracle as O


def csr(g):
    n, s, d = g
    rp, ci = O.csr_from_edges(n, s, d)
    return n, rp, ci


def dense(n, rp, ci):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, ci[rp[i]:rp[i + 1]]] = 1.0
    return A


# ---------------------------------------------------------------- Philox
KAT = [  # Random123 known-answer vectors for philox4x32-10
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
]


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_kat_inputs_module(ctr, key, out):
    assert tuple(int(x) for x in S.philox4x32_10(ctr, key)) == out


@pytest.mark.parametrize("ctr,key,out", KAT)
def test_philox_kat_oracle(ctr, key, out):
    r = O.philox4x32_10(*[np.array([c]) for c in ctr], key[0], key[1])
    assert tuple(int(x[0]) for x in r) == out


def test_refill_draws_range_and_exactness():
    r = O.refill_column(10000, 3, 7, 12345)
    assert r.min() >= -1.0 and r.max() < 1.0
    assert np.array_equal(r.astype(np.float32).astype(np.float64), r)  # exact in FP32
    assert abs(r.mean()) < 0.05


# ------------------------------------------------------------------- CSR
CLOSED_NNZ = [
    (S.complete_graph(17), 17 * 16),
    (S.cycle_graph(23), 46),
    (S.star_graph(31), 60),
    (S.path_graph(19), 36),
    (S.complete_bipartite(4, 9), 72),
    (S.hypercube(6), 6 * 64),
]


@pytest.mark.parametrize("g,nnz", CLOSED_NNZ)
def test_csr_closed_form_nnz(g, nnz):
    n, rp, ci = csr(g)
    assert rp[-1] == nnz and rp[0] == 0 and rp.dtype == np.int64 and ci.dtype == np.int32


def test_csr_invariants_and_dedupe():
    n, s, d = S.chung_lu_edges(3000, seed=5)
    s = np.concatenate([s, s[:500], np.arange(50)])  # repeats and self-loops
    d = np.concatenate([d, d[:500], np.arange(50)])
    n, rp, ci = n, *O.csr_from_edges(n, s, d)
    A = dense(n, rp, ci)
    assert np.array_equal(A, A.T)
    assert np.all(np.diag(A) == 0)
    for i in range(n):
        row = ci[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)
    # the same pattern from scipy's independent COO->CSR path
    import scipy.sparse as sp
    keep = s != d
    M = sp.coo_matrix((np.ones(keep.sum()), (s[keep], d[keep])), shape=(n, n))
    M = ((M + M.T) > 0).astype(np.float64).tocsr()
    M.sort_indices()
    assert np.array_equal(M.indptr, rp) and np.array_equal(M.indices, ci)


# ------------------------------------------------------------------ SpMM
def test_spmm_ones_gives_degree():
    n, rp, ci = csr(S.chung_lu_edges(5000, seed=2))
    y = O.spmm(rp, ci, np.ones((n, 3)))
    assert np.array_equal(y, np.repeat(np.diff(rp)[:, None].astype(float), 3, axis=1))


def test_spmm_closed_forms():
    X = S.normal((29, 4), seed=3)
    n, rp, ci = csr(S.complete_graph(29))
    assert np.allclose(O.spmm(rp, ci, X), X.sum(0) - X, atol=1e-12)
    n, rp, ci = csr(S.cycle_graph(29))
    assert np.allclose(O.spmm(rp, ci, X), np.roll(X, 1, 0) + np.roll(X, -1, 0), atol=1e-12)
    n, rp, ci = csr(S.star_graph(29))
    Y = O.spmm(rp, ci, X)
    assert np.allclose(Y[0], X[1:].sum(0)) and np.allclose(Y[1:], np.repeat(X[:1], 28, 0))


def test_spmm_brute_force_integer_exact():
    n, rp, ci = csr(S.chung_lu_edges(400, alpha=2.3, mean_deg=10, seed=4))
    X = S.small_ints((n, 5), seed=9)
    Y = O.spmm(rp, ci, X)
    A = dense(n, rp, ci)
    ref = np.array([[sum(int(A[i, j]) * int(X[j, c]) for j in range(n)) for c in range(5)]
                    for i in range(0, n, 37)])
    assert np.array_equal(Y[::37], ref)


def test_spmm_rows_from_edges_brute_force():
    """Sampled rows straight from an edge stream (with repeats and self-loops)
    equal rows of the dense brute-force A X."""
    n, s, d = S.chung_lu_edges(300, alpha=2.1, mean_deg=12, seed=5)
    A = np.zeros((n, n))
    for u, v in zip(s.tolist(), d.tolist()):
        if u != v:
            A[u, v] = A[v, u] = 1.0
    X = S.small_ints((n, 5), seed=6)
    rows = np.array([0, 1, 7, 150, 298, 299])
    got = O.spmm_rows_from_edges(n, s, d, X, rows)
    assert np.array_equal(got, (A @ X)[rows])
    hub = int(np.argmax(A.sum(1)))
    assert np.array_equal(O.spmm_rows_from_edges(n, s, d, X, np.array([hub])), (A @ X)[[hub]])


def test_spmm_linearity_symmetry_threads():
    n, rp, ci = csr(S.rmat_edges(12, seed=7))
    X, Z = S.normal((n, 3), seed=1), S.normal((n, 3), seed=2)
    AX, AZ = O.spmm(rp, ci, X), O.spmm(rp, ci, Z)
    assert np.allclose(O.spmm(rp, ci, 2 * X - Z), 2 * AX - AZ, atol=1e-9)
    assert np.allclose(X.T @ AZ, AX.T @ Z, rtol=1e-10, atol=1e-8)
    assert np.array_equal(O.spmm(rp, ci, X, threads=8), AX)
    empty = np.diff(rp) == 0
    assert empty.any() and np.all(AX[empty] == 0)


# ---------------------------------------------------------- Gram / update
def test_gram_update_integer_brute_force():
    V = S.small_ints((7, 6), seed=1)
    W = S.small_ints((7, 3), seed=2)
    C = S.small_ints((6, 3), seed=3)
    G = O.gram(V, W, alpha=2.0)
    for p in range(6):
        for q in range(3):
            assert G[p, q] == 2 * sum(int(V[r, p]) * int(W[r, q]) for r in range(7))
    U = O.block_update(W, V, C, alpha=-1.0, beta=3.0)
    for r in range(7):
        for q in range(3):
            assert U[r, q] == 3 * int(W[r, q]) - sum(int(V[r, p]) * int(C[p, q]) for p in range(6))


# ---------------------------------------------------------------- Jacobi
def spectrum(name):
    if name == "K":
        n = 12
        return S.complete_graph(n), np.array([n - 1] + [-1] * (n - 1), float)
    if name == "C":
        n = 15
        return S.cycle_graph(n), 2 * np.cos(2 * np.pi * np.arange(n) / n)
    if name == "P":
        n = 14
        return S.path_graph(n), 2 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1))
    if name == "star":
        n = 13
        return S.star_graph(n), np.array([np.sqrt(n - 1), -np.sqrt(n - 1)] + [0.0] * (n - 2))
    if name == "Kpq":
        p, q = 4, 6
        return S.complete_bipartite(p, q), np.array([np.sqrt(p * q), -np.sqrt(p * q)] + [0.0] * (p + q - 2))
    if name == "Q":
        from math import comb
        d = 5
        return S.hypercube(d), np.array(sum(([d - 2 * k] * comb(d, k) for k in range(d + 1)), []), float)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["K", "C", "P", "star", "Kpq", "Q"])
def test_jacobi_closed_forms(name):
    g, lam = spectrum(name)
    n, rp, ci = csr(g)
    w, V, sweeps = O.jacobi_eigh(dense(n, rp, ci))
    assert np.allclose(w, np.sort(lam), atol=1e-12)
    assert np.allclose(V.T @ V, np.eye(n), atol=1e-12)


def test_jacobi_random_matches_lapack():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((60, 60))
    a = a + a.T
    w, V, _ = O.jacobi_eigh(a)
    assert np.allclose(w, np.linalg.eigvalsh(a), atol=1e-11)
    assert np.allclose(a @ V, V * w, atol=1e-10)


# ---------------------------------------------------------- Krylov-Schur
def ks(n, rp, ci, nev, b, m, tol=1e-10, seed=3, **kw):
    return O.krylov_schur(lambda X: O.spmm(rp, ci, X), n, nev, b, m, tol,
                          S.normal((n, b), seed=seed), **kw)


def top_by_magnitude(lam, k):
    lam = np.asarray(lam)
    order = np.lexsort((-lam, -np.abs(lam)))
    return lam[order][:k]


@pytest.mark.parametrize("name,nev", [("C", 6), ("P", 6), ("Q", 6), ("K", 5), ("star", 2)])
def test_ks_closed_forms(name, nev):
    g, lam = spectrum(name)
    if name in ("C", "P"):  # bigger instances of the same families
        n = 48
        g = S.cycle_graph(n) if name == "C" else S.path_graph(n)
        lam = (2 * np.cos(2 * np.pi * np.arange(n) / n) if name == "C"
               else 2 * np.cos(np.pi * np.arange(1, n + 1) / (n + 1)))
    if name == "K":
        g, lam = S.complete_graph(40), np.array([39.0] + [-1.0] * 39)
    if name == "star":
        g, lam = S.star_graph(60), np.array([np.sqrt(59), -np.sqrt(59)] + [0.0] * 58)
    if name == "Q":
        from math import comb
        g = S.hypercube(7)
        lam = np.array(sum(([7 - 2 * k] * comb(7, k) for k in range(8)), []), float)
    n, rp, ci = csr(g)
    r = ks(n, rp, ci, nev, 4, 24)
    assert r.converged
    # magnitudes are fixed; with repeated eigenvalues (beyond what b start
    # vectors can separate) the signs among equal magnitudes may differ, so
    # check every value lies in the spectrum
    want = np.sort(np.abs(top_by_magnitude(lam, nev)))
    assert np.allclose(np.sort(np.abs(r.evals)), want, atol=1e-8)
    assert all(np.min(np.abs(lam - t)) < 1e-8 for t in r.evals)
    assert r.resid.max() < 1e-8


def test_ks_vs_jacobi_random_graphs():
    for seed in (11, 12, 13):
        n, rp, ci = csr(S.chung_lu_edges(300, alpha=2.2, mean_deg=8, seed=seed))
        w, _, _ = O.jacobi_eigh(dense(n, rp, ci))
        r = ks(n, rp, ci, 8, 4, 32, tol=1e-12)
        assert r.converged
        assert np.allclose(np.sort(r.evals), np.sort(top_by_magnitude(w, 8)), rtol=1e-10, atol=1e-10)


def test_ks_permutation_invariance():
    n, s, d = S.rmat_edges(10, seed=3)
    rp, ci = O.csr_from_edges(n, s, d)
    p = S.permutation(n, 99)
    rp2, ci2 = O.csr_from_edges(n, p[s], p[d])
    a = ks(n, rp, ci, 8, 4, 32, tol=1e-11)
    b = ks(n, rp2, ci2, 8, 4, 32, tol=1e-11)
    assert np.allclose(a.evals, b.evals, rtol=1e-9)


@pytest.mark.slow
def test_ks_tiny_config_vs_scipy():
    """The smallest workload (Chung-Lu n=65,536, alpha=2.1, mean 16; nev=8,
    block 4, m=32, tol 1e-8) against scipy's ARPACK (independent check)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sl
    n, rp, ci = csr(S.chung_lu_edges(65536, alpha=2.1, mean_deg=16, seed=1))
    r = ks(n, rp, ci, 8, 4, 32, tol=1e-8, seed=3)
    assert r.converged and r.resid.max() < 1e-7
    A = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    w = sl.eigsh(A, k=8, which="LM", tol=1e-13, return_eigenvectors=False)
    assert np.allclose(np.sort(r.evals), np.sort(w), rtol=1e-8)


# --------------------------------------------------- planted mistakes
def _closed_form_pins_pass():
    try:
        test_ks_closed_forms("C", 6)
        test_ks_closed_forms("K", 5)
        test_ks_vs_jacobi_random_graphs()
        return True
    except AssertionError:
        return False


@pytest.mark.parametrize("mutation", ["sign", "transpose", "bad_refill", "ascending"])
def test_planted_mistakes_are_caught(monkeypatch, mutation):
    import importlib
    K = importlib.import_module("oracle.krylov_schur")
    if mutation == "sign":  # projection added instead of subtracted
        def cgs2_wrong_sign(Vk, W):
            C1 = Vk.T @ W
            W += Vk @ C1
            C2 = Vk.T @ W
            W -= Vk @ C2
            return C1 + C2
        monkeypatch.setattr(K, "_cgs2", cgs2_wrong_sign)
    elif mutation == "transpose":  # Cholesky factor used untransposed
        monkeypatch.setattr(K, "_chol_upper", lambda G: np.linalg.cholesky(G))
    elif mutation == "bad_refill":  # refill without orthogonalising
        def refill_not_orthogonal(Vk, W, nb, eta, seed, step, eta_chol=1e-6):
            Q, R, acc, dep, _ = K._columnwise(W, nb, eta)
            if not dep:
                return K._block_qr.__wrapped__(Vk, W, nb, eta, seed, step, eta_chol)
            for j in dep:
                Q[:, j] = 1.0 / np.sqrt(W.shape[0])
            return Q, R, len(dep)
        orig = K._block_qr
        refill_not_orthogonal.__wrapped__ = orig
        K._block_qr.__wrapped__ = orig
        monkeypatch.setattr(K, "_block_qr", refill_not_orthogonal)
    elif mutation == "ascending":  # smallest instead of largest magnitude
        monkeypatch.setattr(K, "_ritz_order", lambda th: np.argsort(np.abs(th)))
    assert not _closed_form_pins_pass()
