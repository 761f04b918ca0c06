"""fe_svds (largest singular values of a directed pattern matrix through
Krylov-Schur on A^T A, two products per step) against the FP64 oracle.

Bars: FP64 storage, same start block: singular values within 1e-10 relative
of the oracle's A^T A Krylov-Schur and the same number of operator
applications; against numpy's dense SVD at n = 2048 within 1e-10; FP32
storage (tol 1e-6) within 1e-8 of the oracle; closed forms exact to 1e-12;
right singular vectors checked with the oracle's products.
"""
import numpy as np
import pytest
import torch

import fe_synth as S
import oracle as O
from bars import resid_bar

pytestmark = pytest.mark.gpu

DIRECTED = 0x2 | 0x4  # FE_DEDUPE | FE_DROP_SELF: arcs kept as given


def handles(fe, n, s, d):
    A = fe.fe_csr_build(n, s, d, DIRECTED)
    At = fe.fe_csr_build(n, d, s, DIRECTED)
    rp, ci = O.csr_directed(n, s, d)
    rpt, cit = O.csr_directed(n, d, s)
    return A, At, rp, ci, rpt, cit


def oracle_residual(rp, ci, rpt, cit, V, sig):
    """||A^T A v - sigma^2 v|| / (sigma^2 ||v||) per column (oracle products)."""
    W = O.spmm(rpt, cit, O.spmm(rp, ci, V, threads=8), threads=8) - V * sig ** 2
    return np.linalg.norm(W, axis=0) / (sig ** 2 * np.linalg.norm(V, axis=0))


@pytest.mark.parametrize("b,m", [(2, 16), (4, 32)])
def test_svds_fp64_matches_oracle(fe, b, m):
    n, s, d = S.rmat_edges(13, seed=31)
    A, At, rp, ci, rpt, cit = handles(fe, n, s, d)
    X0 = S.normal((n, b), seed=4)
    sig_o, _, ref = O.svds(rp, ci, rpt, cit, n, 8, b, m, 1e-10, X0, threads=8)
    r = fe.fe_svds(A, At, 8, b, m, 1e-10, dtype=torch.float64, start=torch.tensor(X0, device="cuda"))
    assert r.status == fe.FE_OK and ref.converged
    assert np.allclose(r.evals, sig_o, rtol=1e-10, atol=0)
    assert r.spmm_calls == ref.spmm_calls
    V = r.evecs.cpu().numpy()
    assert np.all(oracle_residual(rp, ci, rpt, cit, V, r.evals) <= 1e-9)


def test_svds_against_dense_svd(fe):
    n, s, d = S.rmat_edges(11, seed=7)
    A, At, rp, ci, rpt, cit = handles(fe, n, s, d)
    r = fe.fe_svds(A, At, 8, 4, 32, 1e-12, dtype=torch.float64, seed=3, want_vectors=False)
    assert r.status == fe.FE_OK
    D = np.zeros((n, n))
    for i in range(n):
        D[i, ci[rp[i]:rp[i + 1]]] = 1.0
    want = np.linalg.svd(D, compute_uv=False)[:8]
    assert np.allclose(r.evals, want, rtol=1e-10)


def test_svds_fp32_storage(fe):
    n, s, d = S.rmat_edges(15, seed=15)
    A, At, rp, ci, rpt, cit = handles(fe, n, s, d)
    X0 = S.normal((n, 4), seed=5)
    sig_o, _, ref = O.svds(rp, ci, rpt, cit, n, 8, 4, 48, 1e-12, X0, threads=8)
    r = fe.fe_svds(A, At, 8, 4, 48, 1e-6, dtype=torch.float32,
                   start=torch.tensor(X0, dtype=torch.float32, device="cuda"))
    assert r.status == fe.FE_OK and ref.converged
    assert np.all(np.abs(r.evals - sig_o) <= 1e-8 * sig_o)
    assert np.all(r.resid <= resid_bar(1e-6, sig_o ** 2, torch.float32))
    V = r.evecs.double().cpu().numpy()
    # FP32 rounding of v adds up to 2^-23 sigma_1^2 to ||A^T A v - sigma^2 v||
    slack = 2.0 ** -23 * sig_o[0] ** 2 / sig_o ** 2
    assert np.all(oracle_residual(rp, ci, rpt, cit, V, r.evals) <= 1e-6 + slack)


def test_svds_closed_forms(fe):
    p = 300  # out-star: sigma_1 = sqrt(p)
    src = np.zeros(p, dtype=np.int32)
    dst = np.arange(1, p + 1, dtype=np.int32)
    A, At, *_ = handles(fe, p + 1, src, dst)
    r = fe.fe_svds(A, At, 1, 4, 16, 1e-12, dtype=torch.float64, seed=1)
    assert r.status == fe.FE_OK and abs(r.evals[0] - np.sqrt(p)) < 1e-12 * np.sqrt(p)
    P, Q = 40, 70  # all arcs P -> Q: sigma_1 = sqrt(P Q)
    src = np.repeat(np.arange(P), Q).astype(np.int32)
    dst = (P + np.tile(np.arange(Q), P)).astype(np.int32)
    A, At, *_ = handles(fe, P + Q, src, dst)
    r = fe.fe_svds(A, At, 1, 2, 16, 1e-12, dtype=torch.float64, seed=2)
    assert r.status == fe.FE_OK and abs(r.evals[0] - np.sqrt(P * Q)) < 1e-12 * np.sqrt(P * Q)


def test_svds_rejects(fe):
    n, s, d = S.rmat_edges(10, seed=1)
    A = fe.fe_csr_build(n, s, d, DIRECTED)
    Ar = fe.fe_csr_build(n, d, s, DIRECTED | fe.FE_RELABEL_BY_DEGREE)
    with pytest.raises(fe.FeError) as e:
        fe.fe_svds(A, Ar, 4, 4, 32, 1e-8)
    assert e.value.status == fe.FE_EINVAL
    n2, s2, d2 = S.rmat_edges(11, seed=1)
    B = fe.fe_csr_build(n2, d2, s2, DIRECTED)
    with pytest.raises(fe.FeError) as e:
        fe.fe_svds(A, B, 4, 4, 32, 1e-8)
    assert e.value.status == fe.FE_EINVAL
