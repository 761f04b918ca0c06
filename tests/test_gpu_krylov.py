"""fe_krylov_schur on the GPU against the FP64 oracle and closed-form spectra.

Bars: FP64 storage: eigenvalues within 1e-10 relative of the oracle's (same
start block, same refill draws) and the same number of sparse products;
FP32 storage (tol 1e-6): eigenvalues within 1e-8 relative of the FP64
oracle, explicit FP64 residuals <= 1e-6; every returned vector satisfies
||A x - theta x|| / |theta| <= the reported residual (checked on the CPU).
"""
import numpy as np
import pytest
import torch

import fe_synth as S
import oracle as O
from bars import resid_bar

pytestmark = pytest.mark.gpu


def setup(fe, g, relabel=True):
    n, s, d = g
    flags = fe.FE_GRAPH_DEFAULT | (fe.FE_RELABEL_BY_DEGREE if relabel else 0)
    A = fe.fe_csr_build(n, s, d, flags)
    rp, ci = O.csr_from_edges(n, s, d)
    return A, rp, ci


def oracle_ks(rp, ci, n, nev, b, m, tol, X0, **kw):
    return O.krylov_schur(lambda X: O.spmm(rp, ci, X, threads=8), n, nev, b, m, tol, X0, **kw)


def check_vectors(rp, ci, r, slack=10.0):
    X = r.evecs.double().cpu().numpy()
    AX = O.spmm(rp, ci, X)
    res = np.linalg.norm(AX - X * r.evals, axis=0) / (O.ritz_scale(r.evals) * np.linalg.norm(X, axis=0))
    assert np.all(res <= slack * r.resid + 1e-6 * (r.evecs.dtype != torch.float64) + 1e-13)


def test_tiny_config_fp64_matches_oracle(fe):
    """Chung-Lu n=65,536, Pareto 2.1, mean 16; nev=8, block 4, m=32, tol 1e-8, FP64."""
    g = S.chung_lu_edges(65536, alpha=2.1, mean_deg=16, seed=1)
    A, rp, ci = setup(fe, g)
    n = A.n
    X0 = S.normal((n, 4), seed=3)
    ref = oracle_ks(rp, ci, n, 8, 4, 32, 1e-8, X0)
    r = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float64,
                           start=torch.tensor(X0, device="cuda"))
    assert r.status == fe.FE_OK and ref.converged
    assert np.allclose(r.evals, ref.evals, rtol=1e-10, atol=0)
    assert r.spmm_calls == ref.spmm_calls and r.restarts == ref.restarts
    assert r.resid.max() <= 1e-7
    check_vectors(rp, ci, r)
    # eigenvector subspaces: largest principal angle between the GPU's and the
    # oracle's 8-dimensional bases (|lambda_8| = 84.5 is well apart from
    # |lambda_9| = 78.5, so the subspace is determined to ~ resid / gap)
    Q1, _ = np.linalg.qr(r.evecs.cpu().numpy())
    Q2, _ = np.linalg.qr(ref.evecs)
    cos = np.linalg.svd(Q1.T @ Q2, compute_uv=False)
    assert np.sqrt(max(0.0, 1.0 - cos.min() ** 2)) <= 1e-6


CLOSED = {
    "complete40": (S.complete_graph(40), np.array([39.0] + [-1.0] * 39), 5, 4, 24),
    "cycle48": (S.cycle_graph(48), 2 * np.cos(2 * np.pi * np.arange(48) / 48), 6, 4, 24),
    "path48": (S.path_graph(48), 2 * np.cos(np.pi * np.arange(1, 49) / 49), 6, 4, 24),
    "star40k": (S.star_graph(40000), np.array([np.sqrt(39999), -np.sqrt(39999)]), 2, 4, 24),
}


@pytest.mark.parametrize("name", list(CLOSED))
@pytest.mark.parametrize("relabel", [False, True])
def test_closed_forms_fp64(fe, name, relabel):
    g, lam, nev, b, m = CLOSED[name]
    A, rp, ci = setup(fe, g, relabel)
    X0 = S.normal((A.n, b), seed=3)
    r = fe.fe_krylov_schur(A, nev, b, m, 1e-10, dtype=torch.float64,
                           start=torch.tensor(X0, device="cuda"))
    assert r.status == fe.FE_OK
    order = np.lexsort((-lam, -np.abs(lam)))
    want = np.sort(np.abs(lam[order][:nev]))
    assert np.allclose(np.sort(np.abs(r.evals)), want, atol=1e-9)
    assert all(np.min(np.abs(lam - t)) < 1e-9 for t in r.evals)
    ref = oracle_ks(rp, ci, A.n, nev, b, m, 1e-10, X0)
    assert r.refills == ref.refills
    check_vectors(rp, ci, r)


def test_hypercube_fp64(fe):
    from math import comb
    g = S.hypercube(8)
    lam = np.array(sum(([8 - 2 * k] * comb(8, k) for k in range(9)), []), float)
    A, rp, ci = setup(fe, g)
    r = fe.fe_krylov_schur(A, 6, 4, 32, 1e-10, dtype=torch.float64, seed=11)
    assert r.status == fe.FE_OK
    assert all(np.min(np.abs(lam - t)) < 1e-9 for t in r.evals)
    assert np.allclose(sorted(np.abs(r.evals)), [6, 6, 6, 6, 8, 8], atol=1e-9)


@pytest.mark.parametrize("relabel", [False, True])
def test_rmat_fp32_vs_fp64_oracle(fe, relabel):
    g = S.rmat_edges(14, seed=14)
    A, rp, ci = setup(fe, g, relabel)
    n = A.n
    X0 = S.normal((n, 4), seed=3)
    ref = oracle_ks(rp, ci, n, 8, 4, 48, 1e-12, X0)
    r = fe.fe_krylov_schur(A, 8, 4, 48, 1e-6, dtype=torch.float32,
                           start=torch.tensor(X0, dtype=torch.float32, device="cuda"))
    assert r.status == fe.FE_OK
    assert np.all(np.abs(r.evals - ref.evals) <= 1e-8 * np.abs(ref.evals))
    assert np.all(r.resid <= resid_bar(1e-6, r.evals, torch.float32))
    check_vectors(rp, ci, r)


def test_rmat_bf16_storage(fe):
    g = S.rmat_edges(13, seed=13)
    A, rp, ci = setup(fe, g)
    ref = oracle_ks(rp, ci, A.n, 8, 8, 64, 1e-12, S.normal((A.n, 8), seed=3))
    r = fe.fe_krylov_schur(A, 8, 8, 64, 1e-2, dtype=torch.bfloat16, seed=5, max_restarts=200)
    assert r.status in (fe.FE_OK, fe.FE_ENOCONV)
    assert np.all(np.abs(r.evals - ref.evals) <= 1e-3 * np.abs(ref.evals)), (
        r.status, r.restarts, r.evals, ref.evals, r.rho)


def test_random_start_deterministic(fe):
    g = S.chung_lu_edges(20000, alpha=2.3, mean_deg=12, seed=9)
    A, rp, ci = setup(fe, g)
    r1 = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float32, seed=77)
    r2 = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float32, seed=77)
    assert np.array_equal(r1.evals, r2.evals) and r1.spmm_calls == r2.spmm_calls


def test_no_convergence_and_bad_args(fe):
    g = S.rmat_edges(12, seed=1)
    A, rp, ci = setup(fe, g)
    r = fe.fe_krylov_schur(A, 8, 4, 32, 1e-14, dtype=torch.float32, seed=1, max_restarts=1)
    assert r.status == fe.FE_ENOCONV and r.restarts == 1 and np.all(np.isfinite(r.evals))
    for args in [(8, 4, 30), (30, 4, 32), (8, 3, 33)]:
        with pytest.raises(fe.FeError) as e:
            fe.fe_krylov_schur(A, *args, 1e-8)
        assert e.value.status in (fe.FE_EINVAL, fe.FE_EUNSUPPORTED)


def test_mixed_precision_bf16_to_fp32(fe):
    """Storage starts in BF16, then the solve restarts in FP32 from the folded
    wanted Ritz vectors; it still reaches tol 1e-6 and the FP64-oracle
    eigenvalues."""
    g = S.rmat_edges(14, seed=14)
    A, rp, ci = setup(fe, g)
    ref = oracle_ks(rp, ci, A.n, 8, 8, 64, 1e-12, S.normal((A.n, 8), seed=3))
    r = fe.fe_krylov_schur(A, 8, 8, 64, 1e-6, dtype=torch.float32, seed=3, mixed=True)
    assert r.status == fe.FE_OK
    assert r.switch_restart >= 0 and 0 < r.spmm_calls_low < r.spmm_calls
    assert np.all(np.abs(r.evals - ref.evals) <= 1e-8 * np.abs(ref.evals))
    assert np.all(r.resid <= resid_bar(1e-6, r.evals, torch.float32))
    assert r.evecs.dtype == torch.float32
    check_vectors(rp, ci, r)


def test_rmat22_full_size_fp32(fe):
    """R-MAT scale 22 (the benchmark graph), FP32 storage, nev 8, block 4,
    m 48, tol 1e-6, against the oracle's own FP64 eigenvalues of the same
    graph (tol 1e-10, a committed fixture written by
    tests/golden/make_golden.py): within 1e-8 relative.  The FP32
    eigenvectors' residuals are recomputed with the oracle's FP64 product
    over all rows."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "rmat22_evals.json")) as f:
        ref = json.load(f)
    lam = np.array(ref["evals"])
    n, s, d = S.rmat_edges(22, seed=22)
    A = fe.fe_csr_build(n, s, d, fe.FE_GRAPH_DEFAULT | fe.FE_RELABEL_BY_DEGREE)
    assert A.nnz == ref["nnz"]
    r32 = fe.fe_krylov_schur(A, 8, 4, 48, 1e-6, dtype=torch.float32, seed=1)
    assert r32.status == fe.FE_OK
    assert np.all(np.abs(r32.evals - lam) <= 1e-8 * np.abs(lam))
    assert np.all(r32.resid <= resid_bar(1e-6, r32.evals, torch.float32))
    rp, ci = O.csr_build(n, s, d, threads=16)
    X = r32.evecs.double().cpu().numpy()
    R = O.spmm(rp, ci, X, threads=16) - X * r32.evals
    res = np.linalg.norm(R, axis=0) / np.linalg.norm(X, axis=0)
    # the returned vectors are the FP64 Ritz vectors rounded to FP32, which adds
    # up to 2^-24 (||A|| + |theta|) <= 2^-23 |lambda_1| to each residual
    rounding = 2.0 ** -23 * np.abs(lam).max()
    assert np.all(res <= 1e-6 * np.abs(r32.evals) + rounding)


@pytest.mark.parametrize("m", [96, 112])
def test_subspace_beyond_64_fp32(fe, m):
    """m > 64 (the restart reads all m basis columns of each row; p = 56, 64):
    FP32 storage against the FP64 oracle run with the same shape."""
    g = S.rmat_edges(14, seed=14)
    A, rp, ci = setup(fe, g)
    X0 = S.normal((A.n, 8), seed=3)
    ref = oracle_ks(rp, ci, A.n, 8, 8, m, 1e-12, X0)
    r = fe.fe_krylov_schur(A, 8, 8, m, 1e-6, dtype=torch.float32,
                           start=torch.tensor(X0, dtype=torch.float32, device="cuda"))
    assert r.status == fe.FE_OK
    assert np.all(np.abs(r.evals - ref.evals) <= 1e-8 * np.abs(ref.evals))
    assert np.all(r.resid <= resid_bar(1e-6, r.evals, torch.float32))
    check_vectors(rp, ci, r)


def test_subspace_beyond_64_fp64_matches_oracle(fe):
    """FP64 storage at m = 96: the same products and eigenvalues as the oracle."""
    g = S.chung_lu_edges(20000, alpha=2.2, mean_deg=12, seed=21)
    A, rp, ci = setup(fe, g)
    X0 = S.normal((A.n, 8), seed=4)
    ref = oracle_ks(rp, ci, A.n, 8, 8, 96, 1e-10, X0)
    r = fe.fe_krylov_schur(A, 8, 8, 96, 1e-10, dtype=torch.float64,
                           start=torch.tensor(X0, device="cuda"))
    assert r.status == fe.FE_OK and ref.converged
    assert np.allclose(r.evals, ref.evals, rtol=1e-10, atol=0)
    assert r.spmm_calls == ref.spmm_calls
    check_vectors(rp, ci, r)


def test_wide_block_large_subspace_fp32(fe):
    """Block 16, m 112 (the fastest shape on the scale-27 graph): block
    updates and the restart run on the MFMA contraction with 16-column
    groups; FP32 storage against the FP64 oracle run with the same shape."""
    g = S.rmat_edges(14, seed=14)
    A, rp, ci = setup(fe, g)
    X0 = S.normal((A.n, 16), seed=5)
    ref = oracle_ks(rp, ci, A.n, 8, 16, 112, 1e-12, X0)
    r = fe.fe_krylov_schur(A, 8, 16, 112, 1e-6, dtype=torch.float32,
                           start=torch.tensor(X0, dtype=torch.float32, device="cuda"))
    assert r.status == fe.FE_OK
    assert np.all(np.abs(r.evals - ref.evals) <= 1e-8 * np.abs(ref.evals))
    assert np.all(r.resid <= resid_bar(1e-6, r.evals, torch.float32))
    check_vectors(rp, ci, r)


def test_subspace_limits(fe):
    g = S.rmat_edges(12, seed=1)
    A, rp, ci = setup(fe, g)
    for args in [(32, 8, 256), (8, 16, 272), (65, 16, 96)]:  # p = 144 > 128; m > 256; nev > 64
        with pytest.raises(fe.FeError) as e:
            fe.fe_krylov_schur(A, *args, 1e-8, dtype=torch.float32)
        assert e.value.status == fe.FE_EUNSUPPORTED


# ------------------------------------------- many-eigenvalue regime (nev 32)
@pytest.mark.parametrize("b,m", [(4, 128), (8, 192)])
def test_many_eigenvalues_fp64_matches_oracle(fe, b, m):
    """nev = 32 (the paper's many-eigenvalue runs), block 4 / m 128 (keeps
    p = 80 Ritz vectors) and block 8 / m 192 (p = 112): the restart and the
    final Ritz vectors need more than 64 output columns or more than 128
    basis columns, so the contraction reads its coefficients from a padded
    copy in device memory.  FP64 storage: same products and eigenvalues
    (1e-10) as the oracle from the same start block."""
    g = S.chung_lu_edges(20000, alpha=2.2, mean_deg=12, seed=31)
    A, rp, ci = setup(fe, g)
    X0 = S.normal((A.n, b), seed=7)
    ref = oracle_ks(rp, ci, A.n, 32, b, m, 1e-10, X0)
    r = fe.fe_krylov_schur(A, 32, b, m, 1e-10, dtype=torch.float64,
                           start=torch.tensor(X0, device="cuda"))
    assert r.status == fe.FE_OK and ref.converged
    assert np.allclose(r.evals, ref.evals, rtol=1e-10, atol=0)
    assert r.spmm_calls == ref.spmm_calls and r.restarts == ref.restarts
    check_vectors(rp, ci, r)


def test_many_eigenvalues_fp32(fe):
    g = S.rmat_edges(14, seed=14)
    A, rp, ci = setup(fe, g)
    X0 = S.normal((A.n, 4), seed=3)
    ref = oracle_ks(rp, ci, A.n, 32, 4, 128, 1e-12, X0)
    r = fe.fe_krylov_schur(A, 32, 4, 128, 1e-6, dtype=torch.float32,
                           start=torch.tensor(X0, dtype=torch.float32, device="cuda"))
    assert r.status == fe.FE_OK
    assert np.all(np.abs(r.evals - ref.evals) <= 1e-8 * np.abs(ref.evals))
    assert np.all(r.resid <= resid_bar(1e-6, r.evals, torch.float32))
    check_vectors(rp, ci, r)


def test_start_block_with_nan_and_repeated_columns(fe):
    """A caller's start block whose columns are not finite, or repeat, is
    repaired by the block QR's refill (the solver still converges)."""
    g = S.chung_lu_edges(20000, alpha=2.3, mean_deg=12, seed=9)
    A, rp, ci = setup(fe, g)
    ref = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float64, seed=3)
    X0 = torch.tensor(S.normal((A.n, 4), seed=5), device="cuda")
    X0[:, 2] = float("nan")
    r = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float64, start=X0)
    assert r.status == fe.FE_OK and r.refills >= 1
    assert np.allclose(r.evals, ref.evals, rtol=1e-10)
    X1 = torch.tensor(S.normal((A.n, 4), seed=6), device="cuda")
    X1[:, 3] = X1[:, 1]
    r = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float64, start=X1)
    assert r.status == fe.FE_OK and r.refills >= 1
    assert np.allclose(r.evals, ref.evals, rtol=1e-10)


@pytest.mark.parametrize("nev,b,m", [(4, 1, 24), (6, 2, 32), (8, 16, 64), (8, 4, 112),
                                     (8, 8, 112)])
def test_block_widths_fp64_match_oracle(fe, nev, b, m):
    """Block widths 1, 2 (element-load Gram), 16 (widest factor kernels),
    4 with m 112 (the fused CGS2 middle step up to 116 columns) and 8 with
    m 112 (the fused middle step up to 12 basis blocks in FP64, the separate
    update and Gram at 13): FP64 storage, same start block as the oracle:
    same products, eigenvalues within 1e-10."""
    g = S.chung_lu_edges(30000, alpha=2.2, mean_deg=12, seed=17)
    A, rp, ci = setup(fe, g)
    X0 = S.normal((A.n, b), seed=8)
    ref = oracle_ks(rp, ci, A.n, nev, b, m, 1e-9, X0)
    r = fe.fe_krylov_schur(A, nev, b, m, 1e-9, dtype=torch.float64,
                           start=torch.tensor(X0, device="cuda"))
    assert r.status == fe.FE_OK and ref.converged
    assert np.allclose(r.evals, ref.evals, rtol=1e-10, atol=0)
    assert r.spmm_calls == ref.spmm_calls
    check_vectors(rp, ci, r)


def _start_check_graph(fe):
    g = S.chung_lu_edges(16384, alpha=2.2, mean_deg=12, seed=21)
    return setup(fe, g)


def test_start_check_fallback_is_the_random_start_solve(fe):
    """A start block abandoned at restart c (start_drop so large that it
    always fires): the rest of the solve is the solve without a start block
    from the same seed, bit for bit, after m/b + c (m - p)/b products spent
    on the abandoned start; both agree with the FP64 oracle."""
    A, rp, ci = _start_check_graph(fe)
    nev, b, m = 8, 4, 32
    ref = fe.fe_krylov_schur(A, nev, b, m, 1e-8, dtype=torch.float64, seed=7)
    X0 = torch.tensor(S.normal((A.n, b), seed=3), device="cuda")
    for c in (1, 3):
        r = fe.fe_krylov_schur(A, nev, b, m, 1e-8, dtype=torch.float64, seed=7, start=X0,
                               start_check=c, start_drop=1e300)
        p = m - b * max(1, (m - nev) // (2 * b))
        assert r.status == fe.FE_OK and r.start_fallback == c
        assert r.spmm_calls == ref.spmm_calls + m // b + c * (m - p) // b
        assert r.restarts == ref.restarts + c + 1
        assert np.array_equal(r.evals, ref.evals)
        assert torch.equal(r.evecs, ref.evecs)
    orc = oracle_ks(rp, ci, A.n, nev, b, m, 1e-8, X0.cpu().numpy())
    assert np.allclose(ref.evals, orc.evals, rtol=1e-10, atol=0)


def test_start_check_kept_start_changes_nothing(fe):
    """A start block whose estimates fall (start_drop 1: any decrease keeps
    it): the watched solve is the unwatched one, bit for bit; without a start
    block the option is ignored; a mixed solve may abandon its start too."""
    A, rp, ci = _start_check_graph(fe)
    X0 = torch.tensor(S.normal((A.n, 4), seed=3), device="cuda")
    plain = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float64, seed=7, start=X0)
    kept = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float64, seed=7, start=X0,
                              start_check=3, start_drop=1.0)
    assert kept.start_fallback == -1 and plain.start_fallback == -1
    assert np.array_equal(kept.evals, plain.evals) and kept.spmm_calls == plain.spmm_calls
    rnd = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float64, seed=7)
    rnd2 = fe.fe_krylov_schur(A, 8, 4, 32, 1e-8, dtype=torch.float64, seed=7,
                              start_check=3, start_drop=1e300)
    assert rnd2.start_fallback == -1 and np.array_equal(rnd.evals, rnd2.evals)
    X32 = X0.float()
    mx = fe.fe_krylov_schur(A, 8, 4, 32, 1e-6, dtype=torch.float32, seed=7, start=X32,
                            mixed=True, start_check=2, start_drop=1e300)
    assert mx.status == fe.FE_OK and mx.start_fallback == 2
    assert np.all(np.abs(mx.evals - rnd.evals) <= 1e-8 * np.abs(rnd.evals))
    assert np.all(mx.resid <= resid_bar(1e-6, mx.evals, torch.float32))


# ------------------------------------------------- caller-owned workspace
@pytest.mark.parametrize("dtype,mixed,with_start", [(torch.float64, False, True),
                                                    (torch.float32, True, True),
                                                    (torch.float32, False, False)])
def test_workspace_makes_no_device_allocation(fe, dtype, mixed, with_start):
    """A torch buffer of fe_ks_workspace_bytes bytes passed as the solve's
    workspace: the library makes no device allocation during the call (mixed
    storage included, whose switch needs a second subspace), and the result is
    bitwise the result of a solve that allocates its own memory."""
    g = S.chung_lu_edges(30000, alpha=2.2, mean_deg=12, seed=41)
    A, rp, ci = setup(fe, g)
    start = torch.tensor(S.normal((A.n, 4), seed=5), device="cuda").to(dtype) if with_start else None
    kw = dict(dtype=dtype, mixed=mixed, start=start, seed=3)
    r1 = fe.fe_krylov_schur(A, 8, 4, 48, 1e-6, **kw)
    nbytes = fe.fe_ks_workspace_bytes(A, 8, 4, 48, dtype=dtype, mixed=mixed, start=start)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    r2 = fe.fe_krylov_schur(A, 8, 4, 48, 1e-6, workspace=ws, **kw)
    assert r1.status == fe.FE_OK and r2.status == fe.FE_OK
    assert r1.device_allocs > 0 and r2.device_allocs == 0
    assert np.array_equal(r1.evals, r2.evals) and r1.spmm_calls == r2.spmm_calls
    assert torch.equal(r1.evecs, r2.evecs)
    if mixed:
        assert r2.switch_restart >= 0
    with pytest.raises(fe.FeError) as e:
        fe.fe_krylov_schur(A, 8, 4, 48, 1e-6, workspace=ws[: nbytes - 256], **kw)
    assert e.value.status == fe.FE_EINVAL


@pytest.mark.parametrize("keep", [8, 16, 24])
def test_restart_size_option_matches_oracle(fe, keep):
    """opts.keep: the number of Ritz vectors a restart keeps (default formula
    otherwise).  FP64 storage, the oracle run with the same keep: same
    products and eigenvalues."""
    g = S.chung_lu_edges(20000, alpha=2.2, mean_deg=12, seed=51)
    A, rp, ci = setup(fe, g)
    X0 = S.normal((A.n, 4), seed=6)
    ref = oracle_ks(rp, ci, A.n, 8, 4, 32, 1e-10, X0, keep=keep)
    r = fe.fe_krylov_schur(A, 8, 4, 32, 1e-10, dtype=torch.float64,
                           start=torch.tensor(X0, device="cuda"), keep=keep)
    assert r.status == fe.FE_OK and ref.converged
    assert np.allclose(r.evals, ref.evals, rtol=1e-10, atol=0)
    assert r.spmm_calls == ref.spmm_calls and r.restarts == ref.restarts
    for bad in (4, 30, 29):  # below nev; above m - block; m - keep not a multiple of block
        with pytest.raises(fe.FeError) as e:
            fe.fe_krylov_schur(A, 8, 4, 32, 1e-10, dtype=torch.float64, keep=bad)
        assert e.value.status == fe.FE_EINVAL


@pytest.mark.parametrize("n", [301, 4099])
def test_block16_ragged_rows_fp64_match_oracle(fe, n):
    """Block 16 at row counts off the 16-row group and the row intervals of
    the fused CGS2 kernels (middle step, last step with its Gram) and of the
    start block's device Cholesky QR: FP64 storage, same start block as the
    oracle: same products, eigenvalues within 1e-10."""
    g = S.chung_lu_edges(n, alpha=2.2, mean_deg=12, seed=23)
    A, rp, ci = setup(fe, g)
    X0 = S.normal((A.n, 16), seed=9)
    ref = oracle_ks(rp, ci, A.n, 8, 16, 64, 1e-9, X0)
    r = fe.fe_krylov_schur(A, 8, 16, 64, 1e-9, dtype=torch.float64,
                           start=torch.tensor(X0, device="cuda"))
    assert r.status == fe.FE_OK and ref.converged
    assert np.allclose(r.evals, ref.evals, rtol=1e-10, atol=0)
    assert r.spmm_calls == ref.spmm_calls
    check_vectors(rp, ci, r)


def test_block16_small_graph_against_dense_eigh(fe):
    """n = 90 with block 16, m 64 (the subspace nearly fills the space, so
    dependent columns and refills occur): the 8 largest-magnitude
    eigenvalues of the dense matrix."""
    n, s, d = S.chung_lu_edges(90, alpha=2.2, mean_deg=10, seed=5)
    A, rp, ci = setup(fe, (n, s, d))
    D = np.zeros((n, n))
    for i in range(n):
        D[i, ci[rp[i]:rp[i + 1]]] = 1.0
    w = np.linalg.eigvalsh(D)
    want = w[np.argsort(-np.abs(w), kind="stable")][:8]
    r = fe.fe_krylov_schur(A, 8, 16, 64, 1e-10, dtype=torch.float64, seed=4)
    assert r.status == fe.FE_OK
    assert np.allclose(np.sort(r.evals), np.sort(want), rtol=1e-9, atol=1e-9)
