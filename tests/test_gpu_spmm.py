"""Parity of the HIP sparse product (fe_spmm) and CSR build with the oracle.

Bars: integer work (CSR, degree order) bitwise; small-integer X bitwise in
every dtype (all partial sums exact); N(0,1) X entrywise
|dY| <= tol * sum_j |X_j| + output rounding, tol = 1e-5 (FP32 accumulate),
1e-13 (FP64); BF16 X is compared against the oracle fed the same BF16 values.
"""
import numpy as np
import pytest
import torch

import fe_synth as S
import oracle as O

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def to_dev(x, dt):
    return torch.tensor(np.asarray(x), dtype=torch.float64).to(dt).cuda()


def graph(name):
    if name == "chung_lu_64k":
        return S.chung_lu_edges(65536, alpha=2.1, mean_deg=16, seed=1)
    if name == "rmat14":
        return S.rmat_edges(14, seed=14)
    if name == "star40k":  # one hub above the split threshold
        return S.star_graph(40000)
    if name == "complete300":
        return S.complete_graph(300)
    if name == "cycle1001":
        return S.cycle_graph(1001)
    raise KeyError(name)


_cache = {}


def built(fe, name, relabel):
    key = (name, relabel)
    if key not in _cache:
        n, s, d = graph(name)
        flags = fe.FE_GRAPH_DEFAULT | (fe.FE_RELABEL_BY_DEGREE if relabel else 0)
        A = fe.fe_csr_build(n, s, d, flags)
        rp, ci = O.csr_from_edges(n, s, d)
        _cache[key] = (A, rp, ci)
    return _cache[key]


def internal_oracle(A, rp, ci, X):
    """Oracle product expressed in the handle's numbering."""
    perm = A.perm()
    Y = O.spmm(rp, ci, X)
    return Y[perm], perm


@pytest.mark.parametrize("name", ["chung_lu_64k", "rmat14", "star40k", "complete300"])
@pytest.mark.parametrize("relabel", [False, True])
def test_csr_build_matches_oracle(fe, name, relabel):
    A, rp, ci = built(fe, name, relabel)
    grp, gci = A.export()
    perm = A.perm()
    deg = np.diff(rp)
    # degree order: descending degree, ties by ascending id (unique)
    order = np.lexsort((np.arange(A.n), -deg))
    if relabel:
        assert np.array_equal(perm, order)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(A.n, dtype=perm.dtype)
        rp2, ci2 = O.csr_from_edges(A.n, *[inv[v] for v in (O_src(name), O_dst(name))])
        assert np.array_equal(grp, rp2) and np.array_equal(gci, ci2)
    else:
        assert np.array_equal(perm, np.arange(A.n))
        assert np.array_equal(grp, rp) and np.array_equal(gci, ci)
    assert A.nnz == rp[-1] and A.max_deg == deg.max()


def O_src(name):
    return graph(name)[1]


def O_dst(name):
    return graph(name)[2]


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("b", [1, 2, 3, 4, 8, 16, 64])
@pytest.mark.parametrize("name,relabel", [("chung_lu_64k", True), ("rmat14", False),
                                          ("star40k", True), ("complete300", False)])
def test_spmm_small_int_bitwise(fe, name, relabel, dt, b):
    A, rp, ci = built(fe, name, relabel)
    X = S.small_ints((A.n, b), seed=21, lo=-8, hi=8)
    want, perm = internal_oracle(A, rp, ci, X)
    Y = fe.fe_spmm(A, to_dev(X[perm], DT[dt])).double().cpu().numpy()
    if dt == "bf16":
        want = O.round_bf16(want)
    assert np.array_equal(Y, want)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("b", [1, 4, 5, 8, 16, 32])
@pytest.mark.parametrize("name,relabel", [("chung_lu_64k", False), ("rmat14", True),
                                          ("star40k", False), ("cycle1001", True)])
def test_spmm_normal_tolerance(fe, name, relabel, dt, b):
    A, rp, ci = built(fe, name, relabel)
    X = S.normal((A.n, b), seed=5)
    Xd = to_dev(X[A.perm()], DT[dt])
    Xq = Xd.double().cpu().numpy()  # the values the kernel actually reads
    perm = A.perm()
    inv = np.empty_like(perm)
    inv[perm] = np.arange(A.n, dtype=perm.dtype)
    Xo = Xq[inv]  # back to original numbering
    want = O.spmm(rp, ci, Xo)[perm]
    absum = O.spmm(rp, ci, np.abs(Xo))[perm]
    Y = fe.fe_spmm(A, Xd).double().cpu().numpy()
    tol = {"f64": 1e-13, "f32": 1e-5, "bf16": 1e-5}[dt]
    bound = tol * absum + (2.0 ** -8 * np.abs(want) if dt == "bf16" else 0.0)
    assert np.all(np.abs(Y - want) <= bound + 1e-300)


def test_spmm_deterministic_and_threshold_rows(fe):
    # rows whose degrees sit on every bin boundary (1, 2, 64, 65, 2048, 2049, 16384, 16385, 40000)
    degs = [1, 2, 3, 4, 64, 65, 2048, 2049, 16384, 16385, 40000]
    n = 60000
    src, dst = [], []
    base = 1
    for i, d in enumerate(degs):
        src.append(np.full(d, i))
        dst.append(np.arange(base, base + d) % n)
        base += 1000
    s = np.concatenate(src)
    d = np.concatenate(dst)
    A = fe.fe_csr_build(n, s, d, fe.FE_GRAPH_DEFAULT)
    rp, ci = O.csr_from_edges(n, s, d)
    X = S.small_ints((n, 4), seed=3)
    Xd = to_dev(X, torch.float32)
    Y1 = fe.fe_spmm(A, Xd)
    Y2 = fe.fe_spmm(A, Xd)
    assert torch.equal(Y1, Y2)
    assert np.array_equal(Y1.double().cpu().numpy(), O.spmm(rp, ci, X))


def test_spmm_empty_and_tiny(fe):
    A = fe.fe_csr_build(10, np.zeros(0, np.int32), np.zeros(0, np.int32))
    Y = fe.fe_spmm(A, torch.ones((10, 4), dtype=torch.float32, device="cuda"))
    assert torch.count_nonzero(Y) == 0
    A1 = fe.fe_csr_build(1, np.zeros(1, np.int32), np.zeros(1, np.int32))  # only a self-loop
    assert A1.nnz == 0
    Y1 = fe.fe_spmm(A1, torch.full((1, 3), 7.0, dtype=torch.float64, device="cuda"))
    assert torch.count_nonzero(Y1) == 0


def test_spmm_rejects_bad_arguments(fe):
    A, rp, ci = built(fe, "cycle1001", False)
    X = torch.zeros((A.n, 65), dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_spmm(A, X)
    assert e.value.status == fe.FE_EINVAL
    X = torch.zeros((A.n, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_spmm(A, X, X)
    assert e.value.status == fe.FE_EINVAL
    with pytest.raises(fe.FeError) as e:
        fe.fe_csr_build(5, np.array([0, 7], np.int32), np.array([1, 2], np.int32))
    assert e.value.status == fe.FE_EINVAL


@pytest.mark.parametrize("b", [1, 4, 8, 16])
def test_spmm_rmat22_sampled_rows(fe, b):
    """R-MAT scale 22, edge factor 16, (.57,.19,.19,.05), FP32, relabelled as
    in the benchmark; sampled rows (all hub rows plus random rows) against the
    oracle computed row by row from the edge stream."""
    key = "rmat22"
    if key not in _cache:
        n, s, d = S.rmat_edges(22, seed=22)
        A = fe.fe_csr_build(n, s, d, fe.FE_GRAPH_DEFAULT | fe.FE_RELABEL_BY_DEGREE)
        _cache[key] = (A, n, s, d)
    A, n, s, d = _cache[key]
    perm = A.perm()
    X = S.normal((n, b), seed=7)
    Xd = to_dev(X[perm], torch.float32)
    Xq = np.empty_like(X)
    Xq[perm] = Xd.double().cpu().numpy()
    Y = fe.fe_spmm(A, Xd).double().cpu().numpy()
    rng = np.random.default_rng(b)
    new_rows = np.unique(np.concatenate([np.arange(64), rng.integers(0, n, 1500),
                                         np.arange(n - 16, n)]))
    old_rows = perm[new_rows]
    order = np.argsort(old_rows)
    want = O.spmm_rows_from_edges(n, s, d, Xq, old_rows[order])
    absum = O.spmm_rows_from_edges(n, s, d, np.abs(Xq), old_rows[order])
    got = Y[new_rows][order]
    assert np.all(np.abs(got - want) <= 1e-5 * absum + 1e-30)


@pytest.mark.parametrize("name", ["rmat14", "star40k", "cycle1001"])
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("b", [1, 3, 16])
def test_gather_bound_touches_every_stored_nonzero(fe, name, dt, b):
    """The measurement kernel (the product's gathers without its rows) sums the
    X row of every stored nonzero exactly once: on small integers its total is
    exactly the oracle product's total."""
    A, rp, ci = built(fe, name, True)
    X = S.small_ints((A.n, b), seed=5, lo=-3, hi=3)
    perm = A.perm()
    out = fe.fe_spmm_gather_bound(A, to_dev(X[perm], DT[dt]))
    assert out.numel() == fe.lib().fe_spmm_gather_bound_sets()
    assert float(out.sum().item()) == float(O.spmm(rp, ci, X).sum())


def test_gather_bound_empty_matrix(fe):
    A = fe.fe_csr_build(10, np.zeros(0, np.int32), np.zeros(0, np.int32))
    out = fe.fe_spmm_gather_bound(A, torch.ones((10, 4), dtype=torch.float32, device="cuda"))
    assert torch.count_nonzero(out) == 0


@pytest.mark.parametrize("dt", ["f32", "bf16", "f64"])
def test_gather_rows_over_a_given_stream(fe, dt):
    """fe_gather_rows sums X row idx[e] for every entry of the stream; indices
    outside [0, n) are clamped to it."""
    n, b = 5000, 16
    X = S.small_ints((n, b), seed=9, lo=-3, hi=3)
    rng = np.random.default_rng(4)
    idx = rng.integers(-50, n + 50, 200_003).astype(np.int32)
    out = fe.fe_gather_rows(torch.from_numpy(idx).cuda(), to_dev(X, DT[dt]))
    want = X[np.clip(idx, 0, n - 1)].sum()
    assert float(out.sum().item()) == float(want)
    empty = fe.fe_gather_rows(torch.zeros(0, dtype=torch.int32, device="cuda"), to_dev(X, DT[dt]))
    assert torch.count_nonzero(empty) == 0
