"""Parity of fe_gram (C = alpha V^T W) and fe_block_update (W = beta W + alpha V C).

Bars: small-integer inputs bitwise (exact in FP64 arithmetic and in the
storage dtype); N(0,1) inputs: Gram within 1e-13 * sum |V||W| of the FP64
oracle on the same stored values; update within one storage ulp plus
1e-13 * sum of |terms|.
"""
import numpy as np
import pytest
import torch

import fe_synth as S
import oracle as O

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
ULP = {"f64": 2.0 ** -52, "f32": 2.0 ** -23, "bf16": 2.0 ** -7}


def dev(x, dt):
    return torch.tensor(np.asarray(x), dtype=torch.float64).to(dt).cuda()


def host(t):
    return t.double().cpu().numpy()


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,nblk,b", [(1, 1, 1), (37, 3, 4), (1000, 13, 4), (4097, 6, 8),
                                      (777, 2, 16), (5000, 5, 3), (300, 1, 64), (70001, 12, 4),
                                      (1001, 5, 16), (3333, 9, 8), (15, 8, 16), (2001, 17, 4),
                                      (4099, 31, 4), (999, 11, 8), (20003, 16, 8), (17, 15, 8),
                                      (3001, 40, 4), (1003, 24, 8)])
def test_gram_small_int_bitwise(fe, dt, n, nblk, b):
    """Every column-group count per slice and slices split evenly (b = 4, 8:
    up to 8 groups of 16 columns per slice in 4- and 2-byte storage, 4 in
    FP64), ragged and tiny row counts: exact on small integers."""
    V = S.small_ints((nblk, n, b), seed=1, lo=-4, hi=4)
    W = S.small_ints((n, b), seed=2, lo=-4, hi=4)
    C = host(fe.fe_gram(dev(V, DT[dt]), dev(W, DT[dt]), alpha=2.0))
    Vf = V.transpose(1, 0, 2).reshape(n, nblk * b)  # column p = block p // b, col p % b
    assert np.array_equal(C, O.gram(Vf, W, alpha=2.0))


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,nblk,b", [(4099, 13, 4), (100003, 7, 8), (5000, 3, 16), (2000, 20, 2),
                                      (20011, 8, 16), (9999, 15, 8)])
def test_gram_normal(fe, dt, n, nblk, b):
    Vd = dev(S.normal((nblk, n, b), seed=3), DT[dt])
    Wd = dev(S.normal((n, b), seed=4), DT[dt])
    V, W = host(Vd), host(Wd)
    Vf = V.transpose(1, 0, 2).reshape(n, nblk * b)
    want = O.gram(Vf, W)
    bound = 1e-13 * (np.abs(Vf).T @ np.abs(W))
    C = host(fe.fe_gram(Vd, Wd))
    assert np.all(np.abs(C - want) <= bound)
    C2 = host(fe.fe_gram(Vd, Wd))
    assert np.array_equal(C, C2)  # fixed reduction order


def test_gram_w_is_a_block_of_v(fe):
    V = dev(S.normal((5, 3000, 4), seed=5), torch.float32)
    C = host(fe.fe_gram(V, V[4]))
    Vf = host(V).transpose(1, 0, 2).reshape(3000, 20)
    assert np.allclose(C, Vf.T @ Vf[:, 16:20], rtol=1e-12, atol=1e-10)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,nblk,b", [(1, 1, 1), (1000, 3, 4), (4097, 12, 8), (999, 2, 16),
                                      (500, 3, 5), (300, 2, 64)])
def test_update_small_int_bitwise(fe, dt, n, nblk, b):
    V = S.small_ints((nblk, n, b), seed=6, lo=-3, hi=3)
    W = S.small_ints((n, b), seed=7, lo=-3, hi=3)
    C = S.small_ints((nblk * b, b), seed=8, lo=-3, hi=3)
    Wd = dev(W, DT[dt])
    fe.fe_block_update(Wd, dev(V, DT[dt]), dev(C, torch.float64), alpha=-1.0, beta=2.0)
    Vf = V.transpose(1, 0, 2).reshape(n, nblk * b)
    want = O.block_update(W, Vf, C, alpha=-1.0, beta=2.0)
    if dt == "bf16":
        want = O.round_bf16(want)
    assert np.array_equal(host(Wd), want)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,nblk,b", [(10007, 12, 4), (3001, 6, 8), (2048, 3, 16)])
def test_update_normal(fe, dt, n, nblk, b):
    Vd = dev(S.normal((nblk, n, b), seed=9), DT[dt])
    Wd = dev(S.normal((n, b), seed=10), DT[dt])
    C = S.normal((nblk * b, b), seed=11)
    V, W = host(Vd), host(Wd)
    Vf = V.transpose(1, 0, 2).reshape(n, nblk * b)
    want = O.block_update(W, Vf, C, alpha=-0.5, beta=1.0)
    mag = np.abs(W) + 0.5 * (np.abs(Vf) @ np.abs(C))
    fe.fe_block_update(Wd, Vd, dev(C, torch.float64), alpha=-0.5, beta=1.0)
    got = host(Wd)
    assert np.all(np.abs(got - want) <= ULP[dt] * np.abs(want) + 1e-13 * mag + 1e-300)


def test_update_in_place_right_multiply(fe):
    n, b = 5000, 4
    W = S.normal((n, b), seed=12)
    M = np.triu(S.normal((b, b), seed=13)) + 3 * np.eye(b)
    Wd = dev(W, torch.float64)
    fe.fe_block_update(Wd, Wd, dev(M, torch.float64), alpha=1.0, beta=0.0)
    assert np.allclose(host(Wd), W @ M, rtol=1e-14, atol=1e-13)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("b", [3, 5, 12, 4, 16])
def test_update_in_place_every_width(fe, dt, b):
    """W <- 2 W - W C in place (W == V, one block) at widths whose rows
    straddle wavefronts (b = 3, 5, 12) and at the specialised widths: every
    row is read before any of it is written, so the result is exact on small
    integers."""
    n = 10_007
    W = S.small_ints((n, b), seed=44, lo=-3, hi=3)
    C = S.small_ints((b, b), seed=45, lo=-2, hi=2)
    Wd = dev(W, DT[dt])
    fe.fe_block_update(Wd, Wd, dev(C, torch.float64), alpha=-1.0, beta=2.0)
    want = O.block_update(W, W, C, alpha=-1.0, beta=2.0)
    if dt == "bf16":
        want = O.round_bf16(want)
    assert np.array_equal(host(Wd), want)


def test_update_beta_zero_ignores_nan(fe):
    n, b = 100, 4
    W = torch.full((n, b), float("nan"), dtype=torch.float32, device="cuda")
    V = dev(S.normal((1, n, b), seed=1), torch.float32)
    C = dev(np.eye(b), torch.float64)
    fe.fe_block_update(W, V, C, alpha=1.0, beta=0.0)
    assert torch.equal(W, V[0])


def test_update_rejects_overlap(fe):
    V = torch.zeros((3, 100, 4), dtype=torch.float32, device="cuda")
    C = torch.zeros((12, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_block_update(V[1], V, C)
    assert e.value.status == fe.FE_EINVAL


# ----------------------------------------------- fused update + Gram
@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,nblk,b", [(1, 1, 1), (1000, 3, 4), (4097, 12, 4), (4097, 8, 8),
                                      (999, 2, 16), (130, 4, 16), (70001, 12, 4), (65, 5, 2)])
def test_update_gram_small_int_bitwise(fe, dt, n, nblk, b):
    """Integer inputs: W' = W - V C exactly (then rounded to the storage type),
    and [V W']^T W' exactly, from the rounded W'."""
    V = S.small_ints((nblk, n, b), seed=21, lo=-3, hi=3)
    W = S.small_ints((n, b), seed=22, lo=-3, hi=3)
    C = S.small_ints((nblk * b, b), seed=23, lo=-3, hi=3)
    Wd = dev(W, DT[dt])
    Cout = host(fe.fe_block_update_gram(Wd, dev(V, DT[dt]), dev(C, torch.float64)))
    Vf = V.transpose(1, 0, 2).reshape(n, nblk * b)
    Wn = O.block_update(W, Vf, C, alpha=-1.0, beta=1.0)
    if dt == "bf16":
        Wn = O.round_bf16(Wn)
    assert np.array_equal(host(Wd), Wn)
    assert np.array_equal(Cout, O.gram(np.hstack([Vf, Wn]), Wn))


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("n,nblk,b", [(100003, 12, 4), (30001, 6, 8), (4096, 3, 16), (777, 1, 1)])
def test_update_gram_normal(fe, dt, n, nblk, b):
    Vd = dev(S.normal((nblk, n, b), seed=24), DT[dt])
    Wd = dev(S.normal((n, b), seed=25), DT[dt])
    C = S.normal((nblk * b, b), seed=26)
    V, W = host(Vd), host(Wd)
    Vf = V.transpose(1, 0, 2).reshape(n, nblk * b)
    want = O.block_update(W, Vf, C, alpha=-1.0, beta=1.0)
    mag = np.abs(W) + np.abs(Vf) @ np.abs(C)
    Cout = host(fe.fe_block_update_gram(Wd, Vd, dev(C, torch.float64)))
    got = host(Wd)
    assert np.all(np.abs(got - want) <= ULP[dt] * np.abs(want) + 1e-13 * mag + 1e-300)
    X = np.hstack([Vf, got])  # the Gram is taken from the rounded result
    bound = 1e-13 * (np.abs(X).T @ np.abs(got))
    assert np.all(np.abs(Cout - O.gram(X, got)) <= bound)


FUSED_SHAPES = [(4, 1), (4, 3), (4, 7), (4, 11), (4, 15), (4, 19), (4, 23), (4, 27), (4, 31),
                (8, 1), (8, 2), (8, 3), (8, 4), (8, 5), (8, 7), (8, 9), (8, 11), (8, 12), (8, 13),
                (8, 15), (16, 1), (16, 2), (16, 3), (16, 4), (16, 5), (16, 6), (16, 7)]


@pytest.mark.parametrize("dt,b,nblk", [(dt, b, nblk) for dt in ("f64", "f32", "bf16")
                                       for b, nblk in FUSED_SHAPES
                                       if not (dt == "f64" and b == 8 and nblk > 12)])
@pytest.mark.parametrize("n", [1, 17, 40003])
def test_fused_cgs_step_every_tile_count(fe, dt, b, nblk, n):
    """The solver's one-pass CGS2 middle step (b = 4: column groups of 16 in
    one workgroup slice; b = 8, 16: G basis tiles on 16 x 16 MFMA, a half tile
    last when b = 8 and the block count is odd), for every tile count up to
    128 columns of [V W] and for row counts below, at and off the 16-row
    group: on small integers W' and [V W']^T W' are exact.  FP64 at b = 8
    stops at 12 basis blocks (13 is refused: the rejects test)."""
    V = S.small_ints((nblk, n, b), seed=31, lo=-3, hi=3)
    W = S.small_ints((n, b), seed=32, lo=-3, hi=3)
    C = S.small_ints((nblk * b, b), seed=33, lo=-3, hi=3)
    Wd = dev(W, DT[dt])
    Cout = host(fe.fe_block_update_gram(Wd, dev(V, DT[dt]), dev(C, torch.float64)))
    Vf = V.transpose(1, 0, 2).reshape(n, nblk * b)
    Wn = O.block_update(W, Vf, C, alpha=-1.0, beta=1.0)
    if dt == "bf16":
        Wn = O.round_bf16(Wn)
    assert np.array_equal(host(Wd), Wn)
    assert np.array_equal(Cout, O.gram(np.hstack([Vf, Wn]), Wn))


@pytest.mark.parametrize("b,nblk", [(4, 27), (8, 11), (16, 6)])
def test_fused_cgs_step_matches_separate_calls(fe, b, nblk):
    """N(0,1) inputs, FP64: the fused step against fe_block_update followed by
    fe_gram (the same arithmetic up to the order of the FP64 sums)."""
    n = 300001
    Vd = dev(S.normal((nblk, n, b), seed=34), torch.float64)
    W0 = dev(S.normal((n, b), seed=35), torch.float64)
    C = dev(S.normal((nblk * b, b), seed=36), torch.float64)
    W1, W2 = W0.clone(), W0.clone()
    Cf = host(fe.fe_block_update_gram(W1, Vd, C))
    fe.fe_block_update(W2, Vd, C, alpha=-1.0, beta=1.0)
    Cs = host(fe.fe_gram(torch.cat([Vd, W2.unsqueeze(0)]), W2))
    mag = np.abs(host(W0)) + np.abs(host(Vd).transpose(1, 0, 2).reshape(n, -1)) @ np.abs(host(C))
    assert np.all(np.abs(host(W1) - host(W2)) <= 1e-14 * mag)
    assert np.allclose(Cf, Cs, rtol=1e-11, atol=1e-8)


@pytest.mark.parametrize("b", [2, 8])
def test_update_gram_equals_separate_calls(fe, b):
    """FP32 storage: at b = 2 (the plain fused update + Gram) W' is bitwise the
    separate update's; at b = 8 (the MFMA middle step, another FP64 summation
    order) within one FP32 rounding of it."""
    n, nblk = 20000, 6
    Vd = dev(S.normal((nblk, n, b), seed=27), torch.float32)
    W0 = dev(S.normal((n, b), seed=28), torch.float32)
    C = dev(S.normal((nblk * b, b), seed=29), torch.float64)
    W1, W2 = W0.clone(), W0.clone()
    Cf = host(fe.fe_block_update_gram(W1, Vd, C))
    fe.fe_block_update(W2, Vd, C, alpha=-1.0, beta=1.0)
    Cs = host(fe.fe_gram(torch.cat([Vd, W2.unsqueeze(0)]), W2))
    if b == 2:
        assert torch.equal(W1, W2)  # identical FP64 arithmetic per element, same rounding
    else:
        mag = np.abs(host(W0)) + np.abs(host(Vd).transpose(1, 0, 2).reshape(n, -1)) @ np.abs(host(C))
        assert np.all(np.abs(host(W1) - host(W2)) <= ULP["f32"] * np.abs(host(W2)) + 1e-14 * mag)
    assert np.allclose(Cf, Cs, rtol=1e-12, atol=1e-9)


def test_update_gram_rejects(fe):
    V = torch.zeros((3, 100, 4), dtype=torch.float32, device="cuda")
    C = torch.zeros((12, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_block_update_gram(V[1], V, C)
    assert e.value.status == fe.FE_EINVAL
    V3 = torch.zeros((2, 100, 3), dtype=torch.float32, device="cuda")
    W3 = torch.zeros((100, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_block_update_gram(W3, V3, torch.zeros((6, 3), dtype=torch.float64, device="cuda"))
    assert e.value.status == fe.FE_EUNSUPPORTED
    V32 = torch.zeros((32, 100, 4), dtype=torch.float32, device="cuda")  # k + b = 132 > 128
    W4 = torch.zeros((100, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_block_update_gram(W4, V32, torch.zeros((128, 4), dtype=torch.float64, device="cuda"))
    assert e.value.status == fe.FE_EUNSUPPORTED
    V16 = torch.zeros((16, 100, 8), dtype=torch.float32, device="cuda")  # b = 8: k + b = 136
    W8 = torch.zeros((100, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_block_update_gram(W8, V16, torch.zeros((128, 8), dtype=torch.float64, device="cuda"))
    assert e.value.status == fe.FE_EUNSUPPORTED
    V13 = torch.zeros((13, 100, 8), dtype=torch.float64, device="cuda")  # FP64, b = 8: 13 blocks
    W8d = torch.zeros((100, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_block_update_gram(W8d, V13, torch.zeros((104, 8), dtype=torch.float64, device="cuda"))
    assert e.value.status == fe.FE_EUNSUPPORTED
