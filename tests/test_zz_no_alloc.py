"""fe_gram_noalloc (the Gram product with the library's static partials
array, for callers that cannot allocate) against fe_gram, through the C ABI:
bitwise equal, on two calls in a row, the second with a smaller input, in
every storage dtype; and the size limit is an error raised before any launch."""
import numpy as np
import pytest
import torch

import fe_synth as S

pytestmark = pytest.mark.gpu

DT = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}


def _blocks(nblk, n, b, seed, dt):
    V = torch.tensor(S.normal((nblk, n, b), seed=seed), device="cuda").to(dt)
    W = torch.tensor(S.normal((n, b), seed=seed + 1), device="cuda").to(dt)
    return V, W


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16"])
def test_noalloc_gram_equals_gram_twice(fe, dt):
    for (nblk, n, b) in [(12, 300_001, 8), (3, 5_000, 4)]:  # second call smaller
        V, W = _blocks(nblk, n, b, 40 + nblk, DT[dt])
        want = fe.fe_gram(V, W, alpha=-0.5)
        C = torch.full((nblk * b, b), float("nan"), dtype=torch.float64, device="cuda")
        fe.fe_gram_noalloc(V, W, C, alpha=-0.5)
        torch.cuda.synchronize()
        assert torch.equal(C, want), (dt, nblk, n, b)


@pytest.mark.parametrize("b", [1, 2, 5, 16])
def test_noalloc_gram_widths(fe, b):
    nblk, n = 4, 40_000
    V, W = _blocks(nblk, n, b, 7, torch.float32)
    want = fe.fe_gram(V, W)
    C = torch.empty((nblk * b, b), dtype=torch.float64, device="cuda")
    fe.fe_gram_noalloc(V, W, C)
    torch.cuda.synchronize()
    assert torch.equal(C, want)


def test_noalloc_gram_rejects_oversize(fe):
    # 512 row sets x (256 x 16) partials = 2.1M doubles > the 1M-double array
    nblk, n, b = 16, 70_000, 16
    V = torch.zeros((nblk, n, b), dtype=torch.bfloat16, device="cuda")
    W = torch.zeros((n, b), dtype=torch.bfloat16, device="cuda")
    C = torch.zeros((nblk * b, b), dtype=torch.float64, device="cuda")
    with pytest.raises(fe.FeError) as e:
        fe.fe_gram_noalloc(V, W, C)
    assert e.value.status == fe.FE_EUNSUPPORTED
