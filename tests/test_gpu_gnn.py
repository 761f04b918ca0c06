"""Learned-start network on the GPU against the FP64 oracle.

Bars: BF16 forward (BF16 transform operands, FP32 accumulation) against the
exact oracle: output X within 2e-2 relative (Frobenius, per column).  Against
the oracle whose transform operands are rounded to BF16 the same way (the
BF16 reading of the network): X within 1e-3, loss within 1e-4, every
parameter tensor's gradient within 1e-2 relative (Frobenius) -- what is left
is FP32 accumulation and the rare operand whose FP32 and FP64 values round
to different BF16 neighbours, amplified by the subspace loss's near
cancellation.  FP32 compute mode: X within 1e-4, loss within 1e-5, each
gradient tensor within 1e-4 relative.  An Adam step matches the oracle's
Adam on the GPU's own gradients to 1e-5.
"""
import numpy as np
import pytest
import torch

import fe_synth as S
import oracle as O
from oracle import gnn as G

pytestmark = pytest.mark.gpu


def case(fe, n=6000, seed=4, relabel=False):
    n, s, d = S.chung_lu_edges(n, alpha=2.2, mean_deg=10, seed=seed)
    flags = fe.FE_GRAPH_DEFAULT | (fe.FE_RELABEL_BY_DEGREE if relabel else 0)
    A = fe.fe_csr_build(n, s, d, flags)
    rp, ci = O.csr_from_edges(n, s, d)
    z = S.normal((n, 15), seed=seed + 1)
    V, _ = np.linalg.qr(S.normal((n, 8), seed=seed + 2))
    return A, rp, ci, z, V


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("relabel", [False, True])
def test_forward_matches_oracle(fe, relabel):
    A, rp, ci, z, V = case(fe, relabel=relabel)
    net = fe.Gnn(seed=7)
    params = fe.gnn_unflatten(net.get_params())
    X = net.forward(A, torch.tensor(z, dtype=torch.float32, device="cuda")).double().cpu().numpy()
    Xo, _ = G.forward(rp, ci, G.features(rp, z), params)
    for j in range(8):
        assert rel(X[:, j], Xo[:, j]) < 2e-2, j


def cosine(a, b):
    a, b = np.ravel(a), np.ravel(b)
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("compute,relabel,n", [("f32", False, 5000), ("f32", True, 5000),
                                               ("bf16", False, 5000), ("bf16", True, 5000),
                                               ("f32", True, 21111)])
def test_gradients_match_oracle(fe, relabel, compute, n):
    """n = 5000: 20 row intervals with a ragged last one; n = 21111: 83
    intervals, so the fixed-order set sum runs over three groups, the last
    one partial."""
    A, rp, ci, z, V = case(fe, n=n, seed=9, relabel=relabel)
    net = fe.Gnn(seed=3, compute=compute)
    params = fe.gnn_unflatten(net.get_params())
    for l in range(3):  # non-zero biases exercise the bias path
        params[f"b{l}"] = 0.05 * S.normal((64,), seed=20 + l)
    net.set_params(fe.gnn_flatten(params))
    params = fe.gnn_unflatten(fe.gnn_flatten(params))  # the FP32 values the GPU holds
    zt = torch.tensor(z, dtype=torch.float32, device="cuda")
    X = net.forward(A, zt).double().cpu().numpy()
    loss, g = net.backward(A, zt, torch.tensor(V, dtype=torch.float32, device="cuda"),
                           want_grads=True)
    rounding = O.round_bf16 if compute == "bf16" else None
    Xo, cache = G.forward(rp, ci, G.features(rp, z), params, transform_inputs=rounding)
    lo = G.loss(Xo, V)
    go = G.backward(rp, ci, params, cache, G.loss_grad(Xo, V))
    gd = fe.gnn_unflatten(g)
    errs = {name: rel(gd[name], go[name]) for name in go}
    print(f"{compute}: X {rel(X, Xo):.2e} loss {abs(loss - lo):.2e} grads max "
          f"{max(errs.values()):.2e} ({max(errs, key=errs.get)})")
    if compute == "f32":
        assert rel(X, Xo) < 1e-4
        assert abs(loss - lo) < 1e-5
        for name in go:
            assert errs[name] < 1e-4, (name, errs[name])
    else:
        assert rel(X, Xo) < 1e-3
        assert abs(loss - lo) < 1e-4
        for name in go:
            assert errs[name] < 1e-2, (name, errs[name])


def test_adam_step_matches_oracle(fe):
    A, rp, ci, z, V = case(fe, n=3000, seed=11)
    net = fe.Gnn(seed=5)
    p0 = net.get_params().astype(np.float64)
    zt = torch.tensor(z, dtype=torch.float32, device="cuda")
    Vt = torch.tensor(V, dtype=torch.float32, device="cuda")
    _, g = net.backward(A, zt, Vt, want_grads=True)
    net.adam(1e-2)
    torch.cuda.synchronize()
    p1 = net.get_params().astype(np.float64)
    st = {}
    want = G.adam_step({"p": p0.copy()}, {"p": g.astype(np.float64)}, st, lr=1e-2)["p"]
    assert np.allclose(p1, want, rtol=1e-5, atol=1e-7)


def test_adam_clipped_step_matches_oracle(fe):
    A, rp, ci, z, V = case(fe, n=3000, seed=12)
    net = fe.Gnn(seed=6)
    p0 = net.get_params().astype(np.float64)
    zt = torch.tensor(z, dtype=torch.float32, device="cuda")
    Vt = torch.tensor(V, dtype=torch.float32, device="cuda")
    _, g = net.backward(A, zt, Vt, want_grads=True)
    clip = 0.1 * float(np.linalg.norm(g))  # active: scales the step's gradient by 0.1
    net.adam(1e-2, clip=clip)
    torch.cuda.synchronize()
    p1 = net.get_params().astype(np.float64)
    want = G.adam_step({"p": p0.copy()}, {"p": g.astype(np.float64)}, {}, lr=1e-2, clip=clip)["p"]
    assert np.allclose(p1, want, rtol=1e-5, atol=1e-7)
    with pytest.raises(fe.FeError):
        net.adam(1e-2, clip=-1.0)


def test_training_reduces_loss(fe):
    """A few Adam steps on one graph lower the loss (sanity of the whole loop)."""
    A, rp, ci, z, V = case(fe, n=4000, seed=13)
    # targets: the graph's own leading eigenvectors (FP64 solver)
    r = fe.fe_krylov_schur(A, 8, 8, 48, 1e-8, dtype=torch.float64, seed=1)
    Vt = r.evecs.float().contiguous()
    zt = torch.tensor(z, dtype=torch.float32, device="cuda")
    net = fe.Gnn(seed=1)
    l0, _ = net.backward(A, zt, Vt)
    for _ in range(60):
        net.backward(A, zt, Vt)
        net.adam(3e-3)
    l1, _ = net.backward(A, zt, Vt)
    assert l1 < l0 - 0.05, (l0, l1)


@pytest.mark.parametrize("block", [1, 2, 4])
def test_forward_folds_outputs_to_block(fe, block):
    """block < 8: column c is the sum of outputs c, c + block, ... (ascending)."""
    A, rp, ci, z, V = case(fe, n=3000, seed=14, relabel=True)
    net = fe.Gnn(seed=2)
    zt = torch.tensor(z, dtype=torch.float32, device="cuda")
    X8 = net.forward(A, zt)
    Xb = net.forward(A, zt, block=block)
    assert Xb.shape == (A.n, block)
    want = X8[:, 0:block].clone()
    for j in range(block, 8, block):
        want += X8[:, j:j + block]
    assert torch.equal(Xb, want)
    with pytest.raises(fe.FeError):
        net.forward(A, zt, block=3)
