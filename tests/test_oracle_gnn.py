"""Pins for the learned-start network's FP64 oracle (no GPU).

Nothing in the paper fixes this network; it is pinned by central finite
differences, the loss's exact invariances (L depends on span(X) only, L(V) = 0),
permutation equivariance and Adam's closed-form behaviour on a constant
gradient.  What the trained network is worth is not pinned (see the gain test).
"""
import numpy as np
import pytest

import fe_synth as S
import oracle as O
from oracle import gnn as G


def small_graph(n=80, seed=4):
    n, s, d = S.chung_lu_edges(n, alpha=2.3, mean_deg=6, seed=seed)
    rp, ci = O.csr_from_edges(n, s, d)
    return n, rp, ci


def setup(seed=1, n=80):
    n, rp, ci = small_graph(n)
    z = S.normal((n, 15), seed=seed)
    H0 = G.features(rp, z)
    params = G.init_params(seed, scale=2.0)
    for l in range(G.LAYERS):
        params[f"b{l}"] = 0.1 * S.normal((G.HIDDEN,), seed=seed + 10 + l)
    V, _ = np.linalg.qr(S.normal((n, 8), seed=seed + 3))
    return n, rp, ci, H0, params, V


def total_loss(rp, ci, H0, params, V):
    X, _ = G.forward(rp, ci, H0, params)
    return G.loss(X, V)


def test_loss_invariances():
    rng = np.random.default_rng(0)
    V, _ = np.linalg.qr(rng.standard_normal((50, 8)))
    X = rng.standard_normal((50, 8))
    Q = rng.standard_normal((8, 8)) + 3 * np.eye(8)
    assert abs(G.loss(X, V) - G.loss(X @ Q, V)) < 1e-12
    assert abs(G.loss(V, V)) < 1e-13
    assert abs(G.loss(V @ Q, V)) < 1e-12
    assert 0.0 <= G.loss(X, V) <= 1.0
    W, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    Vperp = W[:, :8] - V @ (V.T @ W[:, :8])
    assert abs(G.loss(Vperp, V) - 1.0) < 1e-12  # orthogonal span -> loss 1


def test_loss_grad_finite_differences():
    rng = np.random.default_rng(1)
    V, _ = np.linalg.qr(rng.standard_normal((30, 8)))
    X = rng.standard_normal((30, 8))
    g = G.loss_grad(X, V)
    h = 1e-6
    for _ in range(20):
        i, j = rng.integers(30), rng.integers(8)
        Xp, Xm = X.copy(), X.copy()
        Xp[i, j] += h
        Xm[i, j] -= h
        fd = (G.loss(Xp, V) - G.loss(Xm, V)) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * max(1.0, abs(fd))


def test_backward_finite_differences():
    n, rp, ci, H0, params, V = setup()
    X, cache = G.forward(rp, ci, H0, params)
    grads = G.backward(rp, ci, params, cache, G.loss_grad(X, V))
    rng = np.random.default_rng(2)
    h = 1e-6
    for name, arr in params.items():
        for _ in range(4):
            idx = tuple(rng.integers(s) for s in arr.shape)
            p2 = {k: v.copy() for k, v in params.items()}
            p2[name][idx] += h
            lp = total_loss(rp, ci, H0, p2, V)
            p2[name][idx] -= 2 * h
            lm = total_loss(rp, ci, H0, p2, V)
            fd = (lp - lm) / (2 * h)
            an = grads[name][idx]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (name, idx, fd, an)


def test_forward_permutation_equivariance():
    n, s, d = S.chung_lu_edges(120, alpha=2.3, mean_deg=6, seed=7)
    rp, ci = O.csr_from_edges(n, s, d)
    z = S.normal((n, 15), seed=8)
    params = G.init_params(3)
    X, _ = G.forward(rp, ci, G.features(rp, z), params)
    p = S.permutation(n, 5)  # new vertex p[v] for old v
    rp2, ci2 = O.csr_from_edges(n, p[s], p[d])
    z2 = np.empty_like(z)
    z2[p] = z
    X2, _ = G.forward(rp2, ci2, G.features(rp2, z2), params)
    assert np.allclose(X2[p], X, rtol=1e-12, atol=1e-12)


def test_isolated_vertices_get_zero_aggregation():
    n = 10
    rp, ci = O.csr_from_edges(n, np.array([0, 1]), np.array([1, 2]))
    dinv = G.inv_sqrt_degree(rp)
    assert np.all(dinv[3:] == 0) and np.allclose(dinv[:3], [1, 1 / np.sqrt(2), 1])
    H = np.ones((n, 4))
    S_ = G.ahat(rp, ci, dinv, H)
    assert np.all(S_[3:] == 0)


def test_adam_constant_gradient():
    p = {"w": np.zeros(5)}
    g = {"w": np.array([1.0, -2.0, 0.5, 3.0, -0.1])}
    st = {}
    for t in range(10):
        p = G.adam_step(p, g, st, lr=0.01)
    # bias-corrected Adam on a constant gradient moves by lr * sign(g) each step
    assert np.allclose(p["w"], -0.1 * np.sign(g["w"]), rtol=1e-6)


def test_adam_global_norm_clipping():
    g = {"a": np.array([3.0, 0.0]), "b": np.array([[4.0]])}  # global norm 5
    st = {}
    p = G.adam_step({"a": np.zeros(2), "b": np.zeros((1, 1))}, g, st, lr=0.01, clip=1.0)
    # first moment after one step: (1 - beta1) * g * clip / ||g||
    assert np.allclose(st["m_a"], 0.1 * np.array([0.6, 0.0]), rtol=1e-15)
    assert np.allclose(st["m_b"], 0.1 * np.array([[0.8]]), rtol=1e-15)
    assert np.allclose(st["v_b"], 0.001 * 0.64, rtol=1e-12)
    st2 = {}
    G.adam_step({"a": np.zeros(2), "b": np.zeros((1, 1))}, g, st2, lr=0.01, clip=10.0)
    assert np.allclose(st2["m_a"], 0.1 * g["a"], rtol=1e-15)  # norm below clip: unchanged


def test_forward_rounding_hook():
    """The rounding hook only touches the transforms' operands: identity
    rounding reproduces the exact forward, and BF16 rounding moves the output
    by about the BF16 unit roundoff, not more."""
    n, s, d = S.chung_lu_edges(600, alpha=2.2, mean_deg=8, seed=5)
    rp, ci = O.csr_from_edges(n, s, d)
    params = G.init_params(3)
    F = G.features(rp, S.normal((n, 15), seed=6))
    X0, c0 = G.forward(rp, ci, F, params)
    X1, c1 = G.forward(rp, ci, F, params, transform_inputs=lambda x: x)
    assert np.array_equal(X0, X1)
    Xb, cb = G.forward(rp, ci, F, params, transform_inputs=O.round_bf16)
    err = np.linalg.norm(Xb - X0) / np.linalg.norm(X0)
    assert 1e-5 < err < 3e-2
    assert np.array_equal(cb["H"][0], c0["H"][0]) and np.array_equal(cb["S"][0], c0["S"][0])
