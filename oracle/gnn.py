"""Learned start block: a small graph network, FP64 oracle (forward, loss, backward).

The paper has no learned component; this follows the documented reading of
the learned warm start.  Per vertex i the input is
    h0_i = [log(1 + deg_i), z_i1 .. z_i15]     (z ~ N(0,1), drawn per graph)
and three aggregation layers with hidden width 64 compute
    S_l = Ahat H_{l-1},   Ahat = D^-1/2 A D^-1/2 (isolated vertices scaled by 0)
    Z_l = S_l W_l + H_{l-1} U_l + beta_l,   H_l = relu(Z_l)
followed by the output X = H_3 P (64 -> 8 columns, the start block).

Loss against the solver's eigenvectors V (n x k, orthonormal, k = 8): the
subspace misalignment
    L = 1 - ||V^T Q||_F^2 / k,   Q = X (X^T X)^-1/2,
  = 1 - tr(M G^-1 M^T) / k,      G = X^T X,  M = V^T X,
which is invariant to any invertible right factor of X (only span(X)
matters, as for a Krylov start block).  Its gradient is
    dL/dX = -(2/k) (V M G^-1 - X G^-1 M^T M G^-1).
"""
from __future__ import annotations

import numpy as np

from .ops import spmm

HIDDEN = 64
IN_DIM = 16
OUT_DIM = 8
LAYERS = 3


def param_shapes():
    shapes = {}
    d = IN_DIM
    for l in range(LAYERS):
        shapes[f"W{l}"] = (d, HIDDEN)
        shapes[f"U{l}"] = (d, HIDDEN)
        shapes[f"b{l}"] = (HIDDEN,)
        d = HIDDEN
    shapes["P"] = (HIDDEN, OUT_DIM)
    return shapes


def inv_sqrt_degree(row_ptr: np.ndarray) -> np.ndarray:
    deg = np.diff(row_ptr).astype(np.float64)
    out = np.zeros_like(deg)
    nz = deg > 0
    out[nz] = 1.0 / np.sqrt(deg[nz])
    return out


def features(row_ptr: np.ndarray, z: np.ndarray) -> np.ndarray:
    """[log(1 + deg), z] with z an (n, 15) block of N(0,1) draws."""
    deg = np.diff(row_ptr).astype(np.float64)
    return np.concatenate([np.log1p(deg)[:, None], z], axis=1)


def ahat(row_ptr, col_idx, dinv, H):
    return dinv[:, None] * spmm(row_ptr, col_idx, dinv[:, None] * H)


def forward(row_ptr, col_idx, H0, params, transform_inputs=None):
    """transform_inputs: None (exact), or a rounding function applied to the
    operands of each layer's dense transform (S, H and the weights W, U) as
    they enter it: the reading of the network's BF16 storage (BF16 operands,
    wider accumulation; the bias, the output projection and the cached
    activations stay unrounded)."""
    rnd = transform_inputs if transform_inputs is not None else (lambda x: x)
    dinv = inv_sqrt_degree(row_ptr)
    H = H0
    cache = {"dinv": dinv, "H": [H0], "S": [], "Z": []}
    for l in range(LAYERS):
        S = ahat(row_ptr, col_idx, dinv, H)
        Z = rnd(S) @ rnd(params[f"W{l}"]) + rnd(H) @ rnd(params[f"U{l}"]) + params[f"b{l}"]
        H = np.maximum(Z, 0.0)
        cache["S"].append(S)
        cache["Z"].append(Z)
        cache["H"].append(H)
    X = H @ params["P"]
    return X, cache


def loss(X: np.ndarray, V: np.ndarray) -> float:
    k = V.shape[1]
    G = X.T @ X
    M = V.T @ X
    return float(1.0 - np.trace(M @ np.linalg.solve(G, M.T)) / k)


def loss_grad(X: np.ndarray, V: np.ndarray) -> np.ndarray:
    k = V.shape[1]
    G = X.T @ X
    M = V.T @ X
    Gi = np.linalg.inv(G)
    return -(2.0 / k) * (V @ (M @ Gi) - X @ (Gi @ M.T @ M @ Gi))


def backward(row_ptr, col_idx, params, cache, dX):
    grads = {}
    dinv = cache["dinv"]
    H3 = cache["H"][LAYERS]
    grads["P"] = H3.T @ dX
    dH = dX @ params["P"].T
    for l in reversed(range(LAYERS)):
        Z, S, Hin = cache["Z"][l], cache["S"][l], cache["H"][l]
        dZ = dH * (Z > 0)
        grads[f"W{l}"] = S.T @ dZ
        grads[f"U{l}"] = Hin.T @ dZ
        grads[f"b{l}"] = dZ.sum(axis=0)
        dS = dZ @ params[f"W{l}"].T
        dH = dZ @ params[f"U{l}"].T + ahat(row_ptr, col_idx, dinv, dS)  # Ahat is symmetric
    return grads


def init_params(seed: int = 0, scale: float = 1.0):
    """Glorot-style uniform initialisation (deterministic per seed)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in param_shapes().items():
        if len(shp) == 1:
            p[name] = np.zeros(shp)
        else:
            lim = scale * np.sqrt(6.0 / (shp[0] + shp[1]))
            p[name] = rng.uniform(-lim, lim, size=shp)
    return p


def adam_step(params, grads, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, clip=0.0):
    """One Adam update (Kingma & Ba 2015) with bias correction.

    clip > 0: the gradients are first scaled by min(1, clip / ||g||), ||g||
    the 2-norm over all tensors together (global-norm clipping, Pascanu et
    al. 2013).
    """
    t = state.get("t", 0) + 1
    state["t"] = t
    if clip > 0:
        norm = np.sqrt(sum(float(np.sum(np.square(g))) for g in grads.values()))
        scale = min(1.0, clip / norm) if norm > 0 else 1.0
        grads = {k: g * scale for k, g in grads.items()}
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1 - beta1) * grads[k]
        v[...] = beta2 * v + (1 - beta2) * grads[k] ** 2
        mhat = m / (1 - beta1 ** t)
        vhat = v / (1 - beta2 ** t)
        params[k] = params[k] - lr * mhat / (np.sqrt(vhat) + eps)
    return params
