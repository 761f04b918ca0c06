"""Learned start block: training and evaluation driver (runs on the GPU).

Training data: graphs from fe_synth.learned_start_graph, labelled with the
eigenvectors of the 8 largest-magnitude eigenvalues computed by the plain
solver in FP64 (block 8, subspace 48, tol 1e-8).  Training: one graph per
step, Adam, loss = subspace misalignment (fe.h).  Evaluation: on held-out
graphs, the sparse-product count and wall time (network inference included)
of a solve started from the network's block against random starts.

Fallback: the learned solve reverts to a random start when the network's
output is not finite or its Gram matrix is numerically singular.

    python -m paper_1602_01421_amd.learned train --graphs 400 --epochs 10 --out W.npy
    python -m paper_1602_01421_amd.learned eval --weights W.npy --heldout 40
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                               "gnn_start.npy")


def _torch():
    import torch
    return torch


def build_graph(seed: int, max_log2n: int = 18):
    import fe_synth as S
    from . import fe as F
    n, s, d, desc = S.learned_start_graph(seed, max_log2n=max_log2n)
    A = F.fe_csr_build(n, s, d, F.FE_GRAPH_DEFAULT | F.FE_RELABEL_BY_DEGREE)
    z = _torch().tensor(S.learned_start_features(n, seed), dtype=_torch().float32, device="cuda")
    return A, z, desc


def label(A, seed: int = 1):
    """Eigenvectors of the 8 largest-magnitude eigenvalues (FP64 solve)."""
    from . import fe as F
    torch = _torch()
    r = F.fe_krylov_schur(A, 8, 8, 48, 1e-8, dtype=torch.float64, seed=seed)
    return r.evecs.float().contiguous(), r


def learned_start(net, A, z, dtype):
    """Start block from the network, or None when it must fall back to random."""
    torch = _torch()
    X = net.forward(A, z)
    if not torch.isfinite(X).all():
        return None
    G = (X.double().T @ X.double()).cpu().numpy()
    w = np.linalg.eigvalsh(G)
    if not (w[0] > 1e-10 * w[-1]):
        return None
    return X.to(dtype).contiguous()


def solve(A, start=None, seed=0, dtype=None, tol=1e-8):
    from . import fe as F
    torch = _torch()
    dtype = dtype or torch.float64
    return F.fe_krylov_schur(A, 8, 8, 48, tol, dtype=dtype, start=start, seed=seed,
                             want_vectors=False)


def train(args):
    from . import fe as F
    torch = _torch()
    net = F.Gnn(seed=args.init_seed)
    data = []
    t0 = time.time()
    for gi in range(args.graphs):
        seed = args.first_seed + gi
        A, z, desc = build_graph(seed, args.max_log2n)
        V, r = label(A)
        data.append((A, z, V))
        if gi % 50 == 0:
            print(f"[train] labelled {gi + 1}/{args.graphs}: {desc} products {r.spmm_calls} "
                  f"({time.time() - t0:.0f} s)", flush=True)
    history = []
    rng = np.random.default_rng(args.init_seed)
    for ep in range(args.epochs):
        order = rng.permutation(len(data))
        losses = []
        for i in order:
            A, z, V = data[i]
            loss, _ = net.backward(A, z, V)
            net.adam(args.lr)
            losses.append(loss)
        history.append(float(np.mean(losses)))
        print(f"[train] epoch {ep + 1}/{args.epochs}: mean loss {history[-1]:.4f} "
              f"({time.time() - t0:.0f} s)", flush=True)
    torch.cuda.synchronize()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, net.get_params())
    print(json.dumps({"train_loss": history, "graphs": args.graphs, "epochs": args.epochs,
                      "seconds": time.time() - t0}), flush=True)


def evaluate(weights, heldout, first_seed=3000, max_log2n=18, random_seeds=3, log=print):
    """Learned vs random start on held-out graphs (FP64 storage, tol 1e-8)."""
    from . import fe as F
    torch = _torch()
    net = F.Gnn(seed=0)
    net.set_params(np.load(weights))
    rows = []
    for gi in range(heldout):
        seed = first_seed + gi
        A, z, desc = build_graph(seed, max_log2n)
        rand, t_rand = [], []
        for k in range(random_seeds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rand.append(solve(A, seed=100 + k))
            torch.cuda.synchronize()
            t_rand.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X = learned_start(net, A, z, torch.float64)
        r = solve(A, start=X, seed=1)
        torch.cuda.synchronize()
        t_learned = time.perf_counter() - t0
        row = {"graph": desc, "fallback": X is None,
               "learned_spmm": r.spmm_calls, "learned_s": t_learned,
               "random_spmm": float(np.median([q.spmm_calls for q in rand])),
               "random_s": float(np.median(t_rand)),
               "learned_ok": r.status == F.FE_OK}
        rows.append(row)
        log(f"[eval] {desc}: learned {row['learned_spmm']} products {t_learned*1e3:.1f} ms, "
            f"random {row['random_spmm']:.0f} products {row['random_s']*1e3:.1f} ms")
    ratio_spmm = [r["learned_spmm"] / r["random_spmm"] for r in rows]
    ratio_t = [r["learned_s"] / r["random_s"] for r in rows]
    summary = {"heldout": heldout, "median_spmm_ratio": float(np.median(ratio_spmm)),
               "median_time_ratio": float(np.median(ratio_t)),
               "frac_improved_spmm": float(np.mean([x < 1 for x in ratio_spmm])),
               "fallbacks": int(sum(r["fallback"] for r in rows)), "rows": rows}
    return summary


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--graphs", type=int, default=2000)
    t.add_argument("--first-seed", type=int, default=1000)
    t.add_argument("--epochs", type=int, default=20)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--init-seed", type=int, default=0)
    t.add_argument("--max-log2n", type=int, default=18)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--heldout", type=int, default=200)
    e.add_argument("--max-log2n", type=int, default=18)
    args = ap.parse_args()
    _torch().cuda.set_device(0)
    if args.cmd == "train":
        train(args)
    else:
        s = evaluate(args.weights, args.heldout, max_log2n=args.max_log2n)
        print(json.dumps({k: v for k, v in s.items() if k != "rows"}), flush=True)


if __name__ == "__main__":
    main()
