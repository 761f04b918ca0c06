"""Learned start block: training and evaluation driver (runs on the GPU).

Training data: graphs from fe_synth.learned_start_graph, labelled with the
eigenvectors of the 8 largest-magnitude eigenvalues computed by the plain
solver in FP64 (block 8, subspace 48, tol 1e-8).  Training: one graph per
step, Adam, loss = subspace misalignment (fe.h).  Evaluation: on held-out
graphs, the sparse-product count and wall time (network inference included)
of a solve started from the network's block against random starts.

Fallback: the learned solve reverts to a random start when the network's
output is not finite or its Gram matrix is numerically singular (before the
solve), or when the worst wanted residual estimate has not fallen below its
first value within three restarts (inside the solve, through
fe_ks_opts.start_check).  The solver's default factor for that rule is
tenfold; on graphs whose wanted eigenvalues include a tight cluster the
worst estimate of any start stalls for many restarts, so a tenfold bar
discards good learned starts, and the learned path asks only for a decrease.

    python -m paper_1602_01421_amd.learned train --out W.npy      # the committed weights
    python -m paper_1602_01421_amd.learned eval --weights W.npy --heldout 200

Training runs the forward pass in FP32 (BF16-mode training diverged: the
subspace-loss gradient magnifies BF16 rounding); inference uses the BF16
forward with the trained FP32 weights.
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
# in-solve fallback of a learned start: abandon it when the worst residual
# estimate has not dropped START_DROP-fold within START_CHECK restarts
START_CHECK = 3
START_DROP = 1.0


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


def learned_start(net, A, z, dtype, block: int = 8):
    """Start block (n x block) from the network, or None when it must fall back
    to random.  block < 8 folds the network's 8 outputs (fe_gnn_forward).

    One FP64 Gram of the output decides: a non-finite entry, or a smallest
    eigenvalue below 1e-10 of the largest (numerically dependent columns),
    means fallback.
    """
    from . import fe as F
    X = net.forward(A, z, block=block)
    G = F.fe_gram(X.unsqueeze(0), X).cpu().numpy()
    if not np.all(np.isfinite(G)):
        return None
    w = np.linalg.eigvalsh(0.5 * (G + G.T))
    if not (w[0] > 1e-10 * w[-1]):
        return None
    return X if X.dtype == dtype else X.to(dtype).contiguous()


def solve(A, start=None, seed=0, dtype=None, tol=1e-8):
    from . import fe as F
    torch = _torch()
    dtype = dtype or torch.float64
    return F.fe_krylov_schur(A, 8, 8, 48, tol, dtype=dtype, start=start, seed=seed,
                             want_vectors=False, start_check=START_CHECK if start is not None else 0,
                             start_drop=START_DROP)


def _labelled(args, first_seed, count, t0, tag, budget):
    from . import fe as F
    data = []
    for gi in range(count):
        seed = first_seed + gi
        A, z, desc = build_graph(seed, args.max_log2n)
        V, r = label(A)
        if r.status != F.FE_OK:
            print(f"[train] skipped {tag} {desc}: label solve status {r.status}", flush=True)
            continue
        data.append((A, z, V))
        if gi % 50 == 0:
            print(f"[train] labelled {tag} {gi + 1}/{count}: {desc} products {r.spmm_calls} "
                  f"({time.time() - t0:.0f} s)", flush=True)
        if time.time() - t0 > budget:
            print(f"[train] label budget reached after {len(data)} {tag} graphs", flush=True)
            break
    return data


def val_loss(net, A, z, V):
    """Loss on one graph; 1 (the loss of an output orthogonal to V) when the
    output is rank deficient."""
    from . import fe as F
    try:
        return net.backward(A, z, V)[0]
    except F.FeError as e:
        if e.status != F.FE_EBREAKDOWN:
            raise
        return 1.0


def train(args):
    """Label the training and validation graphs, then run Adam epochs.

    Step size: cosine decay from lr to lr/20 over the planned steps; the
    gradients are clipped to global norm `clip`.  After every epoch the mean
    loss over the validation graphs is taken, and the weights with the lowest
    validation loss so far are written to args.out.  Labelling stops at
    label_budget seconds and the epochs at time_budget seconds (whole run).
    """
    from . import fe as F
    torch = _torch()
    net = F.Gnn(seed=args.init_seed, compute=args.compute)
    if args.init_weights:  # continue from trained weights (fresh Adam state)
        net.set_params(np.load(args.init_weights))
    t0 = time.time()
    val = _labelled(args, args.val_seed, args.val, t0, "validation", args.label_budget)
    data = _labelled(args, args.first_seed, args.graphs, t0, "training", args.label_budget)
    t_label = time.time() - t0
    history, val_hist = [], []
    rng = np.random.default_rng(args.init_seed)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    total_steps = max(1, args.epochs * len(data))
    step = 0
    skipped = 0
    best = float("inf")
    for ep in range(args.epochs):
        t_ep = time.time()
        order = rng.permutation(len(data))
        losses = []
        for i in order:
            A, z, V = data[i]
            lr = args.lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * step / total_steps)))
            step += 1
            try:
                loss, _ = net.backward(A, z, V)
            except F.FeError as e:  # rank-deficient output on this graph: no step
                if e.status != F.FE_EBREAKDOWN:
                    raise
                skipped += 1
                continue
            if np.isfinite(loss):
                net.adam(lr, clip=args.clip)
            losses.append(loss)
        history.append(float(np.nanmean(losses)))
        vl = float(np.mean([val_loss(net, A, z, V) for A, z, V in val])) if val else history[-1]
        val_hist.append(vl)
        if vl < best:
            best = vl
            np.save(args.out, net.get_params())
        print(f"[train] epoch {ep + 1}/{args.epochs}: mean loss {history[-1]:.4f} "
              f"validation {vl:.4f} (best {best:.4f}) ({time.time() - t0:.0f} s)", flush=True)
        if time.time() - t0 + (time.time() - t_ep) > args.time_budget:
            print("[train] time budget reached", flush=True)
            break
    torch.cuda.synchronize()
    print(json.dumps({"train_loss": history, "val_loss": val_hist, "best_val_loss": best,
                      "graphs": len(data), "val_graphs": len(val), "epochs": len(history),
                      "label_s": t_label, "seconds": time.time() - t0, "lr": args.lr,
                      "clip": args.clip, "compute": args.compute,
                      "init_weights": args.init_weights, "skipped_steps": skipped}),
          flush=True)


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
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        r = solve(A, start=X, seed=1)
        torch.cuda.synchronize()
        t_learned = time.perf_counter() - t0
        row = {"graph": desc, "fallback": X is None, "in_solve_fallback": r.start_fallback >= 0,
               "learned_spmm": r.spmm_calls, "learned_s": t_learned, "inference_s": t_inf,
               "random_spmm": float(np.median([q.spmm_calls for q in rand])),
               "random_s": float(np.median(t_rand)),
               "learned_ok": r.status == F.FE_OK,
               "random_ok": all(q.status == F.FE_OK for q in rand)}
        rows.append(row)
        log(f"[eval] {desc}: learned {row['learned_spmm']} products {t_learned*1e3:.1f} ms, "
            f"random {row['random_spmm']:.0f} products {row['random_s']*1e3:.1f} ms")
    def stats(sel):
        if not sel:
            return {}
        rs = [r["learned_spmm"] / r["random_spmm"] for r in sel]
        rt = [r["learned_s"] / r["random_s"] for r in sel]
        return {"graphs": len(sel), "median_spmm_ratio": float(np.median(rs)),
                "median_time_ratio": float(np.median(rt)),
                "total_spmm_ratio": float(sum(r["learned_spmm"] for r in sel)
                                          / sum(r["random_spmm"] for r in sel)),
                "total_time_ratio": float(sum(r["learned_s"] for r in sel)
                                          / sum(r["random_s"] for r in sel)),
                "frac_improved_spmm": float(np.mean([x < 1 for x in rs])),
                "median_inference_ms": 1e3 * float(np.median([r["inference_s"] for r in sel]))}
    # graphs where a solve hit the restart cap carry no time-to-tolerance
    ok = [r for r in rows if r["learned_ok"] and r["random_ok"]]
    summary = {"heldout": heldout, "both_converged": len(ok), **stats(ok),
               "chung_lu": stats([r for r in ok if r["graph"].startswith("chung_lu")]),
               "sbm": stats([r for r in ok if r["graph"].startswith("sbm")]),
               "fallbacks": int(sum(r["fallback"] for r in rows)),
               "in_solve_fallbacks": int(sum(r["in_solve_fallback"] for r in rows)),
               "learned_not_converged": int(sum(not r["learned_ok"] for r in rows)),
               "random_not_converged": int(sum(not r["random_ok"] for r in rows)), "rows": rows}
    return summary


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--graphs", type=int, default=2000)
    t.add_argument("--first-seed", type=int, default=1000)
    t.add_argument("--epochs", type=int, default=200)
    t.add_argument("--lr", type=float, default=5e-4)
    t.add_argument("--init-seed", type=int, default=0)
    t.add_argument("--max-log2n", type=int, default=18)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--compute", default="f32", choices=["bf16", "f32"],
                   help="training forward precision (inference runs BF16 either way)")
    t.add_argument("--clip", type=float, default=1.0, help="global gradient-norm clip (0: off)")
    t.add_argument("--val", type=int, default=100, help="validation graphs")
    t.add_argument("--val-seed", type=int, default=9000)
    t.add_argument("--init-weights", default=None, help="start from these weights")
    t.add_argument("--label-budget", type=float, default=300.0, help="seconds")
    t.add_argument("--time-budget", type=float, default=760.0, help="seconds, whole run")
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--heldout", type=int, default=200)
    e.add_argument("--max-log2n", type=int, default=18)
    e.add_argument("--first-seed", type=int, default=3000)
    e.add_argument("--rows", default=None, help="write the per-graph rows as JSON here")
    args = ap.parse_args()
    _torch().cuda.set_device(0)
    if args.cmd == "train":
        train(args)
    else:
        s = evaluate(args.weights, args.heldout, first_seed=args.first_seed,
                     max_log2n=args.max_log2n, log=lambda m: print(m, flush=True))
        if args.rows:
            with open(args.rows, "w") as f:
                json.dump(s, f, indent=1)
        print(json.dumps({k: v for k, v in s.items() if k != "rows"}), flush=True)


if __name__ == "__main__":
    main()
