"""Precision comparison and the one-GPU large-graph run (GPU; library calls only).

precision
    R-MAT graph (default scale 24, edge factor 16, a/b/c/d .57/.19/.19/.05),
    nev 8, block 8, m 64.  An FP64-storage solve (tol 1e-10) is the reference;
    then FP32 storage (tol 1e-6), BF16 storage (tol 1e-3: BF16 cannot hold a
    basis whose residuals reach 1e-6) and mixed BF16->FP32 storage (tol 1e-6).
    Per precision: largest eigenvalue error relative to the FP64 solve, the
    solver's own explicit FP64 residuals, products, restarts, wall time; plus
    the product alone at block 8 in FP32 and BF16.

large
    R-MAT scale 27 (134M vertices, ~4.2e9 stored nonzeros, int64 offsets),
    nev 8, for each solve shape in --configs (BLOCKxM, default 8x48): the
    product alone at the block width (FP32, median and 10th/90th percentile
    of --spmm-reps launches), an FP64-storage reference solve, the plain FP32
    solve from random starts, learned-start solves in FP32 and mixed storage
    (network inference on the GPU included in their end-to-end time; the
    network's random inputs drawn on the GPU) and a mixed-storage solve from
    a random start (--runs selects).

gnn
    The learned start network's calls at the largest training-graph size
    (Chung-Lu, n = 2^18, Pareto 2.1, mean degree 32): inference (BF16 and
    FP32 transforms), the training step (forward, loss, backward) and the
    Adam step, each timed with HIP events over repeated calls.

svd
    Directed R-MAT (default scale 27: the arcs of the same sample stream, not
    symmetrised; deduplicated, self-loops dropped; the paper's directed page
    graph is not available): the nsv largest singular values through
    Krylov-Schur on A^T A (fe_svds, handles of A and A^T), for each shape in
    --configs (BLOCKxM; the paper's SVD run used 2 vectors per block and a
    basis of 2 x block x nsv), an FP64-storage reference (tol 1e-10) and FP32
    storage (tol 1e-6); plus each product alone at the block width.

ops
    The dense subspace operations alone (the paper's dense-operation figure:
    n = 60M rows, block 4, subspace m = 4 .. 512): fe_gram (V^T W, the
    MvTransMv operation) and fe_block_update (W <- W + V C, MvTimesMatAddMv)
    per m in FP32 (and FP64 up to --f64-max-m), with the algorithmic bytes
    (n (m + b) s and n (m + 2 b) s), GB/s, the fraction of 8 TB/s and, for
    the Gram, FP64 MFMA TFLOP/s.

Each prints one JSON line; progress goes to stdout as the steps finish.

    python -m paper_1602_01421_amd.study precision --scale 24
    python -m paper_1602_01421_amd.study large --scale 27 --weights W.npy
    python -m paper_1602_01421_amd.study gnn
    python -m paper_1602_01421_amd.study svd --scale 27
    python -m paper_1602_01421_amd.study ops
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _log(msg):
    print(msg, flush=True)


def build_rmat(F, scale: int):
    import fe_synth as S
    t0 = time.perf_counter()
    n, s, d = S.rmat_edges(scale, seed=scale)
    t_gen = time.perf_counter() - t0
    _log(f"[study] generated R-MAT scale {scale}: {len(s)} samples in {t_gen:.1f} s")
    t0 = time.perf_counter()
    A = F.fe_csr_build(n, s, d, F.FE_GRAPH_DEFAULT | F.FE_RELABEL_BY_DEGREE)
    t_build = time.perf_counter() - t0
    del s, d
    gc.collect()
    _log(f"[study] CSR n={A.n} nnz={A.nnz} max_deg={A.max_deg} built in {t_build:.1f} s")
    return A, {"gen_s": t_gen, "build_s": t_build}


def time_spmm(F, A, b, dtype, reps=10):
    """One product at width b: 5 warm-up launches, then `reps` launches each
    bracketed by HIP events on the product's stream; the median, 10th and
    90th percentile durations (caches not flushed: X is gathered in steady
    state)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    X = torch.randn((A.n, b), generator=g, device="cuda", dtype=torch.float32).to(dtype)
    Y = torch.empty_like(X)
    st = torch.cuda.Stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    with torch.cuda.stream(st):
        for _ in range(5):
            F.fe_spmm(A, X, Y, stream=st)
        for e0, e1 in ev:
            e0.record(st)
            F.fe_spmm(A, X, Y, stream=st)
            e1.record(st)
    st.synchronize()
    ts = np.array([e0.elapsed_time(e1) / 1e3 for e0, e1 in ev])
    t = float(np.median(ts))
    es = X.element_size()
    algo = 4.0 * A.nnz + 8.0 * (A.n + 1) + 2.0 * A.n * b * es
    del X, Y
    return {"b": b, "dtype": str(dtype).replace("torch.", ""), "ms": t * 1e3,
            "ms_p10": float(np.percentile(ts, 10)) * 1e3,
            "ms_p90": float(np.percentile(ts, 90)) * 1e3, "reps": reps,
            "gedge_col_s": A.nnz * b / t / 1e9, "gbs": algo / t / 1e9,
            "frac": algo / t / 1e9 / HBM_PEAK_GBS}


VERBOSE = False


def run_solve(F, A, label, ref=None, **kw):
    import torch
    torch.cuda.synchronize()
    _log(f"[study] {label}: solving")
    t0 = time.perf_counter()
    r = F.fe_krylov_schur(A, want_vectors=False, verbose=VERBOSE, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    row = {"run": label, "status": int(r.status), "seconds": t, "restarts": r.restarts,
           "spmm_calls": r.spmm_calls, "spmm_calls_bf16": r.spmm_calls_low,
           "switch_restart": r.switch_restart, "refills": r.refills,
           "start_fallback": r.start_fallback,
           "max_resid": float(np.max(r.resid)), "evals": [float(x) for x in r.evals]}
    if ref is not None:
        row["max_eval_rel_err_vs_f64"] = float(np.max(np.abs(r.evals - ref) / np.abs(ref)))
    _log(f"[study] {label}: status {r.status} {t:.2f} s, {r.spmm_calls} products, "
         f"max resid {row['max_resid']:.2e}"
         + (f", eval err {row['max_eval_rel_err_vs_f64']:.2e}" if ref is not None else ""))
    return row, r


def precision(args):
    from . import fe as F
    import torch
    A, info = build_rmat(F, args.scale)
    nev, b, m = 8, args.block, args.m
    out = {"study": "precision", "graph": f"rmat{args.scale}", "n": A.n, "nnz": A.nnz,
           "nev": nev, "block": b, "m": m, **info}
    out["spmm"] = [time_spmm(F, A, b, torch.float32, reps=args.spmm_reps),
                   time_spmm(F, A, b, torch.bfloat16, reps=args.spmm_reps)]
    _log(f"[study] product b={b}: " + ", ".join(f"{x['dtype']} {x['ms']:.2f} ms" for x in out["spmm"]))
    ref_row, ref = run_solve(F, A, "f64", nev=nev, block=b, m=m, tol=1e-10,
                             dtype=torch.float64, seed=1)
    rows = [ref_row]
    rows.append(run_solve(F, A, "f32", ref.evals, nev=nev, block=b, m=m, tol=1e-6,
                          dtype=torch.float32, seed=1)[0])
    rows.append(run_solve(F, A, "bf16", ref.evals, nev=nev, block=b, m=m, tol=1e-3,
                          dtype=torch.bfloat16, seed=1, max_restarts=args.bf16_restarts)[0])
    rows.append(run_solve(F, A, "mixed_bf16_f32", ref.evals, nev=nev, block=b, m=m, tol=1e-6,
                          dtype=torch.float32, seed=1, mixed=True)[0])
    out["solves"] = rows
    print(json.dumps(out), flush=True)


def large(args):
    from . import fe as F
    import torch
    A, info = build_rmat(F, args.scale)
    out = {"study": "large", "graph": f"rmat{args.scale}", "n": A.n, "nnz": A.nnz,
           "max_deg": A.max_deg, **info, "spmm": [], "configs": []}
    shapes = [parse_shape(c) for c in args.configs.split(",")]
    for b in sorted({sh[0] for sh in shapes}):
        x = time_spmm(F, A, b, torch.float32, reps=args.spmm_reps)
        out["spmm"].append(x)
        _log(f"[study] product b={b} FP32: {x['ms']:.2f} ms, {x['gedge_col_s']:.0f} GEdge*col/s, "
             f"{x['gbs']:.0f} GB/s ({100 * x['frac']:.1f}% of 8 TB/s)")
    gc.collect()
    torch.cuda.empty_cache()
    for b, m, keep in shapes:
        out["configs"].append(large_config(F, A, args, 8, b, m, keep))
    print(json.dumps(out), flush=True)


def parse_shape(c):
    """BLOCKxM or BLOCKxMkKEEP (KEEP: Ritz vectors kept at a restart, 0 = the
    library's default)."""
    b, rest = c.split("x")
    m, _, keep = rest.partition("k")
    return int(b), int(m), int(keep or 0)


def large_config(F, A, args, nev, b, m, keep=0):
    """Solves of one shape.  With --seeds S: random starts from seeds 1..S and,
    for every weights file, S draws of the network's random inputs."""
    from .learned import START_CHECK, START_DROP, learned_start
    import functools
    import torch
    _log(f"[study] configuration nev {nev}, block {b}, m {m}, keep {keep or 'default'}")
    run_solve = functools.partial(_run_solve_keep, keep)
    mr = args.max_restarts
    runs = set(args.runs.split(","))
    seeds = list(range(1, max(1, args.seeds) + 1))
    rows, ref_evals = [], None
    if "f64" in runs:
        ref_row, ref = run_solve(F, A, "f64_reference", nev=nev, block=b, m=m, tol=1e-10,
                                 dtype=torch.float64, seed=2, max_restarts=mr)
        rows.append(ref_row)
        ref_evals = ref.evals
        torch.cuda.empty_cache()
    for mixed, tag in ((False, "f32"), (True, "mixed")):
        if tag not in runs:
            continue
        for sd in seeds:
            row, _ = run_solve(F, A, "f32_random_start" if not mixed else "random_start_mixed",
                               ref_evals, nev=nev, block=b, m=m, tol=1e-6, dtype=torch.float32,
                               seed=sd, mixed=mixed, max_restarts=mr)
            row["seed"] = sd
            rows.append(row)
            torch.cuda.empty_cache()
    weights = [w for w in (args.weights or "").split(",") if w]
    if b in (1, 2, 4, 8) and ("learned" in runs or "learned32" in runs):
        for wi, wpath in enumerate(weights):
            for sd in seeds:
                net = F.Gnn(seed=0, compute="bf16")
                net.set_params(np.load(wpath))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                g = torch.Generator(device="cuda")
                g.manual_seed(args.scale * 1000 + sd - 1 if sd > 1 else args.scale)
                z = torch.randn((A.n, 15), generator=g, device="cuda", dtype=torch.float32)
                X = learned_start(net, A, z, torch.float32, block=b)
                del z
                net.close()  # releases the inference workspace (4 x n x 64 floats)
                torch.cuda.synchronize()
                t_inf = time.perf_counter() - t0
                _log(f"[study] network inference {t_inf:.2f} s (weights {wi}, draw {sd}, "
                     f"fallback: {X is None})")
                for tag, mixed in (("learned", True), ("learned32", False)):
                    if tag not in runs:
                        continue
                    row, _ = run_solve(F, A, "learned_start_" + ("mixed" if mixed else "f32"),
                                       ref_evals, nev=nev, block=b, m=m, tol=1e-6,
                                       dtype=torch.float32, seed=1, start=X, mixed=mixed,
                                       max_restarts=mr,
                                       start_check=START_CHECK if X is not None else 0,
                                       start_drop=START_DROP)
                    row.update({"inference_s": t_inf, "end_to_end_s": t_inf + row["seconds"],
                                "fallback": X is None, "weights": wpath, "draw": sd})
                    rows.append(row)
                del X
                torch.cuda.empty_cache()
    return {"nev": nev, "block": b, "m": m, "keep": keep, "max_restarts": mr, "solves": rows}


def _run_solve_keep(keep, F, A, label, ref=None, **kw):
    return run_solve(F, A, label, ref, keep=keep, **kw)


def gnn(args):
    from . import fe as F
    import fe_synth as S
    import torch
    n = 1 << args.log2n
    _, s, d = S.chung_lu_edges(n, alpha=2.1, mean_deg=args.mean_deg, seed=1)
    A = F.fe_csr_build(n, s, d, F.FE_GRAPH_DEFAULT | F.FE_RELABEL_BY_DEGREE)
    _log(f"[study] Chung-Lu n={A.n} nnz={A.nnz} max_deg={A.max_deg}")
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    z = torch.randn((n, 15), generator=g, device="cuda", dtype=torch.float32)
    V, _ = torch.linalg.qr(torch.randn((n, 8), generator=g, device="cuda", dtype=torch.float64))
    V = V.float().contiguous()
    st = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"study": "gnn", "n": A.n, "nnz": A.nnz, "params": int(F.lib().fe_gnn_param_count())}
    for compute in ("bf16", "f32"):
        net = F.Gnn(seed=0, compute=compute)
        X = torch.empty((n, 8), device="cuda", dtype=torch.float32)
        row = {"forward_ms": timed(lambda: net.forward(A, z, X=X), args.reps),
               "train_step_ms": timed(lambda: net.backward(A, z, V), args.reps),
               "adam_ms": timed(lambda: net.adam(1e-4, clip=1.0), args.reps)}
        net.close()
        out[compute] = row
        _log(f"[study] gnn {compute}: forward {row['forward_ms']:.3f} ms, forward+loss+backward "
             f"{row['train_step_ms']:.3f} ms, Adam {row['adam_ms']:.3f} ms")
    print(json.dumps(out), flush=True)


def svd(args):
    from . import fe as F
    import torch
    import fe_synth as S
    t0 = time.perf_counter()
    n, s, d = S.rmat_edges(args.scale, seed=args.scale)
    t_gen = time.perf_counter() - t0
    _log(f"[study] generated R-MAT scale {args.scale}: {len(s)} arcs in {t_gen:.1f} s")
    directed = F.FE_DEDUPE | F.FE_DROP_SELF
    t0 = time.perf_counter()
    A = F.fe_csr_build(n, s, d, directed)
    At = F.fe_csr_build(n, d, s, directed)
    t_build = time.perf_counter() - t0
    del s, d
    gc.collect()
    _log(f"[study] A: n={A.n} nnz={A.nnz} max out-degree {A.max_deg}; A^T max in-degree "
         f"{At.max_deg} (both built in {t_build:.1f} s)")
    out = {"study": "svd", "scale": args.scale, "n": A.n, "nnz": A.nnz,
           "max_out_degree": A.max_deg, "max_in_degree": At.max_deg, "gen_s": t_gen,
           "build_s": t_build, "nsv": args.nsv, "configs": []}
    for cfg in args.configs.split(","):
        b, m = (int(x) for x in cfg.split("x"))
        rows = {"block": b, "m": m, "spmm_A": time_spmm(F, A, b, torch.float32),
                "spmm_At": time_spmm(F, At, b, torch.float32), "solves": []}
        ref = None
        for dt, tol in ((torch.float64, 1e-10), (torch.float32, 1e-6)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = F.fe_svds(A, At, args.nsv, b, m, tol, dtype=dt, seed=1, want_vectors=False,
                          max_restarts=args.max_restarts)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            row = {"storage": str(dt).replace("torch.", ""), "tol": tol, "status": int(r.status),
                   "seconds": t, "applications": r.spmm_calls, "restarts": r.restarts,
                   "max_resid": float(np.max(r.resid)), "svals": [float(x) for x in r.evals]}
            if ref is None:
                ref = r.evals
            else:
                row["max_sval_rel_err_vs_f64"] = float(np.max(np.abs(r.evals - ref) / ref))
            rows["solves"].append(row)
            _log(f"[study] svd {b}x{m} {row['storage']}: status {r.status} {t:.2f} s, "
                 f"{r.spmm_calls} A^T A applications, max resid {row['max_resid']:.2e}, "
                 f"sigma_1 {r.evals[0]:.8g}")
        out["configs"].append(rows)
    print(json.dumps(out), flush=True)


def ops(args):
    """The tall-and-skinny operations alone at n rows, block width b, for basis
    sizes m (multiples of b): Gram V^T W, the block update W - V C (at b = 8
    and 16 the MFMA contraction) and, at b = 4, 8 and 16 with m + b <= 128
    (m <= 96 at b = 8 in FP64), the fused CGS2 middle step (W - V C and
    [V W]^T W in one pass)."""
    from . import fe as F
    import torch
    n, b = args.n, args.b
    out = {"study": "ops", "n": n, "b": b, "rows": []}
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    for dt in (torch.float32, torch.float64):
        es = torch.tensor([], dtype=dt).element_size()
        for m in [int(x) for x in args.ms.split(",")]:
            if (dt == torch.float64 and m > args.f64_max_m) or m % b:
                continue
            nblk = m // b
            V = torch.randn((nblk, n, b), generator=g, device="cuda", dtype=torch.float32).to(dt)
            W = torch.randn((n, b), generator=g, device="cuda", dtype=torch.float32).to(dt)
            C = torch.randn((m, b), generator=g, device="cuda", dtype=torch.float64) * 1e-3
            G = torch.empty((m + b, b), dtype=torch.float64, device="cuda")
            res = {"dtype": str(dt).replace("torch.", ""), "m": m}
            cases = [("gram", lambda: F.fe_gram(V, W, C=G[:m]), n * (m + b) * es, 2.0 * n * m * b),
                     ("update", lambda: F.fe_block_update(W, V, C), n * (m + 2 * b) * es,
                      2.0 * n * m * b)]
            if b in (4, 8, 16) and m + b <= 128 and not (b == 8 and es == 8 and m > 96):
                cases.append(("cgs_mid", lambda: F.fe_block_update_gram(W, V, C, Cout=G),
                              n * (m + 2 * b) * es, 2.0 * n * (2 * m + b) * b))
            for name, fn, byts, flops in cases:
                for _ in range(3):
                    fn()
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(args.reps)]
                for e0, e1 in ev:
                    e0.record()
                    fn()
                    e1.record()
                torch.cuda.synchronize()
                t = float(np.median([e0.elapsed_time(e1) / 1e3 for e0, e1 in ev]))
                res[name] = {"ms": t * 1e3, "gbs": byts / t / 1e9,
                             "frac": byts / t / 1e9 / HBM_PEAK_GBS, "tflops": flops / t / 1e12}
            out["rows"].append(res)
            _log(f"[study] ops {res['dtype']} b={b} m={m:3d}: " + ", ".join(
                f"{k} {v['ms']:8.2f} ms {v['gbs']:6.0f} GB/s ({100 * v['frac']:.0f}%) "
                f"{v['tflops']:5.1f} TFLOP/s" for k, v in res.items() if isinstance(v, dict)))
            del V, W, C, G
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def gathers(args):
    """The product's gather ceiling on R-MAT: the product, its gathers alone in
    storage order, and the hub rows' gathers (degree > --hub) re-ordered column
    band by column band (row order kept within a band), for band widths of
    2^shift columns: whether visiting the matrix tile by tile, so that each
    band's slice of X stays in cache, would make the gathers cheaper."""
    from . import fe as F
    import torch
    A, info = build_rmat(F, args.scale)
    n, nnz, b = A.n, A.nnz, args.b
    X = torch.randn((n, b), device="cuda", dtype=torch.float32)
    Y = torch.empty_like(X)
    out = torch.empty(F.lib().fe_spmm_gather_bound_sets(), dtype=torch.float64, device="cuda")

    def tm(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for e0, e1 in ev:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))

    res = {"study": "gathers", "graph": f"rmat{args.scale}", "n": n, "nnz": nnz, "b": b, **info,
           "product_ms": tm(lambda: F.fe_spmm(A, X, Y)),
           "gathers_storage_order_ms": tm(lambda: F.fe_spmm_gather_bound(A, X, out))}
    _log(f"[study] product {res['product_ms']:.2f} ms, its gathers alone "
         f"{res['gathers_storage_order_ms']:.2f} ms")
    rp, ci = A.export()
    A.close()
    del Y
    deg = np.diff(rp)
    hubs = int((deg > args.hub).sum())
    eh = int(rp[hubs])
    hub = torch.from_numpy(ci[:eh]).cuda()
    rest = torch.from_numpy(ci[eh:]).cuda()
    del ci, rp
    res.update({"hub_degree": args.hub, "hub_rows": hubs, "hub_nonzeros": eh,
                "hub_row_order_ms": tm(lambda: F.fe_gather_rows(hub, X, out)),
                "other_rows_ms": tm(lambda: F.fe_gather_rows(rest, X, out)), "bands": []})
    _log(f"[study] hub rows ({hubs}, {eh / nnz:.3f} of the nonzeros): {res['hub_row_order_ms']:.2f} ms;"
         f" the others {res['other_rows_ms']:.2f} ms")
    del rest
    # the same number of gathers from uniformly random rows, and from one row
    # (every gather a cache hit): the memory system's ends for this row size
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    idx = torch.randint(0, n, (nnz,), generator=g, device="cuda", dtype=torch.int32)
    res["uniform_random_ms"] = tm(lambda: F.fe_gather_rows(idx, X, out))
    idx.zero_()
    res["one_row_ms"] = tm(lambda: F.fe_gather_rows(idx, X, out))
    del idx
    torch.cuda.empty_cache()
    _log(f"[study] {nnz} gathers from uniformly random rows {res['uniform_random_ms']:.2f} ms, "
         f"from one row {res['one_row_ms']:.2f} ms")
    chunks = [hub[i:i + (1 << 30)] for i in range(0, hub.numel(), 1 << 30)]
    for shift in [int(x) for x in args.shifts.split(",")]:
        nb = (n + (1 << shift) - 1) >> shift
        keys = [c >> shift for c in chunks]
        parts = [torch.masked_select(c, k == band) for band in range(nb) for c, k in zip(chunks, keys)]
        del keys
        banded = torch.cat(parts)
        del parts
        t = tm(lambda: F.fe_gather_rows(banded, X, out))
        del banded
        torch.cuda.empty_cache()
        mib = (1 << shift) * b * 4 / 2 ** 20
        res["bands"].append({"columns_per_band": 1 << shift, "bands": nb, "x_slice_mib": mib, "ms": t})
        _log(f"[study] hub rows band by band, {nb} bands of {1 << shift} columns "
             f"({mib:.0f} MiB of X each): {t:.2f} ms")
    print(json.dumps(res), flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    p = sub.add_parser("precision")
    p.add_argument("--scale", type=int, default=24)
    p.add_argument("--block", type=int, default=8)
    p.add_argument("--m", type=int, default=64)
    p.add_argument("--bf16-restarts", type=int, default=200)
    p.add_argument("--spmm-reps", type=int, default=50)
    q = sub.add_parser("large")
    q.add_argument("--scale", type=int, default=27)
    q.add_argument("--configs", default="8x48",
                   help="comma list of BLOCKxM[kKEEP] solve shapes, all nev 8 (e.g. 8x48,"
                        "4x64,8x48k16: KEEP Ritz vectors kept at each restart)")
    q.add_argument("--max-restarts", type=int, default=500)
    q.add_argument("--weights", default=None, help="comma list of learned-start weight files")
    q.add_argument("--seeds", type=int, default=1,
                   help="random starts 1..S and S draws of the network inputs per weights file")
    q.add_argument("--spmm-reps", type=int, default=10)
    q.add_argument("--runs", default="f64,f32,learned,learned32,mixed",
                   help="solves: f64 (reference), f32, learned (mixed storage), learned32, mixed")
    r = sub.add_parser("gnn")
    r.add_argument("--log2n", type=int, default=18)
    r.add_argument("--mean-deg", type=float, default=32.0)
    r.add_argument("--reps", type=int, default=20)
    v = sub.add_parser("svd")
    v.add_argument("--scale", type=int, default=27)
    v.add_argument("--nsv", type=int, default=8)
    v.add_argument("--configs", default="2x32,8x64",
                   help="comma list of BLOCKxM shapes (2x32: the paper's 2 vectors per block, "
                        "basis 2 x 2 x nsv)")
    v.add_argument("--max-restarts", type=int, default=500)
    o = sub.add_parser("ops")
    o.add_argument("--n", type=int, default=60_000_000)
    o.add_argument("--b", type=int, default=4, help="block width")
    o.add_argument("--ms", default="4,8,16,32,64,128,256,512")
    o.add_argument("--f64-max-m", type=int, default=256)
    o.add_argument("--reps", type=int, default=5)
    w = sub.add_parser("gathers")
    w.add_argument("--scale", type=int, default=27)
    w.add_argument("--b", type=int, default=16)
    w.add_argument("--hub", type=int, default=2048, help="hub rows: degree above this")
    w.add_argument("--shifts", default="24,22,20,18,16",
                   help="band widths as powers of two of columns")
    for sp in (p, q, r, v, o, w):
        sp.add_argument("--verbose", action="store_true",
                        help="one line per restart from the solver (stderr)")
    args = ap.parse_args()
    global VERBOSE
    VERBOSE = args.verbose
    import torch
    torch.cuda.set_device(0)
    {"precision": precision, "large": large, "gnn": gnn, "svd": svd, "ops": ops,
     "gathers": gathers}[args.cmd](args)


if __name__ == "__main__":
    main()
