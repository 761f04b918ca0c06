"""Benchmark: block Krylov-Schur hot path on one MI355X.

Workload (default): R-MAT scale 27 (134,217,728 vertices, edge factor 16,
a/b/c/d = .57/.19/.19/.05, seed 27), symmetrised, deduplicated, self-loops
dropped: a 0/1 pattern CSR of 4.2e9 stored nonzeros with 64-bit offsets,
relabelled by degree -- one GPU's share at real shape.  One step = one full
block Krylov-Schur solve for the 8 largest-magnitude eigenpairs, FP32
storage, tol 1e-6, random start, block 16, subspace 112 (every row of the hot
path: sparse products, CGS2 Gram/updates, block QR, Rayleigh-Ritz, restarts
and the FP64 final check).  The configured block 8 / subspace 48 does not
converge on this graph in 500 restarts (three eigenvalues within 2e-4 of
each other); block 16 / 112 is the fastest converging shape measured.

value = sparse work of the solve (nnz x columns multiplied) / solve time,
in GEdge*col/s.  The JSON line also carries the product alone at the solve's
width and the sweep over widths 1..16 (FP32) at scale 27 and at scale 22,
the roofline of the dominant kernel, the time to 8 eigenpairs from the
learned start block against random starts, and the CPU oracle timed on a
bounded sample of the same workload, on all host cores and on one.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "SpMM GEdge·col/s & % HBM roofline; time-to-8-eigs learned vs random start"


PROFILE = os.path.join(ROOT, "profiles", "spmm_rmat27_b16_f32.md")


def measured_traffic(kernel: str):
    """HBM traffic per launch of the dominant kernel from the committed
    rocprofv3 summary (FETCH_SIZE + WRITE_SIZE), or None when the summary is
    missing or the kernel source changed since the counters were taken."""
    import hashlib
    import re
    if kernel != "spmm" or not os.path.exists(PROFILE):
        return None
    text = open(PROFILE).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    h = re.search(r"spmm_source_sha256_16:\s*([0-9a-f]+)", text)
    if not m or not h:
        return None
    src = os.path.join(ROOT, "paper_1602_01421_amd", "csrc", "spmm.hip")
    cur = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    return float(m.group(1)) if cur == h.group(1) else None


def counter_calibration_copy():
    """A plain 1 GiB device copy from a source evicted from the caches, so a
    FETCH_SIZE/WRITE_SIZE profile of this script can scale the counters; then
    five more copies timed with HIP events: the measured streaming bandwidth
    (bytes read + written per second, median), the practical ceiling beside
    the 8 TB/s datasheet peak; then a 1 GiB permutation gather for the same
    scaling on random line-sized reads."""
    import numpy as np
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    flush.add_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    times = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    del src, flush, dst
    # a permutation gather of known bytes: 2^23 rows of 128 bytes (one cache
    # line each) read once in random order, so FETCH_SIZE can be scaled for
    # gathers as well as for streams
    rows = torch.ones((1 << 23, 32), dtype=torch.float32, device="cuda")
    perm = torch.randperm(1 << 23, device="cuda")
    flush = torch.zeros(1 << 28, dtype=torch.float32, device="cuda")
    flush.add_(1.0)
    gathered = rows.index_select(0, perm)
    torch.cuda.synchronize()
    del rows, perm, flush, gathered
    return 2.0 * (1 << 30) / float(np.median(times)) / 1e9


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def spmm_bytes(n, nnz, b, s):
    return 4.0 * nnz + 8.0 * (n + 1) + 2.0 * n * b * s


def time_spmm(P, A, b, dtype, stream, reps):
    """Per-launch durations (s) of `reps` products after 5 warm-up launches,
    each bracketed by HIP events on the product's stream."""
    import torch
    X = torch.randn((A.n, b), device="cuda", dtype=torch.float32).to(dtype)
    Y = torch.empty_like(X)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    with torch.cuda.stream(stream):
        for _ in range(5):
            P.fe_spmm(A, X, Y, stream=stream)
        for e0, e1 in ev:
            e0.record(stream)
            P.fe_spmm(A, X, Y, stream=stream)
            e1.record(stream)
    ev[-1][1].synchronize()
    return [e0.elapsed_time(e1) * 1e-3 for e0, e1 in ev]


def time_gather_bound(P, A, b, dtype, stream, reps):
    """Per-launch durations (s) of the product's gathers alone (no rows):
    fe_spmm_gather_bound on the same matrix and width, timed like time_spmm."""
    import torch
    X = torch.randn((A.n, b), device="cuda", dtype=torch.float32).to(dtype)
    out = torch.empty(P.lib().fe_spmm_gather_bound_sets(), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    with torch.cuda.stream(stream):
        for _ in range(3):
            P.fe_spmm_gather_bound(A, X, out, stream=stream)
        for e0, e1 in ev:
            e0.record(stream)
            P.fe_spmm_gather_bound(A, X, out, stream=stream)
            e1.record(stream)
    ev[-1][1].synchronize()
    return [e0.elapsed_time(e1) * 1e-3 for e0, e1 in ev]


def host_info():
    import platform
    import subprocess
    info = {"nproc": os.cpu_count(), "machine": platform.machine()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Socket(s)",
                             "CPU max MHz", "NUMA node(s)"):
                info[k.strip()] = v.strip()
    except Exception:
        pass
    try:
        info["sched_affinity"] = len(os.sched_getaffinity(0))
    except Exception:
        pass
    return info


def cpu_baseline(n, s, d, block, m, budget_s=12.0):
    """The oracle as it stands, on this host's cores and on one core: one
    expansion step of the same solve restricted to a bounded sample of rows
    (a contiguous range of original vertex ids, which the generator's random
    relabel makes a uniform sample): the FP64 product of those rows with a
    full n x block X, then CGS2 of the sample rows against an m-column basis
    (two Grams, two updates).  Rows are added until the step takes about
    `budget_s` seconds.  The oracle's CSR build is not timed."""
    import numpy as np
    import fe_synth as S
    import oracle as O
    from oracle.krylov_schur import _cgs2
    threads = max(1, min(len(os.sched_getaffinity(0)), O.max_threads()))
    t0 = time.time()
    rp, ci = O.csr_build(n, s, d, threads=threads)
    t_csr = time.time() - t0
    X = S.normal((n, block), seed=3)

    def step(rows, th):
        sub = rp[: rows + 1]
        Vs = S.normal((rows, m), seed=4)
        t = time.perf_counter()
        W = _rows_spmm(O, sub, ci, X, th)
        t_spmm = time.perf_counter() - t
        _cgs2(Vs, W)
        return time.perf_counter() - t, int(sub[-1]), t_spmm

    out = {}
    for label, th in (("all", threads), ("one", 1)):
        rows = 1 << 14
        t, e, ts = step(rows, th)
        while t < budget_s / 4 and rows < n:
            rows = min(n, int(rows * max(2.0, budget_s / max(t, 1e-3) / 2)))
            t, e, ts = step(rows, th)
        out[label] = {"threads": th, "rows": rows, "nnz": e, "s": t,
                      "gedge_col_s": e * block / t / 1e9, "spmm_gedge_col_s": e * block / ts / 1e9}
    del X
    a, o = out["all"], out["one"]
    return {"value": a["gedge_col_s"], "unit": "GEdge·col/s", "cores": a["threads"],
            "kind": "oracle",
            "one_core": {"value": o["gedge_col_s"], "rows": o["rows"], "s": o["s"]},
            "spmm_only": {"all_cores": a["spmm_gedge_col_s"], "one_core": o["spmm_gedge_col_s"],
                          "note": "the product part of the same sample, timed alone"},
            "host": host_info(),
            "sample": f"one expansion step of the same solve on rows [0, {a['rows']}) of "
                      f"{n} ({a['nnz']} nonzeros): FP64 product with an n x {block} block, "
                      f"then CGS2 against {m} basis columns; {a['s']:.1f} s on {a['threads']} "
                      f"threads (one core: {o['rows']} rows, {o['s']:.1f} s); oracle CSR build "
                      f"{t_csr:.0f} s not timed"}


def _rows_spmm(O, sub_rp, ci, X, threads):
    """Rows [0, len(sub_rp) - 1) of A X with the oracle's product loop."""
    import numpy as np
    rows = sub_rp.shape[0] - 1
    Y = np.empty((rows, X.shape[1]))
    O.lib().oracle_spmm(rows, O.ptr(np.ascontiguousarray(sub_rp)), O.ptr(ci),
                        O.ptr(X), X.shape[1], O.ptr(Y), threads)
    return Y


def learned_vs_random(P, A, stream, weights, tol, block, m, seeds=3):
    """Time to 8 eigenpairs from the learned start block vs random starts.

    FP32 storage, nev 8 and tol as the timed steps, at its own shape (`block`
    <= 8, the network's width; for block < 8 its 8 outputs are folded to
    `block` columns).  Both legs run as a serving loop would: the network
    (weights and its inference workspace, about 1 KB per vertex) and the
    solver's workspace are allocated once, before timing, and reused.  The
    learned time is end to end otherwise: drawing the network's N(0,1) inputs
    on the GPU, inference, the fallback check and the solve.  (A solve that
    has to allocate its 70-80 GB subspace right after other large buffers
    were freed pays about 1.4 s for fresh device pages, whichever start it
    has; reusing a workspace takes that out of both legs.)
    """
    import numpy as np
    import torch
    from paper_1602_01421_amd.learned import START_CHECK, START_DROP, learned_start
    params = np.load(weights)
    wbytes = P.fe_ks_workspace_bytes(A, 8, block, m, dtype=torch.float32)
    ws = torch.empty(wbytes, dtype=torch.uint8, device="cuda")
    net = P.Gnn(seed=0, compute="bf16")
    net.set_params(params)

    def solve(start=None, seed=1):
        return P.fe_krylov_schur(A, 8, block, m, tol, dtype=torch.float32, start=start,
                                 seed=seed, stream=stream, want_vectors=False, workspace=ws,
                                 start_check=START_CHECK if start is not None else 0,
                                 start_drop=START_DROP)

    def infer(seed):
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        z = torch.randn((A.n, 15), generator=g, device="cuda", dtype=torch.float32)
        return learned_start(net, A, z, torch.float32, block=block)

    try:
        solve(seed=99)  # warm-up at this block width
        infer(99)  # sizes the network's workspace (result dropped)
        rand = []
        for k in range(seeds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = solve(seed=1 + k)
            torch.cuda.synchronize()
            rand.append((time.perf_counter() - t0, r.spmm_calls, r.status))
        learned = []
        for k in range(seeds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            X = infer(1 + k)
            torch.cuda.synchronize()
            t_inf = time.perf_counter() - t0
            r = solve(start=X, seed=1 + k)
            torch.cuda.synchronize()
            learned.append((time.perf_counter() - t0, r.spmm_calls, r.status, t_inf, X is None,
                            r.start_fallback >= 0))
            del X
    finally:
        net.close()
        del ws
        torch.cuda.empty_cache()
    med = lambda xs: float(np.median(xs))  # noqa: E731
    res = {"block": block, "m": m, "tol": tol, "dtype": "f32", "seeds": seeds,
           "workspaces": "network and solver workspaces allocated once, before timing",
           "random_s": med([x[0] for x in rand]), "random_spmm": med([x[1] for x in rand]),
           "learned_s": med([x[0] for x in learned]),
           "learned_spmm": med([x[1] for x in learned]),
           "inference_s": med([x[3] for x in learned]),
           "random_spmm_each": [int(x[1]) for x in rand],
           "learned_spmm_each": [int(x[1]) for x in learned],
           "fallbacks": int(sum(x[4] for x in learned)),
           "in_solve_fallbacks": int(sum(x[5] for x in learned)),
           "all_converged": all(x[2] == 0 for x in rand + learned)}
    res["time_ratio"] = res["learned_s"] / res["random_s"]
    res["spmm_ratio"] = res["learned_spmm"] / res["random_spmm"]
    log(f"time to 8 eigs (b={block}, m={m}, FP32): random {res['random_s']:.3f} s / "
        f"{res['random_spmm_each']} products, learned {res['learned_s']:.3f} s / "
        f"{res['learned_spmm_each']} products (inference {res['inference_s']*1e3:.1f} ms)")
    return res


def sweep_spmm(P, A, stream, widths, reps, stream_gbs, tag):
    import numpy as np
    import torch
    out = []
    for b in widths:
        ts = time_spmm(P, A, b, torch.float32, stream, reps)
        t = float(np.median(ts))
        by = spmm_bytes(A.n, A.nnz, b, 4)
        out.append({"b": b, "us": t * 1e6, "us_p10": float(np.percentile(ts, 10)) * 1e6,
                    "us_p90": float(np.percentile(ts, 90)) * 1e6, "reps": len(ts),
                    "gedge_col_s": A.nnz * b / t / 1e9, "gbs": by / t / 1e9,
                    "frac": by / t / 1e9 / HBM_PEAK_GBS,
                    "frac_of_stream": by / t / 1e9 / stream_gbs})
        log(f"{tag} spmm b={b:2d}: {t*1e6:9.1f} us  {A.nnz*b/t/1e9:8.1f} GEdge*col/s  "
            f"{by/t/1e9:7.1f} GB/s ({100*by/t/1e9/HBM_PEAK_GBS:.1f}% of HBM)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--scale", type=int, default=27)
    ap.add_argument("--block", type=int, default=16)
    ap.add_argument("--m", type=int, default=112)
    ap.add_argument("--mixed", action="store_true",
                    help="BF16 storage widened to FP32 when BF16 stalls (mixed-precision solve)")
    ap.add_argument("--sweep", default="1,2,4,8,16", help="SpMM-only widths (FP32)")
    ap.add_argument("--sweep-scale", type=int, default=22,
                    help="second graph for the SpMM-only sweep (0 to skip)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_1602_01421_amd", "weights",
                                                      "gnn_start.npy"),
                    help="learned start-block weights ('' to skip the comparison)")
    ap.add_argument("--learned-shape", default="8x120",
                    help="block x m of the learned-vs-random comparison (block <= 8)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--spmm-reps", type=int, default=10)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the path would "
              f"shard by row blocks: each GPU owning a row range of A, X and every subspace "
              f"block, one all-gather of X per product and one all-reduce per Gram)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import fe_synth as S
    import paper_1602_01421_amd as P

    P.lib()
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    stream_gbs = counter_calibration_copy()
    log(f"streaming copy: {stream_gbs:.0f} GB/s (read + write)")
    widths = [int(x) for x in args.sweep.split(",") if x]

    sweep2 = None
    if args.sweep_scale and args.sweep_scale != args.scale:
        n2, s2, d2 = S.rmat_edges(args.sweep_scale, seed=args.sweep_scale)
        A2 = P.fe_csr_build(n2, s2, d2, P.FE_GRAPH_DEFAULT | P.FE_RELABEL_BY_DEGREE)
        del s2, d2
        sweep2 = {"scale": args.sweep_scale, "n": A2.n, "nnz": A2.nnz,
                  "sweep": sweep_spmm(P, A2, stream, widths, 50, stream_gbs,
                                      f"scale {args.sweep_scale}")}
        A2.close()

    t0 = time.time()
    n, s, d = S.rmat_edges(args.scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=args.scale)
    t_gen = time.time() - t0
    log(f"R-MAT scale {args.scale}: {len(s)} samples ({t_gen:.1f} s)")
    t0 = time.time()
    A = P.fe_csr_build(n, s, d, P.FE_GRAPH_DEFAULT | P.FE_RELABEL_BY_DEGREE)
    t_build = time.time() - t0
    log(f"R-MAT scale {args.scale}: n={n} nnz={A.nnz} max_deg={A.max_deg} "
        f"(fe_csr_build {t_build:.1f} s)")

    sweep = sweep_spmm(P, A, stream, widths, args.spmm_reps, stream_gbs, f"scale {args.scale}")

    # whole-path steps: one solve each
    nev, block, m, tol = 8, args.block, args.m, 1e-6

    def solve(seed, profile=False):
        return P.fe_krylov_schur(A, nev, block, m, tol, dtype=torch.float32, seed=seed,
                                 stream=stream, want_vectors=True, profile=profile,
                                 mixed=args.mixed)

    for w in range(args.warmup):
        r = solve(100 + w)
        log(f"warmup solve: status {r.status} restarts {r.restarts} products {r.spmm_calls} "
            f"{r.t_total:.3f} s")
    torch.cuda.synchronize()
    times, cols, results = [], 0, []
    t_all0 = time.perf_counter()
    for k in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = solve(1 + k)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        cols += r.spmm_cols
        results.append(r)
        log(f"step {k}: {times[-1]:.3f} s  status {r.status} restarts {r.restarts} "
            f"products {r.spmm_calls} max resid {r.resid.max():.2e} lambda1 {r.evals[0]:.8g}")
        del r.evecs
    t_all = time.perf_counter() - t_all0
    value = A.nnz * cols / t_all / 1e9

    # per-kernel profile of one more solve (HIP events on the solve's stream)
    rp = solve(1, profile=True)
    del rp.evecs
    classes = {"spmm": (rp.t_spmm, rp.bytes_spmm, rp.spmm_calls),
               "gram": (rp.t_gram, rp.bytes_gram, rp.gram_calls),
               "update": (rp.t_update, rp.bytes_update, rp.update_calls)}
    dom = max(classes, key=lambda c: classes[c][0])
    t_dom, b_dom, calls_dom = classes[dom]
    achieved = b_dom / t_dom / 1e9
    log("profile: " + ", ".join(f"{c} {v[0]*1e3:.1f} ms / {v[2]} launches "
                                 f"({v[1]/max(v[0],1e-12)/1e9:.0f} GB/s)" for c, v in classes.items())
        + f", other {rp.t_other_dev*1e3:.1f} ms, host {rp.t_host*1e3:.1f} ms, total {rp.t_total*1e3:.1f} ms")
    default_cfg = args.scale == 27 and block == 16 and m == 112 and not args.mixed
    roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom) if default_cfg else None,
            "launches": calls_dom, "avg_launch_us": t_dom / calls_dom * 1e6,
            "algorithmic_bytes_per_launch": b_dom / calls_dom,
            "stream_copy_gbs": stream_gbs, "frac_of_stream": achieved / stream_gbs}
    if dom == "spmm":
        # the product's own gathers, without rows: the memory system's ceiling
        # for this index stream (the product also reads offsets and writes Y)
        tg = float(np.median(time_gather_bound(P, A, block, torch.float32, stream, 10)))
        roof["gather_bound_us"] = tg * 1e6
        roof["gather_bound_frac"] = tg / (t_dom / calls_dom)
        log(f"gathers alone at b={block}: {tg*1e3:.2f} ms per launch; the product "
            f"{t_dom/calls_dom*1e3:.2f} ms ({100*roof['gather_bound_frac']:.0f}% of its ceiling)")
    spmm_alone = next((x for x in sweep if x["b"] == block), None)
    if roof["traffic"]:
        roof["traffic_gbs"] = roof["traffic"] / (t_dom / calls_dom) / 1e9  # bytes beyond the L2
    if dom == "spmm" and spmm_alone:
        # the same kernel alone (the sweep's launches at this width): in the
        # solve the first product after each restart shares the GPU with the
        # restart rotation, which lengthens those launches
        roof["standalone_launch_us"] = spmm_alone["us"]
        roof["frac_standalone"] = b_dom / calls_dom / (spmm_alone["us"] * 1e-6) / 1e9 / HBM_PEAK_GBS

    out = {
        "metric": METRIC, "value": value, "unit": "GEdge·col/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_all / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16+f32" if args.mixed else "f32",
        "data": "synthetic",
        "config": {"workload": f"rmat{args.scale}_krylov_schur_nev8_b{block}_m{m}_"
                               + ("mixed_bf16_f32" if args.mixed else "f32"),
                   "scale": args.scale, "n": A.n, "nnz": A.nnz, "edge_factor": 16,
                   "rmat_abcd": [0.57, 0.19, 0.19, 0.05], "nev": nev, "block": block, "m": m,
                   "tol": tol, "relabel": "degree", "storage": "bf16->f32" if args.mixed else "f32"},
        "roofline": roof,
        "time_to_8_eigs_s": float(np.median(times)),
        "spmm_alone_at_block": spmm_alone,
        "solve": {"restarts": [r.restarts for r in results],
                  "spmm_calls_bf16": [r.spmm_calls_low for r in results],
                  "spmm_calls": [r.spmm_calls for r in results],
                  "max_resid": [float(r.resid.max()) for r in results],
                  "evals": [float(x) for x in results[-1].evals]},
        "spmm_sweep": sweep,
        "spmm_sweep_second_graph": sweep2,
        "generate_s": t_gen, "build_s": t_build,
    }
    if args.weights and os.path.exists(args.weights):
        lb, lm = (int(x) for x in args.learned_shape.split("x"))
        out["learned_vs_random"] = learned_vs_random(P, A, stream, args.weights, tol, lb, lm)
    A.close()
    torch.cuda.empty_cache()
    if not args.no_cpu:
        log("timing the CPU oracle on a bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(n, s, d, block, m)
        cb = out["cpu_baseline"]
        log(f"cpu baseline: {cb['value']:.3f} GEdge*col/s on {cb['cores']} threads, "
            f"{cb['one_core']['value']:.3f} on one core (the product alone "
            f"{cb['spmm_only']['all_cores']:.2f} and {cb['spmm_only']['one_core']:.2f})")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
