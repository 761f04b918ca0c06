"""Write the oracle's eigenvalues for the full-size R-MAT graphs (test fixtures).

Calls only the CPU oracle and the seeded input generators: the R-MAT edge
stream (scale s, edge factor 16, a/b/c/d = .57/.19/.19/.05, seed s), the
oracle's own CSR (symmetrised, deduplicated, self-loops dropped) and the
oracle's FP64 block Krylov-Schur for the 8 largest-magnitude eigenvalues at
tol 1e-10.  The eigenvalues do not depend on the solve shape, so the widest
block the tests use (16 columns, subspace 112) is taken because it needs the
fewest restarts.

    python tests/golden/make_golden.py 22      # writes tests/golden/rmat22_evals.json
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import fe_synth as S  # noqa: E402
import oracle as O  # noqa: E402

NEV, BLOCK, M, TOL, START_SEED = 8, 16, 112, 1e-10, 3


def main(scale: int, threads: int) -> str:
    t0 = time.time()
    n, s, d = S.rmat_edges(scale, edge_factor=16, a=0.57, b=0.19, c=0.19, seed=scale)
    rp, ci = O.csr_from_edges(n, s, d)
    del s, d
    t1 = time.time()
    print(f"scale {scale}: n={n} nnz={int(rp[-1])} (edges + oracle CSR {t1 - t0:.0f} s)", flush=True)

    def spmm(X):
        return O.spmm(rp, ci, X, threads=threads)

    r = O.krylov_schur(spmm, n, NEV, BLOCK, M, TOL, S.normal((n, BLOCK), seed=START_SEED))
    t2 = time.time()
    print(f"solve: converged={r.converged} restarts={r.restarts} products={r.spmm_calls} "
          f"max resid {r.resid.max():.2e} ({t2 - t1:.0f} s)", flush=True)
    assert r.converged and r.resid.max() <= 1e-9
    deg = np.diff(rp)
    out = {
        "graph": {"family": "rmat", "scale": scale, "edge_factor": 16,
                  "abcd": [0.57, 0.19, 0.19, 0.05], "seed": scale, "relabel_seed": scale + 1},
        "n": int(n), "nnz": int(rp[-1]), "max_degree": int(deg.max()),
        "solver": {"nev": NEV, "block": BLOCK, "m": M, "tol": TOL, "start_seed": START_SEED,
                   "storage": "f64", "eta": 1e-10},
        "evals": [float(x) for x in r.evals],
        "resid": [float(x) for x in r.resid],
        "restarts": int(r.restarts), "products": int(r.spmm_calls),
        "seconds": round(t2 - t0, 1), "threads": threads,
        "script": "tests/golden/make_golden.py",
    }
    path = os.path.join(HERE, f"rmat{scale}_evals.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    return path


if __name__ == "__main__":
    scale = int(sys.argv[1])
    threads = int(sys.argv[2]) if len(sys.argv) > 2 else (os.cpu_count() or 1)
    print(main(scale, threads))
