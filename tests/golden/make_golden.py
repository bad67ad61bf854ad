"""Write full-size reference eigenvalues with the FP64 oracle (and nothing else).

    python tests/golden/make_golden.py rmat20      # R-MAT scale 20, k = 20 (~20-30 min)
    python tests/golden/make_golden.py grid128w    # weighted 128^3 grid, k = 20 (~1 h)
    python tests/golden/make_golden.py rmat22e16   # held-out R-MAT scale 22, edge factor 16, k = 20

Inputs come from the seeded generators; the start block is the one the bench and the GPU
tests use (start_block(n, 4, 1)).  The inner tolerance is 1e-6 for R-MAT (close to exact
shift-invert residual Arnoldi) and 1e-1 for the grid, whose inner systems need thousands of
iterations, and for the held-out scale-22 R-MAT graph (128 M stored entries), where tighter
inner solves would take the oracle many hours; residual Arnoldi reaches the same eigenpairs with any inner tolerance (the
outer residual test decides), which the GPU tests then check at 1e-9 relative.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import graphgen as gg  # noqa: E402
from oracle import isira_oracle as O  # noqa: E402

CASES = {
    "rmat20": dict(make=lambda: gg.rmat(20, 8, seed=2), k=20, sigma=0.0, tol=1e-8, rtol=1e-6),
    "grid128w": dict(make=lambda: gg.grid3d(128, 128, 128, weights=(0.5, 1.5), seed=3), k=20,
                     sigma=0.0, tol=1e-8, rtol=1e-1),
    "rmat22e16": dict(make=lambda: gg.rmat(22, 16, seed=4000), k=20, sigma=0.0, tol=1e-8, rtol=1e-1),
}


def main(name):
    c = CASES[name]
    g = c["make"]()
    t = time.time()
    res = O.isira(g, c["k"], c["sigma"], c["tol"], gg.start_block(g.n, 4, 1), inner_rtol=c["rtol"])
    el = time.time() - t
    out = {
        "workload": name, "n": g.n, "nnz": g.nnz, "k": c["k"], "sigma": c["sigma"], "tol": c["tol"],
        "start_block": "graphgen.start_block(n, 4, 1)", "oracle_inner_rtol": c["rtol"],
        "evals_sorted": sorted(float(v) for v in res.evals), "evals_locking_order": [float(v) for v in res.evals],
        "resid": [float(v) for v in res.resid], "outer_its": res.outer_its, "inner_its": res.inner_its,
        "oracle_seconds": el, "written_by": "tests/golden/make_golden.py (oracle only)",
    }
    with open(os.path.join(HERE, f"{name}_k{c['k']}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "done", el, np.sort(res.evals))


if __name__ == "__main__":
    main(sys.argv[1])
