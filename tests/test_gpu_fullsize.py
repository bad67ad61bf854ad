"""GPU parity at full size, in the configuration the benchmark times.

The reference eigenvalues come from the FP64 oracle (``tests/golden/make_golden.py``, which
calls nothing but ``oracle/``) on the same seeded graphs with the same start block.  Checks:
eigenvalues within 1e-9 relative of the oracle's, true residuals ||Lx - lambda x||_2 formed
by the oracle's own sparse Laplacian on the CPU (below tol, hence below 1e-8 ||L||_1),
orthonormality, x orthogonal to 1, and the sign convention.  The eigenpairs do not depend
on the inner preconditioner, so the multilevel solves are checked against the same
references, and so are the solves with the trained learned preconditioner pruned as in the
benchmark; the multilevel hierarchy and one cycle are also compared with the oracle's at
full size (its set-up takes up to a minute on the host).
"""
import json
import os

import numpy as np
import pytest

import graphgen as gg
from oracle import isira_oracle as O
from oracle import multilevel_oracle as ML
from ml_levels import hierarchy_with_library_matrices

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

WORKLOADS = {
    "rmat20": lambda: gg.rmat(20, 8, seed=2),
    "grid128w": lambda: gg.grid3d(128, 128, 128, weights=(0.5, 1.5), seed=3),
    # the learned preconditioner's held-out graph: R-MAT scale 22, edge factor 16 (mean degree
    # 32 before deduplication), built with the GPU sorts (same CSR as the numpy path)
    "rmat22e16": lambda: gg.rmat(22, 16, seed=4000, device="cuda"),
}


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07080_amd as pkg

    pkg.load()
    return pkg


_cache = {}


def _setup(P, name):
    path = os.path.join(GOLDEN, f"{name}_k20.json")
    if not os.path.exists(path):
        pytest.skip(f"no oracle reference {path}")
    if name not in _cache:
        gold = json.load(open(path))
        g = WORKLOADS[name]()
        assert (g.n, g.nnz) == (gold["n"], gold["nnz"])
        _cache.clear()  # one full-size graph resident at a time
        _cache[name] = (gold, g, P.Context.from_graph(g), O.laplacian(g))
    return _cache[name]


@pytest.mark.parametrize("name,prec,pc", [("rmat20", 0, 0), ("rmat20", 1, 0), ("rmat20", 0, 2),
                                         ("rmat20", 1, 1), ("grid128w", 1, 0), ("grid128w", 0, 0),
                                         ("grid128w", 1, 2), ("grid128w", 1, 1),
                                         ("rmat22e16", 0, 0), ("rmat22e16", 1, 1)])
def test_fullsize_matches_oracle(P, name, prec, pc):
    gold, g, ctx, L = _setup(P, name)
    k, tol = gold["k"], gold["tol"]
    if pc == P.isira.PC_MULTILEVEL:
        ctx.ml_setup()
    if pc == P.isira.PC_LEARNED:
        # the trained network, pruned as in the benchmark's learned + FP32 form
        from paper_1710_07080_amd import spai_train

        if not os.path.exists(spai_train.DEFAULT_WEIGHTS):
            pytest.skip("no trained weights")
        ctx.spai_install(spai_train.load(), sigma=gold["sigma"])
        assert ctx.spai_prune(0.02) > 0
    ev, X, res, st = ctx.solve(k, gold["sigma"], tol, u0=gg.start_block(g.n, 4, 1), inner_prec=prec,
                               precond=pc)
    assert st["n_converged"] == k
    order = np.argsort(ev)
    ev = ev[order]
    ref = np.array(gold["evals_sorted"])
    rel = np.abs(ev - ref) / ref
    print(f"{name} prec={prec} precond={pc}: per-pair relative error vs oracle: {np.array2string(rel, precision=2)}")
    assert rel.max() <= 1e-9
    Xh = X.cpu().numpy()[order]
    norm1 = 2.0 * O.degrees(g).max()
    for j in range(k):
        x = Xh[j]
        r = np.linalg.norm(L @ x - ev[j] * x)
        assert r <= tol and r <= 1e-8 * norm1
        # the library's own FP64 residual agrees with the oracle's
        assert abs(r - res[order[j]]) <= 1e-10
        i = np.argmax(np.abs(x))
        assert x[i] > 0
    G = Xh @ Xh.T
    assert np.abs(G - np.eye(k)).max() <= 1e-10
    assert np.abs(Xh.sum(axis=1)).max() <= 1e-8 * np.sqrt(g.n)



def test_learned_gain_on_held_out_graph(P):
    """The trained network in the M-hat slot of Remark 3.2, on its held-out evaluation graph
    (R-MAT scale 22, mean degree 32, seed 4000: never seen in training), pruned as in the
    benchmark's learned + FP32 form, against FP32 Jacobi in the same launch configuration:
    both reach the oracle's eigenvalues, and the learned form takes at least 8 % fewer
    inner iterations.  Wall times are printed, not asserted (they move with the rounding
    of the iteration counts by a few per cent)."""
    from paper_1710_07080_amd import spai_train

    if not os.path.exists(spai_train.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    gold, g, ctx, L = _setup(P, "rmat22e16")
    k, tol = gold["k"], gold["tol"]
    ref = np.array(gold["evals_sorted"])
    ctx.spai_install(spai_train.load(), sigma=gold["sigma"])
    assert ctx.spai_prune(0.02) > 0
    runs = {}
    for name, pc in [("fp32_jacobi", P.isira.PC_JACOBI), ("learned_pruned", P.isira.PC_LEARNED)]:
        ev, X, res, st = ctx.solve(k, gold["sigma"], tol, u0=gg.start_block(g.n, 4, 1),
                                   inner_prec=P.isira.FP32, precond=pc)
        assert st["n_converged"] == k and res.max() < tol
        rel = np.abs(np.sort(ev) - ref) / ref
        assert rel.max() <= 1e-9, (name, rel.max())
        runs[name] = st
    print("; ".join(f"{n}: outer {st['outer_total']}, inner {st['inner_total']}, {st['ms_total']:.0f} ms"
                    for n, st in runs.items()))
    assert runs["learned_pruned"]["inner_total"] <= 0.92 * runs["fp32_jacobi"]["inner_total"]


@pytest.mark.parametrize("name", ["rmat20", "grid128w"])
def test_fullsize_multilevel_cycle(P, name):
    """Hierarchy shape (exact) and one cycle in FP64 and FP32 against the oracle's, on the
    benchmark graphs with the default set-up (coarse_max 512, omega 0.9)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _cache.clear()
    g = WORKLOADS[name]()
    ctx = P.Context.from_graph(g)
    i = O.trim_index(O.degrees(g))
    info = ctx.ml_setup()
    h = ML.setup(g, i, coarse_max=512)
    assert info["rows"] == [A.shape[0] for A in h.A]
    assert info["connected"] == [ML.connected_count(A) for A in h.A]
    x = np.random.default_rng(6).standard_normal(g.n)
    ref = np.insert(ML.vcycle(h, O.trim(x, i)), i, 0.0)
    # The coarsest level is solved exactly: the library applies an explicit inverse formed by
    # Cholesky, the oracle a sparse direct solve, and either carries an error of about
    # kappa(A_L) u (4 u kappa allowed).  Against the oracle's cycle over the library's own
    # level matrices that is the only term besides the cycle's rounding; against the
    # oracle's own matrices their rounding differences (a few u each, pinned entry by entry on
    # the CPU) add about as much again through the same solve.
    hl = hierarchy_with_library_matrices(P, g, i, h, 512)
    ref_l = np.insert(ML.vcycle(hl, O.trim(x, i)), i, 0.0)
    ev = np.linalg.eigvalsh(h.A[-1].toarray()) if h.A[-1].shape[0] > 1 else np.ones(1)
    kappa = ev[-1] / ev[0]
    u = 2.0 ** -53
    for prec, bound, bound_l in [(0, 1e-12 + 8 * u * kappa, 1e-12 + 4 * u * kappa), (1, 3e-5, 3e-5)]:
        y = ctx.ml_apply(torch.as_tensor(x, device="cuda"), prec=prec).cpu().numpy()
        err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
        err_l = np.linalg.norm(y - ref_l) / np.linalg.norm(ref_l)
        print(f"{name} cycle prec={prec}: relative error {err:.2e} against the oracle (bound "
              f"{bound:.1e}, coarsest condition {kappa:.2e}), {err_l:.2e} against the oracle's cycle "
              f"over the library's matrices (bound {bound_l:.1e}), levels {info['rows']}")
        assert err <= bound and err_l <= bound_l
