"""CPU parity of the library's multilevel set-up (host code) with the oracle's: the
aggregation rule uses no floating point, so the hierarchy's shape -- vertices, stored
off-diagonal entries and vertices with neighbours on every level -- must be equal."""
import numpy as np
import pytest

import graphgen as gg
from oracle import isira_oracle as O
from oracle import multilevel_oracle as ML


@pytest.fixture(scope="module")
def P():
    import paper_1710_07080_amd as pkg

    pkg.load()
    return pkg


def _star_with_paths():
    edges, nxt = [], 31
    for leaf in range(1, 31):
        edges.append((0, leaf))
        prev = leaf
        for _ in range(3):
            edges.append((prev, nxt))
            prev, nxt = nxt, nxt + 1
    u, v = zip(*edges)
    return gg.generators._csr_from_undirected(nxt, np.array(u), np.array(v), lcc=False)


CASES = [
    ("path", lambda: gg.path_graph(101), 4, None),
    ("grid2d", lambda: gg.grid2d(40, 33), 0, None),
    ("grid3d_w", lambda: gg.grid3d(20, 17, 13, weights=(0.5, 1.5), seed=3), 32, None),
    ("rmat12", lambda: gg.rmat(12, 8, seed=3), 16, None),
    ("rmat14", lambda: gg.rmat(14, 8, seed=9), 64, None),
    ("rand_w", lambda: gg.random_connected(2000, 3000, seed=4, weights=(0.2, 3.0)), 16, None),
    ("star_paths", _star_with_paths, 8, None),
    ("star", lambda: gg.star_graph(300), 8, None),
    ("chunglu", lambda: gg.chung_lu(20000, 2.1, 8.0, seed=14), 128, None),
    ("rmat12_trim_min", lambda: gg.rmat(12, 8, seed=3), 16, "min"),
    # above 65,536 rows the library builds the levels with several host threads
    ("grid3d_big", lambda: gg.grid3d(48, 48, 40, weights=(0.5, 1.5), seed=5), 64, None),
    ("rmat17", lambda: gg.rmat(17, 8, seed=13), 64, None),
]


@pytest.mark.parametrize("name,make,cm,trim", CASES, ids=[c[0] for c in CASES])
def test_hierarchy_shape_matches_oracle(P, name, make, cm, trim):
    g = make()
    d = O.degrees(g)
    i = O.trim_index(d) if trim is None else int(np.argmin(d))
    info = P.isira.ml_shape(g, i, coarse_max=cm)
    h = ML.setup(g, i, coarse_max=cm)
    assert info["levels"] == len(h.A)
    assert info["rows"] == [A.shape[0] for A in h.A]
    assert info["offdiag_nnz"] == [A.nnz - int(np.count_nonzero(A.diagonal())) for A in h.A]
    assert info["connected"] == [ML.connected_count(A) for A in h.A]
    assert info["coarsest_dense"] == info["connected"][-1] <= cm


def test_shape_errors(P):
    g = gg.grid2d(10, 10)
    with pytest.raises(P.IsiraError) as e:
        P.isira.ml_shape(g, 0, omega=1.0)
    assert e.value.code == P.isira.ISIRA_E_ARG
    with pytest.raises(P.IsiraError) as e:
        P.isira.ml_shape(g, 500)
    assert e.value.code == P.isira.ISIRA_E_ARG
    with pytest.raises(P.IsiraError) as e:
        P.isira.ml_shape(g, 0, coarse_max=0, max_levels=2)
    assert e.value.code == P.isira.ISIRA_E_PRECOND


GALERKIN = [c for c in CASES if c[0] in ("grid3d_w", "rmat14", "rand_w", "star_paths", "chunglu", "rmat12_trim_min",
                                         "grid3d_big", "rmat17")]


@pytest.mark.parametrize("name,make,cm,trim", GALERKIN, ids=[c[0] for c in GALERKIN])
def test_galerkin_levels_match_oracle_entrywise(P, name, make, cm, trim):
    """Every level's matrix A_{l+1} = P_l^T A_l P_l of the library's set-up against the
    oracle's, entry by entry: both sum the same fine entries in other orders, so each entry
    differs by at most 2 (K - 1) u times the sum of the absolute values of its K fine terms
    (u = 2^-53); the test allows 2 K u.  The coarse vertices are matched through the aggregates (same rule, other
    numbering)."""
    import scipy.sparse as sp

    g = make()
    d = O.degrees(g)
    i = O.trim_index(d) if trim is None else int(np.argmin(d))
    h = ML.setup(g, i, coarse_max=cm)
    keep = np.delete(np.arange(g.n), i)
    pi = keep.copy()  # oracle vertex index -> library vertex index on the current level
    Aabs = abs(h.A[0]).tocsr()
    # number of terms summed into each entry: one weight off the diagonal, the row's weights
    # (all of them, the trimmed vertex's too) on the diagonal
    K = Aabs.copy()
    K.data[:] = 1.0
    K = (K - sp.diags(K.diagonal()) + sp.diags(g.counts()[keep].astype(np.float64))).tocsr()
    u = 2.0 ** -53
    worst = 0.0
    for lvl, A in enumerate(h.A):
        W, dg, agg = P.isira.ml_level_matrix(g, i, lvl, coarse_max=cm)
        Alib = (sp.diags(dg) - W).tocsr()[pi][:, pi]
        diff = abs(Alib - A).tocsr()
        bound = (2.0 * u * K.multiply(Aabs)).tocsr()
        # entries outside the oracle's pattern must be exactly zero
        outside = diff - diff.multiply(bound > 0)
        assert outside.count_nonzero() == 0 or abs(outside).max() == 0.0, (name, lvl)
        ratio = diff.multiply(bound > 0)
        if ratio.nnz:
            b = bound[ratio.nonzero()]
            r = np.asarray(ratio[ratio.nonzero()]).ravel() / np.asarray(b).ravel()
            worst = max(worst, float(r.max()))
            assert r.max() <= 1.0, (name, lvl, float(r.max()))
        if lvl + 1 < len(h.A):
            agg_o = h.agg[lvl]
            nxt = -np.ones(h.A[lvl + 1].shape[0], dtype=np.int64)
            mem = np.flatnonzero(agg_o >= 0)
            lib_ids = agg[pi[mem]]
            assert np.all(lib_ids >= 0)
            nxt[agg_o[mem]] = lib_ids
            # one library aggregate per oracle aggregate, and the same members
            assert np.all(nxt >= 0) and np.unique(nxt).size == nxt.size
            assert np.array_equal(nxt[agg_o[mem]], agg[pi[mem]])
            Pm = h.P[lvl]
            Aabs = (Pm.T @ Aabs @ Pm).tocsr()
            K = (Pm.T @ K @ Pm).tocsr()
            pi = nxt
    print(f"{name}: {len(h.A)} levels, largest entry difference / its rounding bound {worst:.3f}")
