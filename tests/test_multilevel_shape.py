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
