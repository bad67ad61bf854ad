"""The seeded generators produce simple, connected, undirected graphs in sorted CSR."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import graphgen as gg

CASES = [
    lambda: gg.path_graph(7), lambda: gg.cycle_graph(8), lambda: gg.grid2d(6, 5),
    lambda: gg.grid3d(4, 3, 5, weights=(0.5, 1.5), seed=3), lambda: gg.complete_graph(6),
    lambda: gg.star_graph(9), lambda: gg.hypercube(4), lambda: gg.spider(3, 4),
    lambda: gg.random_connected(80, 100, seed=1, weights=(0.5, 1.5)),
    lambda: gg.rmat(10, 8, seed=5), lambda: gg.chung_lu(3000, 2.1, 24.0, seed=6),
]


@pytest.mark.parametrize("make", CASES)
def test_simple_connected_symmetric(make):
    g = make()
    assert g.row_ptr.dtype == np.int32 and g.col.dtype == np.int32
    assert g.row_ptr[0] == 0 and np.all(np.diff(g.row_ptr) >= 1)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert np.all(rows != g.col)  # no self loops
    for i in range(0, g.n, max(1, g.n // 50)):
        seg = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert np.all(np.diff(seg) > 0)  # sorted, unique
    vals = np.ones(g.nnz) if g.w is None else g.w
    A = sp.csr_matrix((vals, g.col, g.row_ptr), shape=(g.n, g.n))
    assert abs(A - A.T).max() == 0
    if g.w is not None:
        assert g.w.min() > 0
    assert connected_components(A, directed=False)[0] == 1


def test_seeded_and_deterministic():
    a = gg.rmat(9, 8, seed=11)
    b = gg.rmat(9, 8, seed=11)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.row_ptr, b.row_ptr)
    g = gg.grid3d(3, 3, 3, weights=(0.5, 1.5), seed=3)
    first = np.random.default_rng(3).uniform(0.5, 1.5, size=1)[0]
    # vertex 0's first edge is its +x edge to vertex 1, and it is drawn first
    assert g.col[0] == 1 and g.w[0] == first
    U = gg.start_block(50, 3, 1)
    assert U.shape == (50, 3) and U.flags.f_contiguous


def _dup_weighted(device=None):
    # repeated undirected edges with different weights (the first occurrence keeps its
    # weight), self loops, and three components: the largest is not the one of vertex 0
    rng = np.random.default_rng(21)
    u = np.concatenate([[0, 1, 0], 3 + rng.integers(0, 200, 900), 250 + rng.integers(0, 40, 60)])
    v = np.concatenate([[1, 0, 0], 3 + rng.integers(0, 200, 900), 250 + rng.integers(0, 40, 60)])
    w = rng.uniform(0.5, 1.5, u.size)
    return gg.generators._csr_from_undirected(300, u, v, w, lcc=True, relabel_seed=5, device=device)


@pytest.mark.parametrize("make", [
    lambda d: gg.rmat(12, 8, seed=5, device=d), lambda d: gg.rmat(11, 16, seed=4000, device=d),
    lambda d: gg.chung_lu(20000, 2.1, 24.0, seed=6, device=d), _dup_weighted,
    lambda d: gg.generators._csr_from_undirected(50, np.arange(49), np.arange(1, 50), lcc=False,
                                                 device=d),
])
def test_torch_path_gives_the_same_csr(make):
    """The torch-sorted path (used on the GPU for the large workloads) returns exactly the
    CSR of the numpy/scipy path: same vertex count, pattern, order and weights."""
    a = make(None)
    b = make("cpu")
    assert a.n == b.n and a.nnz == b.nnz
    assert np.array_equal(a.row_ptr, b.row_ptr) and b.row_ptr.dtype == np.int32
    assert np.array_equal(a.col, b.col) and b.col.dtype == np.int32
    assert (a.w is None) == (b.w is None)
    if a.w is not None:
        assert np.array_equal(a.w, b.w)
