"""Pins of the multilevel-preconditioner oracle against facts fixed by its definition and by
mathematics, not by re-running its own code: aggregates of small graphs derived by hand
from the rule, Galerkin coarse matrices in closed form, the textbook two-grid error
propagation operator formed from dense matrices, exactness when no coarsening happens,
symmetry and definiteness of the cycle, conservation laws of the Galerkin product, and
end-to-end eigenvalues against dense eigendecomposition."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import graphgen as gg
from oracle import isira_oracle as O
from oracle import multilevel_oracle as ML


def lap_from_edges(n, edges):
    L = np.zeros((n, n))
    for a, b in edges:
        L[a, b] -= 1.0
        L[b, a] -= 1.0
        L[a, a] += 1.0
        L[b, b] += 1.0
    return sp.csr_matrix(L)


def test_aggregate_path_by_hand():
    # order: 1..8 (two neighbours), then 0, 9.  Phase 1: 1 -> {0,1,2}, 4 -> {3,4,5},
    # 7 -> {6,7,8}; phase 2: 9 joins the aggregate of 8.
    L = lap_from_edges(10, [(i, i + 1) for i in range(9)])
    assert ML.aggregate(L).tolist() == [0, 0, 0, 1, 1, 1, 2, 2, 2, 2]


def test_aggregate_cycle_and_star_by_hand():
    L = lap_from_edges(6, [(i, (i + 1) % 6) for i in range(6)])
    # order 0..5: 0 -> {0,1,5}; 2 is blocked by 1; 3 -> {2,3,4}
    assert ML.aggregate(L).tolist() == [0, 0, 1, 1, 1, 0]
    S = lap_from_edges(6, [(0, j) for j in range(1, 6)])
    assert ML.aggregate(S).tolist() == [0] * 6


def test_aggregate_phase2_counts_and_ties():
    # two stars (hubs 0 and 4) and a middle vertex 8 adjacent to 3 and 7: the hubs come
    # first and take their stars; 8 touches one member of each -> tie -> smaller id 0
    edges = [(0, 1), (0, 2), (0, 3), (4, 5), (4, 6), (4, 7), (8, 3), (8, 7)]
    assert ML.aggregate(lap_from_edges(9, edges)).tolist() == [0, 0, 0, 0, 1, 1, 1, 1, 0]
    # with an extra edge 8-6, vertex 8 has three neighbours (visited third, blocked) and
    # two of them in aggregate 1 -> joins 1
    edges2 = edges + [(8, 6)]
    assert ML.aggregate(lap_from_edges(9, edges2)).tolist() == [0, 0, 0, 0, 1, 1, 1, 1, 1]


def test_isolated_vertices_stay_out():
    # trimming the centre of a star leaves only isolated leaves; a path hanging off a
    # star keeps its own aggregates while the bare leaves get -1
    S = lap_from_edges(6, [(0, j) for j in range(1, 6)]).toarray()[1:, 1:]
    assert ML.aggregate(sp.csr_matrix(S)).tolist() == [-1] * 5
    L = lap_from_edges(7, [(0, 1), (0, 2), (0, 3), (3, 4), (4, 5), (5, 6)]).toarray()[1:, 1:]
    # remaining graph: 1, 2 isolated; path 3-4-5-6 (labels 2..5): order 3, 4 (two
    # neighbours), then 2, 5: 3 -> {2,3,4}; 5 joins by phase 2
    assert ML.aggregate(sp.csr_matrix(L)).tolist() == [-1, -1, 0, 0, 0, 0]


def test_isolated_vertices_solved_exactly():
    g = gg.star_graph(40)
    i = O.trim_index(O.degrees(g))
    h = ML.setup(g, i, coarse_max=8)  # only isolated leaves: one diagonal level
    assert len(h.A) == 1
    Lhat = O.trimmed_matrix(O.laplacian(g), i).toarray()
    assert np.allclose(ML.operator_matrix(h) @ Lhat, np.eye(g.n - 1), atol=1e-12)
    # paths of four vertices hanging off each of 30 leaves of a star's centre: trimming the
    # centre leaves 30 such paths; each becomes one aggregate, i.e. an isolated coarse
    # vertex solved exactly there
    edges, nxt = [], 31
    for leaf in range(1, 31):
        edges.append((0, leaf))
        prev = leaf
        for _ in range(3):
            edges.append((prev, nxt))
            prev, nxt = nxt, nxt + 1
    n = nxt
    u, v = zip(*edges)
    g2 = gg.generators._csr_from_undirected(n, np.array(u), np.array(v), lcc=False)
    i2 = O.trim_index(O.degrees(g2))
    h = ML.setup(g2, i2, coarse_max=8)
    assert [A.shape[0] for A in h.A] == [n - 1, 30]
    assert ML.connected_count(h.A[1]) == 0
    B = ML.operator_matrix(h)
    assert np.allclose(B, B.T, atol=1e-12)
    assert np.linalg.eigvalsh(B).min() > 0
    # coarse_max = 0 coarsens a connected graph until no vertex has a neighbour
    h0 = ML.setup(gg.grid2d(9, 7), 0, coarse_max=0)
    assert ML.connected_count(h0.A[-1]) == 0 and len(h0.A) >= 3


def test_galerkin_of_path_is_coarse_path():
    L = lap_from_edges(10, [(i, i + 1) for i in range(9)])
    P = ML.prolongation(ML.aggregate(L))
    Ac = (P.T @ L @ P).toarray()
    assert np.array_equal(Ac, np.array([[1.0, -1, 0], [-1, 2, -1], [0, -1, 1]]))


def test_single_level_is_exact_inverse():
    g = gg.grid2d(6, 5)
    i = O.trim_index(O.degrees(g))
    h = ML.setup(g, i, coarse_max=10_000)
    assert len(h.A) == 1
    Lhat = O.trimmed_matrix(O.laplacian(g), i).toarray()
    B = ML.operator_matrix(h)
    assert np.allclose(B @ Lhat, np.eye(g.n - 1), atol=1e-10)


def _weights(Ad, omega):
    """omega, or 1 for a row without off-diagonal entries (from the dense matrix)."""
    off = Ad - np.diag(np.diag(Ad))
    return np.where(np.any(off != 0, axis=1), omega, 1.0)


def _dense_levels(h):
    return [A.toarray() for A in h.A], [P.toarray() for P in h.P]


@pytest.mark.parametrize("g,cmax", [(gg.grid2d(8, 8), 20), (gg.rmat(8, 4, seed=3), 30),
                                    (gg.grid3d(4, 4, 4, weights=(0.5, 1.5), seed=2), 12)])
def test_two_grid_error_propagation(g, cmax):
    """I - B A = (I - S A)(I - P A_c^{-1} P^T A)(I - S A), S = omega D^-1: the textbook
    two-grid operator with one pre- and one post-sweep, from dense matrices."""
    i = O.trim_index(O.degrees(g))
    h = ML.setup(g, i, coarse_max=cmax)
    assert len(h.A) == 2, [A.shape for A in h.A]
    (A, Ac), (P,) = _dense_levels(h)
    S = np.diag(_weights(A, h.omega) / np.diag(A))
    I = np.eye(A.shape[0])
    E = (I - S @ A) @ (I - P @ np.linalg.solve(Ac, P.T @ A)) @ (I - S @ A)
    B = ML.operator_matrix(h)
    assert np.allclose(I - B @ A, E, atol=1e-10)


def test_three_level_recursion():
    """The level-0 cycle is the two-grid formula with A_1^{-1} replaced by the level-1
    cycle B_1."""
    g = gg.grid2d(12, 12)
    i = O.trim_index(O.degrees(g))
    h = ML.setup(g, i, coarse_max=6)
    assert len(h.A) >= 3
    As, Ps = _dense_levels(h)
    A, P = As[0], Ps[0]
    B1 = ML.operator_matrix(h, 1)
    S = np.diag(_weights(A, h.omega) / np.diag(A))
    I = np.eye(A.shape[0])
    E = (I - S @ A) @ (I - P @ B1 @ P.T @ A) @ (I - S @ A)
    B = ML.operator_matrix(h)
    assert np.allclose(I - B @ A, E, atol=1e-10)


@pytest.mark.parametrize("g", [gg.rmat(9, 6, seed=5), gg.grid3d(5, 5, 4, weights=(0.5, 1.5), seed=1),
                               gg.random_connected(300, 500, seed=4, weights=(0.2, 3.0))])
def test_cycle_symmetric_positive_definite(g):
    i = O.trim_index(O.degrees(g))
    h = ML.setup(g, i, coarse_max=8)
    assert len(h.A) >= 3
    B = ML.operator_matrix(h)
    assert np.allclose(B, B.T, atol=1e-12 * np.abs(B).max())
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_galerkin_conservation_laws():
    """Off-diagonals stay <= 0, row sums stay >= 0, and 1^T A 1 (on level 0 the total
    weight of the edges to the trimmed vertex) passes to the next level less the
    diagonals of the vertices without neighbours, which leave the hierarchy."""
    g = gg.rmat(10, 8, seed=7)
    d = O.degrees(g)
    i = O.trim_index(d)
    h = ML.setup(g, i, coarse_max=16)
    L = O.laplacian(g)
    grounded = -L[i].toarray().ravel().sum() + L[i, i]  # sum of weights of edges at i
    assert len(h.A) >= 3
    mass = grounded
    for A in h.A:
        Ad = A.toarray()
        off = Ad - np.diag(np.diag(Ad))
        assert off.max() <= 0.0
        assert Ad.sum(axis=1).min() >= -1e-9
        assert abs(Ad.sum() - mass) <= 1e-9 * grounded
        lone = ~np.any(off != 0, axis=1)
        mass = Ad.sum() - np.diag(Ad)[lone].sum()


def test_multilevel_pcg_needs_far_fewer_iterations_than_jacobi():
    g = gg.grid2d(48, 48)
    d = O.degrees(g)
    i = O.trim_index(d)
    L = O.laplacian(g)
    Lhat = O.trimmed_matrix(L, i)
    b = np.random.default_rng(1).standard_normal(g.n - 1)
    h = ML.setup(g, i, coarse_max=64)
    A = lambda x: Lhat @ x
    x_ml, it_ml, _ = O.pcg(A, b, lambda x: ML.vcycle(h, x), 1e-10, 1000)
    dh = O.trim(d, i)
    x_j, it_j, _ = O.pcg(A, b, lambda x: x / dh, 1e-10, 1000)
    ref = spla.spsolve(Lhat.tocsc(), b)
    assert np.linalg.norm(x_ml - ref) <= 1e-8 * np.linalg.norm(ref)
    assert it_ml * 4 < it_j, (it_ml, it_j)


def test_isira_with_multilevel_matches_dense():
    g = gg.rmat(9, 8, seed=11)
    k = 6
    u0 = gg.start_block(g.n, 4, 1)
    res = O.isira(g, k, 0.0, 1e-10, u0, inner_rtol=1e-1,
                  apply_minv_hat_factory=ML.preconditioner_factory(g, coarse_max=16))
    ref, _ = O.smallest_positive_eigenpairs_dense(g, k)
    assert np.allclose(np.sort(res.evals), ref, rtol=1e-9, atol=0)
