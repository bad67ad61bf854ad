"""Pins of the SPAI network oracle: central finite differences of its hand-written
backward pass, the SPD construction, BF16 rounding, and the Jacobi special case."""
import math
import pathlib

import numpy as np
import pytest

import graphgen as gg
from oracle import spai_oracle as SO
from oracle import isira_oracle as O

# trained network weights shipped with the package (plain FP32 array, no pickle)
WEIGHTS = pathlib.Path(__file__).resolve().parents[1] / "paper_1710_07080_amd" / "weights" / "spai_rmat_h16.npy"


def _samples(g, trim, S, seed):
    rng = np.random.default_rng(seed)
    R = rng.standard_normal((g.n, S))
    Z = rng.standard_normal((g.n, S))
    R[trim] = 0.0
    Z[trim] = 0.0
    return R, Z


@pytest.mark.parametrize("gname", ["rand_w", "rmat", "grid"])
def test_backward_matches_central_differences(gname):
    g = {"rand_w": lambda: gg.random_connected(40, 70, seed=3, weights=(0.5, 1.5)),
         "rmat": lambda: gg.rmat(7, 8, seed=4),
         "grid": lambda: gg.grid2d(6, 5)}[gname]()
    trim = O.trim_index(O.degrees(g))
    sigma = 0.1 if gname == "rand_w" else 0.0
    rng = np.random.default_rng(1)
    p = SO.init_params(2).astype(np.float64) + 0.2 * rng.standard_normal(SO.NPARAM)
    R, Z = _samples(g, trim, 3, 5)
    L, grad = SO.loss_grad(g, p, sigma, trim, R, Z, round_bf16=False)
    assert L == pytest.approx(SO.loss(g, p, sigma, trim, R, Z, round_bf16=False), rel=1e-14)
    idx = np.unique(np.concatenate([rng.choice(SO.NPARAM, 80, replace=False),
                                    [SO.OFF[k][0] for k in SO.OFF]]))
    h = 1e-6
    for i in idx:
        pp = p.copy()
        pm = p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (SO.loss(g, pp, sigma, trim, R, Z, False) - SO.loss(g, pm, sigma, trim, R, Z, False)) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, grad[i])


def test_M_is_symmetric_sdd_and_spd():
    g = gg.rmat(8, 8, seed=6)
    trim = O.trim_index(O.degrees(g))
    p = SO.init_params(3).astype(np.float64)
    p[SO.OFF["ce"][0]] = 3.0  # large edge values: stress the dominance bound
    fw = SO.forward(g, p.astype(np.float32), 0.0, trim)
    M = SO.dense_M(g, fw["diag"], fw["offd"])
    keep = np.array([i for i in range(g.n) if i != trim])
    Mh = M[np.ix_(keep, keep)]
    assert np.array_equal(Mh, Mh.T)
    off = np.abs(Mh).sum(axis=1) - np.abs(np.diag(Mh))
    assert np.all(np.diag(Mh) > 0) and np.all(off < np.diag(Mh))
    assert np.linalg.eigvalsh(Mh).min() > 0
    assert np.all(M[trim] == 0) and np.all(M[:, trim] == 0)


def test_bf16_rounding_published_format():
    # bfloat16 keeps 8 significant bits; ties go to the even significand
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 1.0 + 2 ** -7, 3.0e38], dtype=np.float32)
    out = SO.bf16_round(vals)
    assert list(out[:5]) == [1.0, 1.0, 1.0 + 2 ** -6, -2.5, 1.0 + 2 ** -7]
    assert np.isfinite(out[5])


def test_zero_network_is_jacobi():
    g = gg.random_connected(30, 40, seed=7, weights=(0.5, 1.5))
    trim = 4
    P = {k: np.zeros(v) if v > 1 else 0.0 for k, (o, v) in SO.OFF.items()}
    P = SO.unpack(np.zeros(SO.NPARAM))
    P["bd"] = float(np.log(np.e - 1.0))
    fw = SO.forward(g, SO.pack(P), 0.3, trim, round_bf16=False)
    d = O.degrees(g)
    ref = 1.0 / (d - 0.3)
    ref[trim] = 0.0
    assert np.allclose(fw["diag"], ref, rtol=1e-14)
    assert np.all(fw["offd"] == 0.0)


def test_prune_by_hand():
    # path 0-1-2 with M_00 = 4, M_11 = 1, M_22 = 9 and m_01 = 0.5, m_12 = -1.2:
    # sqrt(M_00 M_11) = 2, sqrt(M_11 M_22) = 3; tau = 0.2 keeps |0.5| >= 0.4 and
    # |-1.2| >= 0.6; tau = 0.3 drops m_01 (0.5 < 0.6) and keeps m_12 (1.2 >= 0.9); tau = 0.25
    # keeps m_01 at equality (0.5 >= 0.5)
    g = gg.path_graph(3)
    diag = np.array([4.0, 1.0, 9.0])
    # CSR order: row 0: (0,1); row 1: (1,0), (1,2); row 2: (2,1)
    offd = np.array([0.5, 0.5, -1.2, -1.2])
    assert g.col.tolist() == [1, 0, 2, 1]
    assert SO.prune(g, diag, offd, 0.2).tolist() == [0.5, 0.5, -1.2, -1.2]
    assert SO.prune(g, diag, offd, 0.3).tolist() == [0.0, 0.0, -1.2, -1.2]
    assert SO.prune(g, diag, offd, 0.25).tolist() == [0.5, 0.5, -1.2, -1.2]
    assert SO.prune(g, diag, offd, 0.5).tolist() == [0.0] * 4


def test_prune_keeps_spd_and_nests():
    g = gg.rmat(9, 8, seed=6)
    trim = O.trim_index(O.degrees(g))
    params = np.load(WEIGHTS)
    fw = SO.forward(g, params, 0.0, trim)
    keep = np.array([i for i in range(g.n) if i != trim])
    prev = None
    for tau in [0.0, 0.01, 0.03, 0.1, 0.3]:
        off = SO.prune(g, fw["diag"], fw["offd"], tau)
        if tau == 0.0:
            assert np.array_equal(off, fw["offd"])  # every nonzero is kept
        kept = off != 0.0
        assert np.array_equal(off[kept], fw["offd"][kept])  # kept values are unchanged
        if prev is not None:
            assert not np.any(kept & ~prev)  # a larger threshold keeps a subset
        prev = kept
        M = SO.dense_M(g, fw["diag"], off)[np.ix_(keep, keep)]
        assert np.array_equal(M, M.T)
        offsum = np.abs(M).sum(axis=1) - np.diag(M)
        assert np.all(offsum < np.diag(M))
        assert np.linalg.eigvalsh(M).min() > 0
    assert 0 < int(prev.sum()) < fw["offd"].size


def test_isira_with_pruned_learned_matches_dense():
    g = gg.rmat(9, 8, seed=11)
    k = 6
    params = np.load(WEIGHTS)

    def factory(trim, sigma):
        fw = SO.forward(g, params, sigma, trim)
        off = SO.prune(g, fw["diag"], fw["offd"], 0.02)
        return lambda x: O.trim(SO.apply(g, fw["diag"], off, trim, np.insert(x, trim, 0.0)), trim)

    res = O.isira(g, k, 0.0, 1e-10, gg.start_block(g.n, 4, 1), inner_rtol=1e-1,
                  apply_minv_hat_factory=factory)
    ref, _ = O.smallest_positive_eigenpairs_dense(g, k)
    assert np.allclose(np.sort(res.evals), ref, rtol=1e-9, atol=0)


def _weighted_graph(n, edges):
    """CSRGraph from an explicit edge list (u, v, w), built by hand without the generators'
    component and relabelling steps."""
    rows = {i: [] for i in range(n)}
    for u, v, w in edges:
        rows[u].append((v, w))
        rows[v].append((u, w))
    rp, col, wt = [0], [], []
    for i in range(n):
        for v, w in sorted(rows[i]):
            col.append(v)
            wt.append(w)
        rp.append(len(col))
    return gg.CSRGraph(n, np.array(rp, np.int32), np.array(col, np.int32), np.array(wt, np.float64))


def test_features_star_by_hand():
    # Star, centre 0 joined to leaves 1..4 (unit weights), trimmed vertex 0, sigma = 0.5.
    # Centre: d = n = 4, every neighbour has log d = 0, it is the trimmed vertex itself (no
    # self loop, so not adjacent to it).  Leaf: d = n = 1, its one neighbour has log d = log 4,
    # and it is adjacent to the trimmed vertex.
    g = gg.star_graph(5)
    f = SO.features(g, 0.5, 0)
    l4 = math.log(4.0)
    centre = [1.0, l4, l4, 0.0, 0.0, 0.125, 0.25, 0.0]
    leaf = [1.0, 0.0, 0.0, l4, l4, 0.5, 1.0, 1.0]
    assert f.shape == (5, SO.F)
    assert np.allclose(f[0], centre, rtol=1e-15, atol=0)
    for i in range(1, 5):
        assert np.allclose(f[i], leaf, rtol=1e-15, atol=0)


def test_features_weighted_path_by_hand():
    # Path 0-1-2-3 with weights 2, 0.5, 3 and the trimmed vertex 1, sigma = 0.25.
    # Weighted degrees d = (2, 2.5, 3.5, 3); neighbour counts (1, 2, 2, 1).  The columns are
    # [1, log d_i, log n_i, mean_j log d_j, max_j log d_j, sigma/d_i, 1/n_i, adjacent to 1].
    # Every pair of columns that a slip could confuse differs somewhere: log d vs log n
    # (vertex 0: log 2 vs 0), mean vs max (vertex 1: (log 2 + log 3.5)/2 vs log 3.5),
    # sigma/d vs 1/n, and the adjacency flag (vertices 0 and 2, not 1 itself or 3).
    g = _weighted_graph(4, [(0, 1, 2.0), (1, 2, 0.5), (2, 3, 3.0)])
    f = SO.features(g, 0.25, 1)
    L = math.log
    want = np.array([
        [1.0, L(2.0), 0.0, L(2.5), L(2.5), 0.125, 1.0, 1.0],
        [1.0, L(2.5), L(2.0), 0.5 * (L(2.0) + L(3.5)), L(3.5), 0.1, 0.5, 0.0],
        [1.0, L(3.5), L(2.0), 0.5 * (L(2.5) + L(3.0)), L(3.0), 0.25 / 3.5, 0.5, 1.0],
        [1.0, L(3.0), 0.0, L(3.5), L(3.5), 0.25 / 3.0, 1.0, 0.0],
    ])
    assert np.allclose(f, want, rtol=1e-15, atol=1e-300)


def test_features_vertex_next_to_trimmed_hub():
    # Two triangles sharing vertex 0 (the hub, degree 4) plus a pendant vertex 5 on vertex 3:
    # the adjacency flag is 1 exactly for the neighbours of the trimmed vertex (1, 2, 3, 4)
    # and the neighbour max picks the hub's log 4 for them while the mean does not.
    g = _weighted_graph(6, [(0, 1, 1.0), (0, 2, 1.0), (1, 2, 1.0), (0, 3, 1.0), (0, 4, 1.0),
                            (3, 4, 1.0), (3, 5, 1.0)])
    f = SO.features(g, 0.0, 0)
    L = math.log
    assert f[:, 7].tolist() == [0.0, 1.0, 1.0, 1.0, 1.0, 0.0]
    # vertex 1: neighbours 0 (d 4) and 2 (d 2)
    assert np.allclose(f[1, 3:5], [0.5 * (L(4.0) + L(2.0)), L(4.0)], rtol=1e-15)
    # vertex 3: neighbours 0 (d 4), 4 (d 2), 5 (d 1)
    assert np.allclose(f[3, 1:5], [L(3.0), L(3.0), (L(4.0) + L(2.0) + 0.0) / 3.0, L(4.0)], rtol=1e-15)
    # vertex 5: its one neighbour is 3 (d 3)
    assert np.allclose(f[5], [1.0, 0.0, 0.0, L(3.0), L(3.0), 0.0, 1.0, 0.0], rtol=1e-15, atol=0)
