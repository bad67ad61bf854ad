"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test compares the oracle with something other than itself: closed-form spectra,
invariants of graph Laplacians (Theorem 1.2), the exactness of trimming (Theorems 2.4 and
2.8), the Sherman-Morrison-Woodbury identity (eq. (3.5)), dense eigendecomposition of a
Laplacian built here by a loop over the edge list, and published generator outputs.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
from oracle import isira_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_laplacian_from_edges(g):
    """Independent construction: walk the stored entries one by one."""
    L = np.zeros((g.n, g.n))
    for i in range(g.n):
        for idx in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = int(g.col[idx])
            w = 1.0 if g.w is None else float(g.w[idx])
            L[i, j] -= w
            L[i, i] += w
    return L


SMALL = [
    gg.path_graph(9),
    gg.cycle_graph(10),
    gg.grid2d(5, 4),
    gg.star_graph(7),
    gg.hypercube(3),
    gg.spider(3, 4),
    gg.random_connected(40, 50, seed=1),
    gg.random_connected(35, 70, seed=2, weights=(0.5, 1.5)),
    gg.grid3d(3, 3, 3, weights=(0.5, 1.5), seed=3),
]


# ----------------------------------------------------------------------------- Laplacian


@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_laplacian_matches_edge_loop(g):
    ref = dense_laplacian_from_edges(g)
    got = O.laplacian(g).toarray()
    if g.w is None:
        assert np.array_equal(got, ref)
    else:  # weighted degrees: only the summation order differs
        assert np.abs(got - ref).max() <= 4e-16 * ref.max() * g.counts().max()


@pytest.mark.parametrize("g", SMALL + [gg.rmat(10, 8, seed=5)], ids=lambda g: g.name)
def test_null_vector_and_quadratic_form(g):
    # Theorem 1.2: L 1 = 0; x^T L x = sum over edges w_ij (x_i - x_j)^2 >= 0
    one = np.ones(g.n)
    scale = O.degrees(g).max()
    assert np.abs(O.laplacian_apply(g, one)).max() <= 1e-13 * scale
    x = np.random.default_rng(0).standard_normal(g.n)
    quad = 0.0
    for i in range(g.n):
        for idx in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = int(g.col[idx])
            w = 1.0 if g.w is None else float(g.w[idx])
            quad += 0.5 * w * (x[i] - x[j]) ** 2
    assert abs(x @ O.laplacian_apply(g, x) - quad) <= 1e-11 * abs(quad)
    if g.w is None:
        assert O.laplacian(g).diagonal().sum() == g.nnz  # trace = 2|E|


def _closed_form(name):
    if name == "path":
        n = 12
        return gg.path_graph(n), np.sort(2 - 2 * np.cos(np.arange(n) * np.pi / n))
    if name == "cycle":
        n = 11
        return gg.cycle_graph(n), np.sort(2 - 2 * np.cos(2 * np.pi * np.arange(n) / n))
    if name == "complete":
        n = 7
        return gg.complete_graph(n), np.array([0.0] + [float(n)] * (n - 1))
    if name == "star":
        n = 8
        return gg.star_graph(n), np.array([0.0] + [1.0] * (n - 2) + [float(n)])
    if name == "hypercube":
        d = 4
        vals = []
        for i in range(d + 1):
            vals += [2.0 * i] * math.comb(d, i)
        return gg.hypercube(d), np.array(vals)
    if name == "grid":
        nx, ny = 6, 5
        px = 2 - 2 * np.cos(np.arange(nx) * np.pi / nx)
        py = 2 - 2 * np.cos(np.arange(ny) * np.pi / ny)
        return gg.grid2d(nx, ny), np.sort((px[:, None] + py[None, :]).ravel())
    raise KeyError(name)


@pytest.mark.parametrize("name", ["path", "cycle", "complete", "star", "hypercube", "grid"])
def test_closed_form_spectra_of_oracle_laplacian(name):
    g, lam = _closed_form(name)
    got = np.linalg.eigvalsh(O.laplacian(g).toarray())
    assert np.allclose(got, lam, atol=1e-12 * max(1.0, lam.max()))


def test_spider_antisymmetric_modes():
    # p identical legs of length l: 2 - 2 cos((2j-1) pi / (2l+1)) with multiplicity >= p-1
    p, l = 4, 3
    got = np.linalg.eigvalsh(O.laplacian(gg.spider(p, l)).toarray())
    for j in range(1, l + 1):
        lam = 2 - 2 * np.cos((2 * j - 1) * np.pi / (2 * l + 1))
        assert np.sum(np.abs(got - lam) < 1e-10) >= p - 1


# ------------------------------------------------------------------------- hyper-params


def test_trim_index_and_delta():
    # Remark 4.1: maximum degree, lowest index among ties; delta = 2 max diag(L)
    assert O.trim_index(O.degrees(gg.star_graph(6))) == 0
    assert O.trim_index(O.degrees(gg.cycle_graph(9))) == 0
    g = gg.path_graph(6)  # degrees 1 2 2 2 2 1
    assert O.trim_index(O.degrees(g)) == 1
    assert O.deflation_shift(O.degrees(g)) == 4.0
    gw = gg.random_connected(30, 40, seed=4, weights=(0.5, 1.5))
    d = dense_laplacian_from_edges(gw).diagonal()
    assert O.trim_index(O.degrees(gw)) == int(np.flatnonzero(d == d.max())[0])
    assert O.deflation_shift(O.degrees(gw)) == pytest.approx(2 * d.max(), rel=1e-15)


# ------------------------------------------------------------------------- trimming


def _rhs_perp_one(n, seed):
    r = np.random.default_rng(seed).standard_normal(n)
    return r - r.mean()


@pytest.mark.parametrize("g", [gg.random_connected(60, 80, seed=7), gg.grid2d(7, 6),
                               gg.random_connected(50, 90, seed=8, weights=(0.5, 1.5))],
                         ids=lambda g: g.name)
def test_trimming_theorem_exact_and_independent_of_index(g):
    # Theorem 2.4: enlarging the solution of the trimmed system solves L z = r, 1^T z = 0,
    # for every choice of the trimmed index; it equals the pseudo-inverse solution.
    Ld = dense_laplacian_from_edges(g)
    r = _rhs_perp_one(g.n, 1)
    ref = np.linalg.pinv(Ld) @ r
    for i in [0, g.n // 3, g.n - 1, O.trim_index(O.degrees(g))]:
        keep = [t for t in range(g.n) if t != i]
        zhat = np.linalg.solve(Ld[np.ix_(keep, keep)], r[keep])
        z = O.enlarge(zhat, i, g.n)
        assert abs(z.sum()) <= 1e-12 * np.abs(z).max()
        assert np.allclose(Ld @ z, r, atol=1e-10)
        assert np.allclose(z, ref, atol=1e-10 * np.abs(ref).max())


@pytest.mark.parametrize("sigma_frac,c", [(0.0, 0), (0.5, 0), (0.0, 3), (0.6, 3)])
def test_inner_solve_shifted_deflated(sigma_frac, c):
    # Theorem 2.8: the enlarged solution of eq. (2.15) solves
    # (L + delta V V^T - sigma I) z = r with 1^T z = 0, whatever the trimmed index.
    g = gg.random_connected(70, 120, seed=11, weights=(0.5, 1.5))
    Ld = dense_laplacian_from_edges(g)
    lam, X = np.linalg.eigh(Ld)
    V = X[:, 1:1 + c]
    delta = 2 * Ld.diagonal().max()
    Lt = Ld + delta * V @ V.T
    lam_t = np.sort(np.linalg.eigvalsh(Lt))[1]  # smallest positive of the deflated L
    sigma = sigma_frac * lam_t
    r = _rhs_perp_one(g.n, 2)
    A = Lt - sigma * np.eye(g.n)
    # reference: the unique solution orthogonal to 1 (eigen-expansion of the deflated L)
    lt, Xt = np.linalg.eigh(Lt)
    ref = Xt[:, 1:] @ ((Xt[:, 1:].T @ r) / (lt[1:] - sigma))
    L = O.laplacian(g)
    d = O.degrees(g)
    for i in [O.trim_index(d), 0, g.n - 1]:
        z, its, rel = O.inner_solve(L, d, r, i, sigma, delta, V, 1e-14, 5000)
        assert its > 0 and rel <= 1e-14
        assert abs(z.sum()) <= 1e-11 * np.abs(z).max()
        assert np.allclose(A @ z, r, atol=1e-9 * np.abs(r).max())
        assert np.allclose(z, ref, atol=1e-9 * np.abs(ref).max())


def test_trimmed_operator_without_rank_one_term():
    # Remark 3.1: dropping (sigma/n) 1 1^T leaves (L-hat - sigma I) + delta V-hat V-hat^T, the
    # trimmed principal submatrix of L + delta V V^T - sigma I built from the edge list;
    # at sigma = 0 both operators coincide.
    g = gg.random_connected(50, 90, seed=14, weights=(0.5, 1.5))
    Ld = dense_laplacian_from_edges(g)
    lam, X = np.linalg.eigh(Ld)
    V = X[:, 1:3]
    delta = 2 * Ld.diagonal().max()
    i = O.trim_index(O.degrees(g))
    keep = [t for t in range(g.n) if t != i]
    Lhat = O.trimmed_matrix(O.laplacian(g), i)
    Vhat = V[keep]
    x = np.random.default_rng(3).standard_normal(g.n - 1)
    sigma = 0.3 * lam[1]
    dense = (Ld + delta * V @ V.T - sigma * np.eye(g.n))[np.ix_(keep, keep)]
    y = O.trimmed_operator(Lhat, g.n, sigma, delta, Vhat, rank_one=False)(x)
    assert np.allclose(y, dense @ x, atol=1e-11 * np.abs(dense @ x).max())
    y1 = O.trimmed_operator(Lhat, g.n, sigma, delta, Vhat)(x)
    assert np.allclose(y1 - y, (sigma / g.n) * x.sum(), atol=1e-11 * np.abs(y).max())
    y0 = O.trimmed_operator(Lhat, g.n, 0.0, delta, Vhat, rank_one=False)(x)
    assert np.array_equal(y0, O.trimmed_operator(Lhat, g.n, 0.0, delta, Vhat)(x))
    # the inner solve then solves that trimmed system (SPD here: sigma < its smallest eigenvalue)
    assert np.linalg.eigvalsh(dense).min() > 0
    r = _rhs_perp_one(g.n, 4)
    z, its, rel = O.inner_solve(O.laplacian(g), O.degrees(g), r, i, sigma, delta, V, 1e-14, 5000,
                                rank_one=False)
    zhat = np.linalg.solve(dense, r[keep])
    assert np.allclose(z, O.enlarge(zhat, i, g.n), atol=1e-9 * np.abs(zhat).max())


def test_trimmed_operator_inertia():
    # K-hat is congruent to a Schur complement of J (L~ - sigma I) J^T (proof of Theorem
    # 2.8): it is positive definite iff sigma < lambda_{c+1}, with one negative
    # eigenvalue for lambda_{c+1} < sigma < lambda_{c+2}.
    g = gg.random_connected(40, 60, seed=13)
    Ld = dense_laplacian_from_edges(g)
    lam, X = np.linalg.eigh(Ld)
    c = 2
    V = X[:, 1:1 + c]
    delta = 2 * Ld.diagonal().max()
    lt = np.sort(np.linalg.eigvalsh(Ld + delta * V @ V.T))
    L = O.laplacian(g)
    i = 5
    Lhat = O.trimmed_matrix(L, i)
    Vhat = O.trim(V, i)
    for sigma, nneg in [(0.5 * lt[1], 0), (0.5 * (lt[1] + lt[2]), 1)]:
        A = O.trimmed_operator(Lhat, g.n, sigma, delta, Vhat)
        K = np.column_stack([A(e) for e in np.eye(g.n - 1)])
        assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())
        assert int(np.sum(np.linalg.eigvalsh(K) < 0)) == nneg


def test_smw_preconditioner_is_exact_inverse():
    # eq. (3.5): the SMW form equals (M + delta V V^T)^{-1}
    rng = np.random.default_rng(3)
    nm1, c = 50, 4
    dhat = rng.uniform(1, 10, nm1)
    sigma = 0.3
    V = np.linalg.qr(rng.standard_normal((nm1, c)))[0]
    delta = 20.0
    P = O.jacobi_smw_preconditioner(dhat, sigma, delta, V)
    x = rng.standard_normal(nm1)
    ref = np.linalg.solve(np.diag(dhat - sigma) + delta * V @ V.T, x)
    assert np.allclose(P(x), ref, rtol=1e-12, atol=1e-13)


def test_pcg_solves_spd_system():
    rng = np.random.default_rng(4)
    B = rng.standard_normal((40, 40))
    A = B @ B.T + 40 * np.eye(40)
    b = rng.standard_normal(40)
    x, its, rel = O.pcg(lambda v: A @ v, b, lambda v: v / np.diag(A), 1e-13, 500)
    assert rel <= 1e-13 and its <= 60
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-11)


def test_cgs2_orthogonality():
    rng = np.random.default_rng(5)
    Q = np.linalg.qr(rng.standard_normal((200, 12)))[0]
    z = rng.standard_normal(200) + Q @ rng.standard_normal(12) * 1e6
    out, before, after = O.cgs2(Q, z)
    assert np.abs(Q.T @ out).max() <= 1e-14 * after
    assert before == pytest.approx(np.linalg.norm(z))


def test_single_gram_schmidt_pass_when_little_is_removed():
    """The second-pass test the solver applies (Daniel, Gragg, Kaufman, Stewart): when one
    classical Gram-Schmidt pass keeps at least 1/sqrt(2) of the norm, its result is
    orthogonal to working precision, and CGS2 changes it only at rounding level; with heavy
    cancellation one pass is not enough.  Plain arithmetic on random data, no library
    orthogonalization."""
    rng = np.random.default_rng(8)
    n, m = 5000, 60
    Q = np.linalg.qr(rng.standard_normal((n, m)))[0]
    worst = 0.0
    for t in range(20):
        z = rng.standard_normal(n) + Q @ rng.standard_normal(m) * rng.uniform(0.0, 0.8)
        one = z - Q @ (Q.T @ z)
        kept = np.linalg.norm(one) / np.linalg.norm(z)
        assert kept >= 1 / np.sqrt(2)  # the case the test lets through
        two, _, after = O.cgs2(Q, z)
        worst = max(worst, np.abs(Q.T @ one).max() / np.linalg.norm(one))
        assert np.linalg.norm(one - two) <= 1e-14 * after
    assert worst <= 1e-14
    z = rng.standard_normal(n) + Q @ rng.standard_normal(m) * 1e8  # heavy cancellation
    one = z - Q @ (Q.T @ z)
    assert np.linalg.norm(one) / np.linalg.norm(z) < 1 / np.sqrt(2)
    assert np.abs(Q.T @ one).max() / np.linalg.norm(one) > 1e-12  # a second pass is needed


def test_splitmix64_published_outputs():
    gold = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    got = O.splitmix64(1234567, np.arange(3))
    assert [str(int(v)) for v in got] == gold["seed_1234567_first_three"]
    assert hex(int(O.splitmix64(0, [0])[0])) == gold["seed_0_first"]
    seq0 = [int(h, 16) for h in gold["seed_0_first_four"]]
    assert [int(v) for v in O.splitmix64(0, np.arange(4))] == seq0
    u = O.splitmix64_uniform(9, np.arange(100000))
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01


def _uniform_from_published(z: int) -> Fraction:
    # the replacement generator's reading: the top 53 bits of an output, as a fraction of
    # 2^53, mapped affinely onto [-1, 1); exact rational arithmetic on the published integer
    return Fraction(2 * (z >> 11), 1 << 53) - 1


def test_replacement_vector_from_published_outputs():
    """Entry l of replacement vector `draw` is output number draw*n + l of the sequence
    started from the seed, mapped to [-1, 1): checked against the published SplitMix64
    outputs (seed 0: four outputs; seed 1234567: three), exactly."""
    gold = json.load(open(os.path.join(GOLDEN, "splitmix64.json")))
    seq0 = [int(h, 16) for h in gold["seed_0_first_four"]]
    seq1 = [int(v) for v in gold["seed_1234567_first_three"]]
    # seed 0, n = 2: draw 0 holds outputs 0, 1 and draw 1 holds outputs 2, 3
    for draw in (0, 1):
        got = O.replacement_vector(2, 0, draw)
        want = [_uniform_from_published(seq0[2 * draw + l]) for l in range(2)]
        assert [Fraction(float(v)) for v in got] == want
    # seed 1234567, n = 3, draw 0: outputs 0, 1, 2; n = 1: draw j is output j
    got = O.replacement_vector(3, 1234567, 0)
    assert [Fraction(float(v)) for v in got] == [_uniform_from_published(z) for z in seq1]
    for draw in range(3):
        v = O.replacement_vector(1, 1234567, draw)
        assert Fraction(float(v[0])) == _uniform_from_published(seq1[draw])


# ------------------------------------------------------------------------- Algorithm 3.2


def _check_result(g, res, k, tol, lam_ref, rel=1e-9):
    Ld = dense_laplacian_from_edges(g)
    assert res.converged == k
    assert np.all(np.diff(res.evals) >= -1e-12)  # found in ascending order
    assert np.allclose(np.sort(res.evals), lam_ref, rtol=rel, atol=0)
    X = res.evecs
    assert np.abs(X.T @ X - np.eye(k)).max() <= 1e-10
    assert np.abs(X.sum(axis=0)).max() <= 1e-9
    for j in range(k):
        assert np.linalg.norm(Ld @ X[:, j] - res.evals[j] * X[:, j]) <= max(tol, 1e-13)
        assert res.resid[j] <= tol


def test_isira_grid64_closed_form():
    # 64 x 64 grid: lambda = 4 sin^2(i pi/128) + 4 sin^2(j pi/128); 10 smallest positive
    g = gg.grid2d(64, 64)
    i, j = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    lam = np.sort((4 * np.sin(i * np.pi / 128) ** 2 + 4 * np.sin(j * np.pi / 128) ** 2).ravel())[1:11]
    res = O.isira(g, 10, 0.0, 1e-10, gg.start_block(g.n, 4, 1), inner_rtol=1e-10)
    assert res.converged == 10
    assert np.allclose(np.sort(res.evals), lam, rtol=1e-9, atol=0)
    assert res.resid.max() <= 1e-10
    assert np.abs(np.sum(res.evals) - 0.11553176561244477) <= 1e-12


@pytest.mark.parametrize("case", [
    dict(g=gg.random_connected(150, 200, seed=21), k=8, sigma=0.0, q=10, m=14),
    dict(g=gg.random_connected(160, 400, seed=22, weights=(0.5, 1.5)), k=6, sigma=0.0, q=8, m=12),
    dict(g=gg.random_connected(120, 150, seed=23), k=5, sigma="half", q=None, m=None),
    dict(g=gg.rmat(8, 8, seed=24), k=8, sigma=0.0, q=12, m=20),
], ids=["rand150", "rand160w", "rand120shift", "rmat8"])
def test_isira_matches_dense_eig(case):
    g = case["g"]
    k = case["k"]
    lam_all = np.linalg.eigvalsh(dense_laplacian_from_edges(g))
    sigma = 0.5 * lam_all[1] if case["sigma"] == "half" else case["sigma"]
    tol = 1e-9
    res = O.isira(g, k, sigma, tol, gg.start_block(g.n, 3, 5), q=case["q"], m=case["m"],
                  inner_rtol=1e-6)
    _check_result(g, res, k, tol, lam_all[1:k + 1], rel=1e-8)


@pytest.mark.parametrize("name,k,k0", [("hypercube", 10, 6), ("star", 5, 5), ("path", 5, 2),
                                       ("cycle", 6, 3)])
def test_isira_closed_form_multiplicities(name, k, k0):
    # Single-vector expansion keeps the basis inside the block-Krylov space of the start
    # block, so an eigenvalue of multiplicity M needs a start block of >= M columns.
    g, lam = {"hypercube": lambda: _closed_form("hypercube"),
              "star": lambda: (gg.star_graph(20), np.array([0.0] + [1.0] * 18 + [20.0])),
              "path": lambda: (gg.path_graph(120), np.sort(2 - 2 * np.cos(np.arange(120) * np.pi / 120))),
              "cycle": lambda: (gg.cycle_graph(90), np.sort(2 - 2 * np.cos(2 * np.pi * np.arange(90) / 90))),
              }[name]()
    res = O.isira(g, k, 0.0, 1e-10, gg.start_block(g.n, k0, 2), inner_rtol=1e-8)
    _check_result(g, res, k, 1e-10, lam[1:k + 1], rel=1e-9)


def test_isira_spider_multiplicity():
    p, l = 5, 4
    g = gg.spider(p, l)
    lam = np.linalg.eigvalsh(dense_laplacian_from_edges(g))
    k = 8
    res = O.isira(g, k, 0.0, 1e-10, gg.start_block(g.n, p - 1, 3), inner_rtol=1e-8)
    _check_result(g, res, k, 1e-10, lam[1:k + 1], rel=1e-9)
    first = 2 - 2 * np.cos(np.pi / (2 * l + 1))
    assert np.sum(np.abs(res.evals - first) < 1e-9) >= p - 1



def test_isira_whisker_eigenvalues():
    # K_12 with two leaves (12, 13) and two 2-paths (0-14-15, 0-16-17) on vertex 0.  The leaf
    # mode (+1 on 12, -1 on 13, 0 elsewhere) is an eigenvector of L for eigenvalue 1 (each
    # leaf row reads x_leaf - x_0 = x_leaf); the antisymmetric 2-path modes (a, b on 14, 15 and
    # -a, -b on 16, 17) reduce to the 2x2 matrix [[2, -1], [-1, 1]], eigenvalues
    # (3 -+ sqrt 5) / 2.
    g = gg.whiskered_clique(12)
    golden = (3.0 - math.sqrt(5.0)) / 2.0  # 0.3819660112501051
    # the leaf mode is an exact eigenvector for 1, entry by entry
    x = np.zeros(g.n)
    x[12], x[13] = 1.0, -1.0
    assert np.array_equal(O.laplacian_apply(g, x), x)
    k = 4
    res = O.isira(g, k, 0.0, 1e-11, gg.start_block(g.n, 2, 4), inner_rtol=1e-10)
    ev = np.sort(res.evals)
    assert abs(ev[0] - golden) <= 1e-10 * golden
    assert np.sum(np.abs(ev - 1.0) <= 1e-10) == 2  # the leaf mode and one more mode at 1
    # the remaining value against a dense eigensolver (not a closed form)
    lam = np.linalg.eigvalsh(dense_laplacian_from_edges(g))
    assert abs(ev[1] - lam[2]) <= 1e-9 * lam[2]


def _minres_norm_check(K, b, P, x, rel):
    # eta is the P-norm of the residual (P the preconditioner, the inverse of M)
    r = b - K @ x
    true = math.sqrt(r @ (P @ r)) / math.sqrt(b @ (P @ b))
    assert abs(true - rel) <= 1e-6 * max(true, 1e-300) + 1e-13


def test_minres_spd_and_indefinite():
    # MINRES (Paige-Saunders, preconditioned): on the SPD trimmed Laplacian and on an
    # indefinite shift of it, the iterate converges to the unique solution, and the
    # recursively updated residual norm equals the true P-norm of b - K x.
    g = gg.random_connected(80, 160, seed=21, weights=(0.5, 1.5))
    L = O.laplacian(g).toarray()
    d = L.diagonal()
    i = int(np.argmax(d))
    keep = [t for t in range(g.n) if t != i]
    Lh = L[np.ix_(keep, keep)]
    mu = np.linalg.eigvalsh(Lh)
    b = np.random.default_rng(5).standard_normal(g.n - 1)
    for sigma in [0.0, 0.5 * mu[0], 0.5 * (mu[2] + mu[3])]:  # SPD, SPD, 3 negative eigenvalues
        K = Lh - sigma * np.eye(g.n - 1)
        P = np.diag(1.0 / (d[keep] - sigma))
        x, its, rel = O.minres(lambda v: K @ v, b, lambda v: P @ v, 1e-12, 2000)
        assert rel <= 1e-12 and 0 < its <= 2000
        xs = np.linalg.solve(K, b)
        assert np.allclose(x, xs, atol=1e-9 * np.abs(xs).max())
        _minres_norm_check(K, b, P, x, rel)
        # stopped early, the recursion still reports the true residual norm
        x5, its5, rel5 = O.minres(lambda v: K @ v, b, lambda v: P @ v, 0.0, 5)
        assert its5 == 5
        _minres_norm_check(K, b, P, x5, rel5)


def test_inner_solve_minres_indefinite():
    # Thm 2.8 with sigma between lambda_{c+1} and lambda_{c+2} of the deflated L: K-hat has one
    # negative eigenvalue, PCG does not apply, MINRES still returns the solution of
    # (L + delta V V^T - sigma I) z = r with 1^T z = 0, for any trimmed index.
    g = gg.random_connected(70, 120, seed=11, weights=(0.5, 1.5))
    Ld = dense_laplacian_from_edges(g)
    lam, X = np.linalg.eigh(Ld)
    V = X[:, 1:3]
    delta = 2 * Ld.diagonal().max()
    Lt = Ld + delta * V @ V.T
    lt, Xt = np.linalg.eigh(Lt)
    sigma = 0.5 * (lt[1] + lt[2])
    r = _rhs_perp_one(g.n, 2)
    ref = Xt[:, 1:] @ ((Xt[:, 1:].T @ r) / (lt[1:] - sigma))
    L = O.laplacian(g)
    d = O.degrees(g)
    for i in [O.trim_index(d), 0]:
        z, its, rel = O.inner_solve(L, d, r, i, sigma, delta, V, 1e-13, 5000, solver="minres")
        assert rel <= 1e-13
        assert abs(z.sum()) <= 1e-10 * np.abs(z).max()
        assert np.allclose((Lt - sigma * np.eye(g.n)) @ z, r, atol=1e-8 * np.abs(r).max())
        assert np.allclose(z, ref, atol=1e-8 * np.abs(ref).max())


@pytest.mark.parametrize("g,k", [(gg.grid2d(9, 7), 6), (gg.random_connected(120, 300, seed=4), 8),
                                 (gg.rmat(8, 8, seed=9), 8)], ids=lambda x: getattr(x, "name", str(x)))
def test_isira_moving_shift_matches_dense(g, k):
    # Algorithm 3.2 with the purge step's moving shift (sigma <- theta_2, MINRES inner solves)
    # reaches the k smallest positive eigenvalues of the dense eigendecomposition.
    lam, _ = O.smallest_positive_eigenpairs_dense(g, k)
    U0 = gg.start_block(g.n, 4, 1)
    res = O.isira(g, k, 0.0, 1e-10, U0, inner_rtol=1e-10, moving_shift=True)
    assert res.converged == k
    assert np.allclose(np.sort(res.evals), lam, rtol=1e-9, atol=0)
    assert res.resid.max() < 1e-10
