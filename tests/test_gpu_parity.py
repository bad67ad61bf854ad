"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Every case is seeded; sizes span several tiles, ragged tails, rows split into chunks (longer
than a work unit of the product: 2048 nonzeros, 4096 in the hub-cached shape) and rows
summed by a whole workgroup.
"""
import math

import numpy as np
import pytest

import graphgen as gg
from oracle import isira_oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07080_amd as pkg

    pkg.load()
    return pkg


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _hub_graph():
    # a hub of degree 9000 (split into 5 chunks of the 2048-nonzero units), rows of about
    # 1500 and 2000 nonzeros (one unit each), and a random sparse remainder -- every SpMV
    # row class of the stream shape at once
    n = 12000
    rng = np.random.default_rng(77)
    u = [np.zeros(9000, dtype=np.int64), np.full(2000, 1), np.full(1500, 2)]
    v = [np.arange(1, 9001), rng.integers(3, n, 2000), rng.integers(3, n, 1500)]
    tree_order = rng.permutation(n)
    parents = tree_order[(rng.random(n - 1) * np.arange(1, n)).astype(np.int64)]
    u += [tree_order[1:], rng.integers(0, n, 20000)]
    v += [parents, rng.integers(0, n, 20000)]
    from graphgen.generators import _csr_from_undirected

    return _csr_from_undirected(n, np.concatenate(u), np.concatenate(v), lcc=True, name="hubs")


GRAPHS = {
    "grid64": lambda: gg.grid2d(64, 64),
    "grid3d_w": lambda: gg.grid3d(20, 17, 13, weights=(0.5, 1.5), seed=3),
    "rmat14": lambda: gg.rmat(14, 8, seed=9),
    "hubs": _hub_graph,
    "star": lambda: gg.star_graph(5000),
    "path": lambda: gg.path_graph(1001),
    # n > 4 * 8192 with a quarter of the gathers on the 8192 highest-degree labels: the
    # hub-cached SpMV shape
    "rmat17": lambda: gg.rmat(17, 8, seed=13),
    "chunglu": lambda: gg.chung_lu(120000, 2.1, 12.0, seed=14),
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_laplacian_apply_fp64(P, name):
    g = GRAPHS[name]()
    ctx = P.Context.from_graph(g)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(g.n)
    y = ctx.laplacian_apply(_dev(x)).cpu().numpy()
    ref = O.laplacian_apply(g, x)
    # dot-product error bound: |dy| <= gamma_{d+1} sum_j |L_ij x_j|
    absL = O.laplacian(g)
    absL.data = np.abs(absL.data)
    bound = (g.counts().max() + 2) * 2.0 ** -53 * 1.01 * (absL @ np.abs(x))
    assert np.all(np.abs(y - ref) <= bound + 1e-300)
    inf = ctx.info()
    assert inf["n"] == g.n and inf["nnz"] == g.nnz
    assert inf["trim_index"] == O.trim_index(O.degrees(g))
    # weighted degrees: only the summation order differs from the oracle's
    assert inf["delta_default"] == pytest.approx(O.deflation_shift(O.degrees(g)), rel=4e-16 * g.counts().max())


def _big_power_law(weighted):
    # more than 2^20 vertices in degree order (the hub-cached shape) with rows split into
    # many chunks; weights, when asked for, are a symmetric hash of the edge's end points
    # mapped to [0.5, 1.5)
    g = gg.rmat(21, 16, seed=77, device="cpu")
    if weighted:
        rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
        a = np.minimum(rows, g.col.astype(np.int64))
        b = np.maximum(rows, g.col.astype(np.int64))
        h = (a * 2654435761 + b * 40503) % 1000003
        g = gg.CSRGraph(g.n, g.row_ptr, g.col, 0.5 + h / 1000003.0, name=g.name + "_w")
    return g


@pytest.mark.parametrize("weighted", [False, True])
def test_laplacian_apply_large_power_law(P, weighted):
    """The product on an R-MAT scale-21 graph (1.2 M vertices, hub rows of 100 K entries) in
    FP64 and FP32 against the oracle's Laplacian, within the dot-product error bounds."""
    g = _big_power_law(weighted)
    assert g.n > (1 << 20) and g.counts().max() > 8 * 8192
    print(f"large power-law product: n={g.n} nnz={g.nnz} weighted={weighted}", flush=True)
    ctx = P.Context.from_graph(g)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(g.n)
    ref = O.laplacian_apply(g, x)
    absL = O.laplacian(g)
    absL.data = np.abs(absL.data)
    mag = absL @ np.abs(x)
    y = ctx.laplacian_apply(_dev(x)).cpu().numpy()
    bound = (g.counts().max() + 2) * 2.0 ** -53 * 1.01 * mag
    assert np.all(np.abs(y - ref) <= bound + 1e-300)
    x32 = x.astype(np.float32)
    y32 = ctx.laplacian_apply_f32(_dev(x32, torch.float32)).cpu().numpy().astype(np.float64)
    ref32 = O.laplacian_apply(g, x32.astype(np.float64))
    bound32 = (g.counts().max() + 4) * 2.0 ** -24 * 1.01 * (absL @ np.abs(x32.astype(np.float64)))
    assert np.all(np.abs(y32 - ref32) <= bound32)


@pytest.mark.parametrize("name", ["grid3d_w", "rmat14", "hubs", "rmat17", "chunglu"])
def test_laplacian_apply_fp32(P, name):
    g = GRAPHS[name]()
    ctx = P.Context.from_graph(g)
    x = np.random.default_rng(2).standard_normal(g.n).astype(np.float32)
    y = ctx.laplacian_apply_f32(_dev(x, torch.float32)).cpu().numpy().astype(np.float64)
    ref = O.laplacian_apply(g, x.astype(np.float64))
    absL = O.laplacian(g)
    absL.data = np.abs(absL.data)
    # FP32 weights/degrees (relative 2^-24 each) plus FP32 accumulation of d+1 terms
    bound = (g.counts().max() + 4) * 2.0 ** -24 * 1.01 * (absL @ np.abs(x.astype(np.float64)))
    assert np.all(np.abs(y - ref) <= bound)


@pytest.mark.parametrize("case", [
    dict(g="grid64", c=0, sigma=0.0, trim=None),
    dict(g="grid3d_w", c=3, sigma=0.0, trim=None),
    dict(g="rmat14", c=5, sigma=0.0, trim=None),
    dict(g="rmat14", c=2, sigma="half", trim=17),
    dict(g="hubs", c=9, sigma="half", trim=None),
    dict(g="rmat17", c=6, sigma=0.0, trim=None),
], ids=["grid64", "grid3d_c3", "rmat14_c5", "rmat14_shift_trim17", "hubs_c9_shift", "rmat17_c6"])
def test_inner_solve_fp64(P, case):
    g = GRAPHS[case["g"]]()
    ctx = P.Context.from_graph(g)
    L = O.laplacian(g)
    d = O.degrees(g)
    # deflation vectors: accurate low eigenvectors from the oracle's own solve
    c = case["c"]
    res = O.isira(g, max(c, 1), 0.0, 1e-9, gg.start_block(g.n, 4, 3), inner_rtol=1e-8)
    V = res.evecs[:, :c]
    # sigma below lambda_1 <= lambda_{c+1} keeps the trimmed operator (2.15) SPD
    sigma = 0.5 * res.evals[0] if case["sigma"] == "half" else 0.0
    i = O.trim_index(d) if case["trim"] is None else case["trim"]
    delta = O.deflation_shift(d)
    r = np.random.default_rng(4).standard_normal(g.n)
    r -= r.mean()
    z_ref, its_ref, _ = O.inner_solve(L, d, r, i, sigma, delta, V, 1e-12, 20000)
    z, its, rel = ctx.inner_solve(_dev(r), _dev(V.T) if c else None, sigma=sigma, delta=delta,
                                  trim=i, rtol=1e-12, max_it=20000, prec=P.isira.FP64)
    z = z.cpu().numpy()
    assert rel <= 1e-12
    assert abs(its - its_ref) <= max(3, 0.05 * its_ref)
    assert abs(z.sum()) <= 1e-10 * np.abs(z).max()
    assert np.linalg.norm(z - z_ref) <= 1e-8 * np.linalg.norm(z_ref)


@pytest.mark.parametrize("case", [
    dict(g="rmat14", c=3, where="between"),   # one negative eigenvalue of K-hat
    dict(g="grid3d_w", c=2, where="between"),
    dict(g="rmat14", c=2, where="below"),     # SPD: MINRES and PCG reach the same solution
], ids=["rmat14_indefinite", "grid3d_indefinite", "rmat14_spd"])
def test_inner_solve_minres(P, case):
    """Preconditioned MINRES on the trimmed deflated system (2.15) against the oracle's MINRES,
    with sigma between lambda_{c+1} and lambda_{c+2} (indefinite, Thm 2.8) or below."""
    g = GRAPHS[case["g"]]()
    ctx = P.Context.from_graph(g)
    L = O.laplacian(g)
    d = O.degrees(g)
    c = case["c"]
    res = O.isira(g, c + 2, 0.0, 1e-10, gg.start_block(g.n, 4, 3), inner_rtol=1e-8)
    order = np.argsort(res.evals)
    V = res.evecs[:, order[:c]]  # the c smallest: deflated, lambda_{c+1..c+2} remain lowest
    lam = res.evals[order]
    sigma = 0.5 * (lam[c] + lam[c + 1]) if case["where"] == "between" else 0.5 * lam[0]
    i = O.trim_index(d)
    delta = O.deflation_shift(d)
    r = np.random.default_rng(6).standard_normal(g.n)
    r -= r.mean()
    z_ref, its_ref, rel_ref = O.inner_solve(L, d, r, i, sigma, delta, V, 1e-12, 20000, solver="minres")
    z, its, rel = ctx.inner_solve(_dev(r), _dev(V.T), sigma=sigma, delta=delta, trim=i, rtol=1e-12,
                                  max_it=20000, prec=P.isira.FP64, solver=P.isira.SOLVER_MINRES)
    z = z.cpu().numpy()
    assert rel <= 1e-12 and rel_ref <= 1e-12
    assert abs(its - its_ref) <= max(3, 0.05 * its_ref)
    assert abs(z.sum()) <= 1e-9 * np.abs(z).max()
    assert np.linalg.norm(z - z_ref) <= 1e-7 * np.linalg.norm(z_ref)
    # the solved system itself
    Kz = L @ z + delta * V @ (V.T @ z) - sigma * z
    assert np.linalg.norm(Kz - r) <= 1e-8 * np.linalg.norm(r) * max(1.0, np.abs(z).max())
    if case["where"] == "below":
        zp, _, _ = ctx.inner_solve(_dev(r), _dev(V.T), sigma=sigma, delta=delta, trim=i, rtol=1e-12,
                                   max_it=20000, prec=P.isira.FP64)
        assert np.linalg.norm(zp.cpu().numpy() - z) <= 1e-8 * np.linalg.norm(z)
    # FP32 MINRES: the recursion reaches a loose tolerance
    z32, its32, rel32 = ctx.inner_solve(_dev(r), _dev(V.T), sigma=sigma, delta=delta, trim=i, rtol=1e-4,
                                        max_it=20000, prec=P.isira.FP32, solver=P.isira.SOLVER_MINRES)
    assert rel32 <= 1e-4


@pytest.mark.parametrize("name,k", [("grid64", 8), ("rmat14", 10), ("grid3d_w", 8)])
def test_solve_moving_shift(P, name, k):
    """Algorithm 3.2 with the purge step's moving shift (sigma <- theta_2, MINRES inner
    solves) against the oracle run the same way."""
    g = GRAPHS[name]()
    ctx = P.Context.from_graph(g)
    U0 = gg.start_block(g.n, 4, 2)
    ev, X, resid, st = ctx.solve(k, 0.0, 1e-9, u0=U0, shift_mode=P.isira.SHIFT_MOVING)
    assert st["sigma_last"] > 0.0
    res_o = O.isira(g, k, 0.0, 1e-9, U0, inner_rtol=1e-6, moving_shift=True)
    _compare(res_o, ev, X.cpu().numpy(), resid, g, 1e-9)


def test_inner_solve_fp32_accuracy(P):
    g = GRAPHS["rmat14"]()
    ctx = P.Context.from_graph(g)
    L = O.laplacian(g)
    d = O.degrees(g)
    res = O.isira(g, 3, 0.0, 1e-9, gg.start_block(g.n, 4, 3), inner_rtol=1e-8)
    V = res.evecs
    r = np.random.default_rng(5).standard_normal(g.n)
    r -= r.mean()
    i = O.trim_index(d)
    z_ref, _, _ = O.inner_solve(L, d, r, i, 0.0, O.deflation_shift(d), V, 1e-12, 20000)
    z, its, rel = ctx.inner_solve(_dev(r), _dev(V.T), rtol=1e-4, max_it=5000, prec=P.isira.FP32)
    z = z.cpu().numpy()
    assert rel <= 1e-4
    # the inexact solve is accurate to about rtol times the condition number in K-norm;
    # check the true residual of the constrained system instead
    Lt = L @ z + O.deflation_shift(d) * V @ (V.T @ z)
    assert np.linalg.norm(Lt - r) <= 2e-3 * np.linalg.norm(r)


# from no basis column to the widest basis of a k = 64 solve; the graph size is not a
# multiple of the 512-row tile of the column dots
@pytest.mark.parametrize("ncols", [0, 3, 12, 127, 128, 129, 190])
def test_orthonormalize(P, ncols):
    g = GRAPHS["rmat14"]()
    assert g.n % 64 != 0
    ctx = P.Context.from_graph(g)
    rng = np.random.default_rng(6 + ncols)
    Q = np.linalg.qr(rng.standard_normal((g.n, max(ncols, 1))))[0][:, :ncols]
    Q -= Q.mean(axis=0)
    Q = np.linalg.qr(Q)[0] if ncols else Q
    z = rng.standard_normal(g.n) + Q @ rng.standard_normal(ncols) * 100 + 50.0
    u, norms = ctx.orthonormalize(_dev(Q.T) if ncols else None, _dev(z))
    u = u.cpu().numpy()
    Qo = np.column_stack([Q, np.ones(g.n) / math.sqrt(g.n)])
    ref, before, after = O.cgs2(Qo, z)
    assert norms[0] == pytest.approx(before, rel=1e-13)
    assert norms[1] == pytest.approx(after, rel=1e-10)
    assert np.allclose(u, ref / after, atol=1e-13)
    assert np.abs(Qo.T @ u).max() <= 1e-14


# ---------------------------------------------------------------------- full solves


def _compare(res_o, ev, X, resid, g, tol, rel=1e-9):
    k = len(ev)
    assert k == res_o.converged
    assert np.allclose(np.sort(ev), np.sort(res_o.evals), rtol=rel, atol=0)
    assert np.abs(X @ X.T - np.eye(k)).max() <= 1e-10
    assert np.abs(X.sum(axis=1)).max() <= 1e-9
    L = O.laplacian(g)
    for j in range(k):
        r_true = np.linalg.norm(L @ X[j] - ev[j] * X[j])
        assert r_true <= tol and resid[j] <= tol
        assert abs(r_true - resid[j]) <= 1e-3 * tol + 1e-14


def test_solve_grid64_closed_form(P):
    g = gg.grid2d(64, 64)
    ctx = P.Context.from_graph(g)
    U0 = gg.start_block(g.n, 4, 1)
    ev, X, resid, st = ctx.solve(10, 0.0, 1e-10, u0=U0)
    X = X.cpu().numpy()
    i, j = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    lam = np.sort((4 * np.sin(i * np.pi / 128) ** 2 + 4 * np.sin(j * np.pi / 128) ** 2).ravel())[1:11]
    assert st["n_converged"] == 10
    assert np.allclose(np.sort(ev), lam, rtol=1e-9, atol=0)
    res_o = O.isira(g, 10, 0.0, 1e-10, U0, inner_rtol=1e-10)
    _compare(res_o, ev, X, resid, g, 1e-10)
    # sign convention: largest-magnitude entry positive
    for x in X:
        assert x[np.argmax(np.abs(x))] > 0


@pytest.mark.parametrize("prec", [0, 1])
def test_solve_whisker_closed_form(P, prec):
    """R-MAT-style whiskers in miniature (K_12 with two leaves and two 2-paths on one
    vertex): the solve reaches the closed-form eigenvalues (3 - sqrt 5) / 2 and 1 (twice)."""
    g = gg.whiskered_clique(12)
    ctx = P.Context.from_graph(g)
    # 18 vertices: the basis must stay below n - 1 - k columns
    ev, X, resid, st = ctx.solve(4, 0.0, 1e-11, u0=gg.start_block(g.n, 2, 4), inner_prec=prec,
                                 q=6, m=12)
    ev = np.sort(ev)
    golden = (3.0 - math.sqrt(5.0)) / 2.0
    assert st["n_converged"] == 4
    assert abs(ev[0] - golden) <= 1e-10 * golden
    assert np.sum(np.abs(ev - 1.0) <= 1e-10) == 2
    assert resid.max() <= 1e-11


@pytest.mark.parametrize("case", [
    dict(g=lambda: gg.random_connected(3000, 4000, seed=31), k=8, sigma=0.0, q=12, m=20, prec=0),
    dict(g=lambda: gg.random_connected(2500, 6000, seed=32, weights=(0.5, 1.5)), k=6, sigma=0.0, q=None, m=None, prec=0),
    dict(g=lambda: gg.rmat(12, 8, seed=3), k=12, sigma="half", q=None, m=None, prec=0),
    dict(g=lambda: gg.rmat(12, 8, seed=3), k=12, sigma=0.0, q=16, m=24, prec=1),
    dict(g=lambda: gg.grid3d(12, 11, 10, weights=(0.5, 1.5), seed=3), k=8, sigma=0.0, q=None, m=None, prec=1),
], ids=["rand3000_restart", "rand2500w", "rmat12_shift", "rmat12_fp32_restart", "grid3d_w_fp32"])
def test_solve_matches_dense(P, case):
    g = case["g"]()
    k = case["k"]
    Ld = O.laplacian(g).toarray()
    lam = np.linalg.eigvalsh(Ld)
    sigma = 0.5 * lam[1] if case["sigma"] == "half" else 0.0
    ctx = P.Context.from_graph(g)
    U0 = gg.start_block(g.n, 4, 5)
    tol = 1e-9
    opts = {}
    if case["q"]:
        opts.update(q=case["q"], m=case["m"])
    ev, X, resid, st = ctx.solve(k, sigma, tol, u0=U0, inner_prec=case["prec"], **opts)
    X = X.cpu().numpy()
    assert st["n_converged"] == k
    assert np.allclose(np.sort(ev), lam[1:k + 1], rtol=1e-9, atol=0)
    for j in range(k):
        assert np.linalg.norm(Ld @ X[j] - ev[j] * X[j]) <= tol
    assert np.abs(X @ X.T - np.eye(k)).max() <= 1e-10
    assert np.abs(X.sum(axis=1)).max() <= 1e-9


def test_solve_rmat14_vs_oracle(P):
    g = gg.rmat(14, 8, seed=11)
    ctx = P.Context.from_graph(g)
    U0 = gg.start_block(g.n, 4, 2)
    ev, X, resid, st = ctx.solve(16, 0.0, 1e-9, u0=U0)
    res_o = O.isira(g, 16, 0.0, 1e-9, U0, inner_rtol=1e-6)
    _compare(res_o, ev, X.cpu().numpy(), resid, g, 1e-9)


@pytest.mark.parametrize("name,k", [("rmat12", 8), ("grid3d_w", 6)])
def test_default_start_block_is_the_oracle_generator(P, name, k):
    """Without a start block the library draws column j from the replacement generator of
    the orthonormalization step: SplitMix64(seed) at counters j*n + (caller label), mapped
    to [-1, 1).  The oracle's replacement_vector (pinned on the CPU to the published
    SplitMix64 outputs) gives those columns, so a solve started from them as an explicit
    block must be bit-identical to the solve without one, and both reach the oracle's
    eigenvalues from that block."""
    g = gg.rmat(12, 8, seed=3) if name == "rmat12" else GRAPHS[name]()
    ctx = P.Context.from_graph(g)
    seed, k0 = 987654321, 4
    U0 = np.column_stack([O.replacement_vector(g.n, seed, j) for j in range(k0)])
    print(f"default start block: {name} n={g.n} k={k} seed={seed}", flush=True)
    ev_a, X_a, r_a, st_a = ctx.solve(k, 0.0, 1e-9, seed=seed, k0=k0)
    ev_b, X_b, r_b, st_b = ctx.solve(k, 0.0, 1e-9, u0=U0, seed=seed)
    assert st_a["n_converged"] == k and st_b["n_converged"] == k
    assert st_a["outer_total"] == st_b["outer_total"]
    assert st_a["inner_total"] == st_b["inner_total"]
    assert np.array_equal(ev_a, ev_b) and np.array_equal(r_a, r_b)
    assert torch.equal(X_a, X_b)
    res_o = O.isira(g, k, 0.0, 1e-9, U0, inner_rtol=1e-6, seed=seed)
    _compare(res_o, ev_a, X_a.cpu().numpy(), r_a, g, 1e-9)


@pytest.mark.parametrize("which", ["max_degree", "min_degree", "label0"])
def test_solve_trim_index_choices(P, which):
    """Thm 2.4: the enlarged inner solution does not depend on the trimmed vertex, so every
    trim choice (the paper's Table 2 compares a degree-1 vertex, vertex 1 and the
    maximum-degree vertex) reaches the same eigenpairs; the oracle runs with the same one."""
    g = gg.rmat(13, 8, seed=12)
    d = O.degrees(g)
    trim = {"max_degree": int(np.argmax(d)), "min_degree": int(np.argmin(d)), "label0": 0}[which]
    ctx = P.Context.from_graph(g)
    U0 = gg.start_block(g.n, 4, 3)
    ev, X, resid, st = ctx.solve(10, 0.0, 1e-9, u0=U0, trim_index=trim)
    assert st["trim_index"] == trim
    res_o = O.isira(g, 10, 0.0, 1e-9, U0, inner_rtol=1e-6, trim=trim)
    _compare(res_o, ev, X.cpu().numpy(), resid, g, 1e-9)


def test_solve_without_rank_one_term(P):
    """Remark 3.1: with sigma > 0 the inner operator may leave out (sigma/n) 1-hat 1-hat^T;
    the GPU with that option matches the oracle run the same way, and both reach the
    eigenpairs of the exact method."""
    g = gg.rmat(11, 8, seed=15)
    d = O.degrees(g)
    i = O.trim_index(d)
    Lhat = O.trimmed_matrix(O.laplacian(g), i).toarray()
    sigma = 0.5 * np.linalg.eigvalsh(Lhat).min()  # keeps L-hat - sigma I positive definite
    ctx = P.Context.from_graph(g)
    U0 = gg.start_block(g.n, 4, 5)
    ev, X, resid, st = ctx.solve(8, sigma, 1e-9, u0=U0, drop_rank_one=1)
    res_o = O.isira(g, 8, sigma, 1e-9, U0, inner_rtol=1e-6, rank_one=False)
    _compare(res_o, ev, X.cpu().numpy(), resid, g, 1e-9)
    ev_exact, _, _, _ = ctx.solve(8, sigma, 1e-9, u0=U0)
    assert np.allclose(np.sort(ev), np.sort(ev_exact), rtol=1e-9, atol=0)


def test_solve_errors(P):
    g = gg.grid2d(8, 8)
    ctx = P.Context.from_graph(g)
    with pytest.raises(P.IsiraError) as e:
        ctx.solve(0)
    assert e.value.code == P.isira.ISIRA_E_ARG
    with pytest.raises(P.IsiraError) as e:
        ctx.solve(3, sigma=2.5)  # >= min degree 2
    assert e.value.code == P.isira.ISIRA_E_ARG
    with pytest.raises(P.IsiraError) as e:
        ctx.solve(3, precond=P.isira.PC_LEARNED)
    assert e.value.code == P.isira.ISIRA_E_PRECOND
    # max_outer cap: partial result, NOT_CONVERGED
    ev, X, resid, st = ctx.solve(5, 0.0, 1e-12, max_outer=3, u0=gg.start_block(g.n, 4, 1))
    assert st["return_code"] == P.isira.ISIRA_NOT_CONVERGED
    assert len(ev) == st["n_converged"] < 5
