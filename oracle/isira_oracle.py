"""Plain FP64 CPU oracle of iSIRA (Huang, Lin, Lu, Yau, arXiv 1710.07080).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
module: only the tests, the smoke check and the bench's CPU-baseline leg use it.  It shares
no code with the GPU library; both read the same seeded inputs from ``graphgen``.

Every routine is written to be checked against the paper by eye: trimmed vectors are
really of length n-1 (entry i deleted), the deflated operator is applied term by term,
and the outer loop follows Algorithm 3.2 step by step.  Library primitives used as
steps: scipy CSR matrix-vector products, numpy dense products, ``numpy.linalg.eigh``
for the small Rayleigh-Ritz problem.

Readings of points the paper leaves open (each also listed in the design notes):
  * inner solver = PCG on the SPD trimmed system, stopped at ||r|| <= rtol ||b||;
  * the shift sigma is fixed for the whole solve (0 <= sigma < lambda_1); the purge step's
    moving shift is an option (sigma <- theta_2 after each lock, inner solver MINRES);
  * the rank-one term (sigma/n) 1 1^T of eq. (2.15) is kept in the operator and
    dropped from the preconditioner (Remark 3.1 applied to the preconditioner only);
  * W is carried incrementally (one new column per expansion);
  * a Ritz pair is locked only when a fresh residual ||L y - theta y|| also passes;
  * orthonormalization is classical Gram-Schmidt applied twice against [U V 1/sqrt(n)];
  * the trim index is argmax diag(L) with the lowest index on ties.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np
import scipy.sparse as sp

# ----------------------------------------------------------------------------------------
# Graph Laplacian (Section 1.1, eq. (1.1); Remark 1.3 for positive edge weights)
# ----------------------------------------------------------------------------------------


def adjacency(g) -> sp.csr_matrix:
    """W (or A for unit weights) as a scipy CSR matrix, from the off-diagonal CSR."""
    vals = np.ones(g.nnz) if g.w is None else np.asarray(g.w, dtype=np.float64)
    return sp.csr_matrix((vals, g.col.astype(np.int64), g.row_ptr.astype(np.int64)), shape=(g.n, g.n))


def degrees(g) -> np.ndarray:
    """D_ii = sum_j W_ij (Section 1.1; weighted degree of Remark 1.3)."""
    return np.asarray(adjacency(g).sum(axis=1)).ravel()


def laplacian(g) -> sp.csr_matrix:
    """L = D - W (eq. (1.1))."""
    W = adjacency(g)
    return (sp.diags(degrees(g)) - W).tocsr()


def laplacian_apply(g, x: np.ndarray) -> np.ndarray:
    """y = L x = D x - W x."""
    return degrees(g) * x - adjacency(g) @ x


# ----------------------------------------------------------------------------------------
# Hyper-parameters (Remark 4.1)
# ----------------------------------------------------------------------------------------


def trim_index(d: np.ndarray) -> int:
    """Remark 4.1(i): trim the vertex of maximum degree (lowest index among ties)."""
    return int(np.argmax(d))  # numpy argmax returns the first maximum


def deflation_shift(d: np.ndarray) -> float:
    """Remark 4.1(ii): delta = 2 * max diag(L) (Gershgorin)."""
    return 2.0 * float(np.max(d))


# ----------------------------------------------------------------------------------------
# Trimming (Section 2.1, Theorems 2.2 and 2.4) and the trimmed shifted deflated
# system (Section 2.3, Theorem 2.8, eq. (2.15))
# ----------------------------------------------------------------------------------------


def trim(x: np.ndarray, i: int) -> np.ndarray:
    """Delete the i-th entry (or row) -- the hat operation of Theorems 2.4 and 2.8."""
    return np.delete(x, i, axis=0)


def trimmed_matrix(L: sp.csr_matrix, i: int) -> sp.csr_matrix:
    """L-hat: L with row i and column i removed (eq. (2.3))."""
    keep = np.concatenate([np.arange(i), np.arange(i + 1, L.shape[0])])
    return L[keep][:, keep].tocsr()


def enlarge(zhat: np.ndarray, i: int, n: int) -> np.ndarray:
    """eq. (2.5): insert a zero at position i, then subtract (1^T zhat / n) * 1_n."""
    z = np.insert(zhat, i, 0.0)
    return z - (np.sum(zhat) / n) * np.ones(n)


def trimmed_operator(Lhat: sp.csr_matrix, n: int, sigma: float, delta: float,
                     Vhat: np.ndarray, rank_one: bool = True) -> Callable[[np.ndarray], np.ndarray]:
    """K-hat of eq. (2.15):  (L-hat - sigma I) + (sigma/n) 1 1^T + delta V-hat V-hat^T,
    acting on (n-1)-vectors.  With V empty and sigma = 0 this is eq. (2.4).
    ``rank_one=False`` leaves out the (sigma/n) 1 1^T term, as Remark 3.1 allows."""

    def apply(x: np.ndarray) -> np.ndarray:
        y = Lhat @ x - sigma * x
        if rank_one:
            y = y + (sigma / n) * np.sum(x) * np.ones_like(x)
        if Vhat.shape[1] > 0:
            y = y + delta * (Vhat @ (Vhat.T @ x))
        return y

    return apply


def jacobi_smw_preconditioner(dhat: np.ndarray, sigma: float, delta: float,
                              Vhat: np.ndarray) -> Callable[[np.ndarray], np.ndarray]:
    """Remark 3.2 with M-hat_sigma = diag(d-hat - sigma) and, when V is non-empty, the
    Sherman-Morrison-Woodbury inverse of eq. (3.5):
        (M + delta V V^T)^{-1} = (I - delta M^{-1} V (I_c + delta V^T M^{-1} V)^{-1} V^T) M^{-1}.
    The rank-one term of eq. (2.15) is not included (Remark 3.1)."""
    minv = 1.0 / (dhat - sigma)
    return smw_preconditioner(lambda x: minv * x, delta, Vhat)


def smw_preconditioner(apply_minv: Callable[[np.ndarray], np.ndarray], delta: float,
                       Vhat: np.ndarray) -> Callable[[np.ndarray], np.ndarray]:
    """eq. (3.5) for a preconditioner given by the action of M^{-1} (an SPD operator)."""
    c = Vhat.shape[1]
    if c == 0:
        return apply_minv
    Y = np.column_stack([apply_minv(Vhat[:, j]) for j in range(c)])  # M^{-1} V
    G = np.eye(c) + delta * (Vhat.T @ Y)

    def apply(x: np.ndarray) -> np.ndarray:
        y = apply_minv(x)
        return y - delta * (Y @ np.linalg.solve(G, Vhat.T @ y))

    return apply


def pcg(apply_A, b: np.ndarray, apply_P, rtol: float, maxit: int):
    """Textbook preconditioned conjugate gradients from x0 = 0, stopped when the
    recursively updated residual satisfies ||r|| <= rtol * ||b||.
    Returns (x, iterations, relative residual of the recursion)."""
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    r = b.copy()
    z = apply_P(r)
    p = z.copy()
    rho = r @ z
    it = 0
    rel = 1.0
    while it < maxit:
        it += 1
        q = apply_A(p)
        alpha = rho / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        rel = np.linalg.norm(r) / bnorm
        if rel <= rtol:
            break
        z = apply_P(r)
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    return x, it, rel


def minres(apply_A, b: np.ndarray, apply_P, rtol: float, maxit: int):
    """Preconditioned MINRES (Paige and Saunders, SIAM J. Numer. Anal. 12 (1975); the
    preconditioned form as in Elman, Silvester and Wathen's book) for a symmetric, possibly
    indefinite A with an SPD preconditioner P, from x0 = 0.  Each step extends the Lanczos
    basis of the P-inner product by one vector, updates the QR factorization of the
    tridiagonal Lanczos matrix by one Givens rotation, and updates x along the new
    direction; eta is the P^{-1}-norm of the residual, recursively updated.  Stopped when
    |eta| <= rtol * eta_0.  Returns (x, iterations, |eta| / eta_0)."""
    x = np.zeros_like(b)
    v_old = np.zeros_like(b)
    v = b.copy()
    z = apply_P(v)
    gamma = math.sqrt(max(0.0, v @ z))
    if gamma == 0.0:
        return x, 0, 0.0
    eta0 = eta = gamma
    gamma_old = 1.0
    c_old = c = 1.0
    s_old = s = 0.0
    w_old = np.zeros_like(b)
    w = np.zeros_like(b)
    it = 0
    rel = 1.0
    while it < maxit:
        it += 1
        z = z / gamma
        Az = apply_A(z)
        dlt = Az @ z
        v_new = Az - (dlt / gamma) * v - (gamma / gamma_old) * v_old
        z_new = apply_P(v_new)
        gamma_new = math.sqrt(max(0.0, v_new @ z_new))
        a0 = c * dlt - c_old * s * gamma
        a1 = math.hypot(a0, gamma_new)
        a2 = s * dlt + c_old * c * gamma
        a3 = s_old * gamma
        c_old, s_old = c, s
        c, s = a0 / a1, gamma_new / a1
        w_new = (z - a3 * w_old - a2 * w) / a1
        x = x + (c * eta) * w_new
        eta = -s * eta
        rel = abs(eta) / eta0
        v_old, v = v, v_new
        w_old, w = w, w_new
        gamma_old, gamma = gamma, gamma_new
        z = z_new
        if rel <= rtol or gamma == 0.0:
            break
    return x, it, rel


def inner_solve(L: sp.csr_matrix, d: np.ndarray, r: np.ndarray, i: int, sigma: float,
                delta: float, V: np.ndarray, rtol: float, maxit: int,
                apply_minv_hat: Optional[Callable] = None, Lhat: Optional[sp.csr_matrix] = None,
                rank_one: bool = True, solver: str = "pcg"):
    """Subspace expansion of Algorithm 3.2: (i) solve the trimmed system (eq. (2.4) when
    V is empty and sigma = 0, eq. (2.15) otherwise) with the Remark 3.2 preconditioner,
    (ii) enlarge by eq. (2.5).  The right-hand side r must be orthogonal to 1 (Lemma 2.1).
    ``apply_minv_hat`` replaces the Jacobi M^{-1} by another SPD approximate inverse of
    L-hat - sigma I acting on (n-1)-vectors.  ``solver="minres"`` solves with preconditioned
    MINRES instead of PCG, for a shift that makes the trimmed system indefinite (Thm 2.8).
    Returns (z*, iterations, relative residual)."""
    n = L.shape[0]
    if Lhat is None:
        Lhat = trimmed_matrix(L, i)
    Vhat = trim(V, i)
    rhat = trim(r, i)
    A = trimmed_operator(Lhat, n, sigma, delta, Vhat, rank_one)
    if apply_minv_hat is None:
        P = jacobi_smw_preconditioner(trim(d, i), sigma, delta, Vhat)
    else:
        P = smw_preconditioner(apply_minv_hat, delta, Vhat)
    if solver == "minres":
        zhat, its, rel = minres(A, rhat, P, rtol, maxit)
    else:
        zhat, its, rel = pcg(A, rhat, P, rtol, maxit)
    return enlarge(zhat, i, n), its, rel


# ----------------------------------------------------------------------------------------
# Orthonormalization and the counter-based replacement generator
# ----------------------------------------------------------------------------------------

_GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64(seed: int, counters) -> np.ndarray:
    """SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) as a counter-based generator: output
    number c (c = 0, 1, ...) is the mixing function applied to seed + (c + 1) * golden-gamma,
    which is the c-th output of the sequential generator started from ``seed``."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (c + np.uint64(1)) * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_uniform(seed: int, counters) -> np.ndarray:
    """The top 53 bits of SplitMix64 output mapped to [-1, 1)."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def replacement_vector(n: int, seed: int, draw: int) -> np.ndarray:
    """Entry l of replacement vector number ``draw`` is the generator at counter draw*n + l."""
    return splitmix64_uniform(seed, np.uint64(draw) * np.uint64(n) + np.arange(n, dtype=np.uint64))


def cgs2(Q: np.ndarray, z: np.ndarray):
    """Classical Gram-Schmidt applied twice against the orthonormal columns of Q.
    Returns (z orthogonalized, ||z|| before, ||z|| after)."""
    before = np.linalg.norm(z)
    for _ in range(2):
        z = z - Q @ (Q.T @ z)
    return z, before, np.linalg.norm(z)


# ----------------------------------------------------------------------------------------
# Algorithm 3.2 (iSIRA)
# ----------------------------------------------------------------------------------------


@dataclasses.dataclass
class IsiraResult:
    evals: np.ndarray
    evecs: np.ndarray
    resid: np.ndarray  # ||L v - lambda v||_2, fresh FP64 products
    converged: int
    outer_its: list  # per eigenpair
    inner_its: list  # per eigenpair (sum of PCG iterations)
    trim_index: int
    delta: float
    restarts: int = 0
    breakdowns: int = 0
    refreshes: int = 0
    history: list = dataclasses.field(default_factory=list)  # ||r|| per outer iteration
    # per outer iteration: (seconds, inner iterations, basis width + locked pairs, seconds of
    # its inner solve); set-up seconds before the first one (timing records for cost models,
    # no arithmetic)
    outer_log: list = dataclasses.field(default_factory=list)
    setup_seconds: float = 0.0


def isira(g, k: int, sigma: float, tol: float, U0: np.ndarray, *, m: Optional[int] = None,
          q: Optional[int] = None, inner_rtol: float = 1e-12, max_inner: int = 5000,
          max_outer: int = 100000, trim: Optional[int] = None, delta: Optional[float] = None,
          seed: int = 12345, apply_minv_hat_factory: Optional[Callable] = None,
          time_budget: Optional[float] = None, rank_one: bool = True,
          moving_shift: bool = False) -> IsiraResult:
    """Algorithm 3.2 with the readings listed in the module docstring.

    k: number of wanted eigenpairs (d in Algorithm 3.2); U0: n-by-k0 start block, whose
    column means are removed before orthonormalization; q, m: restart size and maximal
    subspace dimension (defaults q = k + 10, m = 2 q).
    ``apply_minv_hat_factory(i, sigma)`` may return an SPD approximate inverse of
    L-hat - sigma I on (n-1)-vectors to replace the Jacobi preconditioner.
    ``time_budget`` (seconds) stops the loop early; the partial result is returned.
    ``rank_one=False`` drops (sigma/n) 1 1^T from the inner operator (Remark 3.1).
    ``moving_shift=True`` follows the purge step's "move sigma to about theta_2": after each
    locked pair sigma becomes the smallest remaining Ritz value, capped at half the minimum
    degree (the Jacobi part of the preconditioner stays SPD); the trimmed system may then be
    indefinite, so every inner solve of such a run uses preconditioned MINRES."""
    import time as _time

    t_start = _time.perf_counter()
    n = g.n
    L = laplacian(g)
    dvec = degrees(g)
    q = k + 10 if q is None else q
    m = 2 * q if m is None else m
    if not (1 <= k <= q < m):
        raise ValueError("need 1 <= k <= q < m")
    i = trim_index(dvec) if trim is None else int(trim)
    dl = deflation_shift(dvec) if delta is None else float(delta)
    sigma_cap = 0.5 * float(np.min(dvec))
    if moving_shift and apply_minv_hat_factory is not None:
        raise ValueError("a preconditioner built for one shift cannot follow a moving shift")
    ones = np.ones(n) / math.sqrt(n)
    minv_hat = None if apply_minv_hat_factory is None else apply_minv_hat_factory(i, sigma)
    Lhat = trimmed_matrix(L, i)

    # orthonormal start block, each column orthogonal to 1 (REQUIRE of Algorithm 3.2)
    cols = []
    draws = 0
    breakdowns = 0
    for j in range(U0.shape[1]):
        z = U0[:, j] - np.mean(U0[:, j])
        Q = np.column_stack(cols + [ones])
        z, before, after = cgs2(Q, z)
        while after <= 1e-10 * before:
            breakdowns += 1
            z, before, after = cgs2(Q, replacement_vector(n, seed, draws))
            draws += 1
        cols.append(z / after)
    U = np.column_stack(cols)
    V = np.zeros((n, 0))
    W = np.column_stack([L @ U[:, j] for j in range(U.shape[1])])  # W = (L + delta V V^T) U, V empty
    H = U.T @ W
    H = 0.5 * (H + H.T)
    evals, evecs, outer_its, inner_its, history = [], [], [], [], []
    restarts = refreshes = 0
    outer = 0
    # timing records (no arithmetic): per outer iteration its seconds, inner iterations, the
    # columns of U and V it worked with, and the seconds of its inner solve
    setup_s = _time.perf_counter() - t_start
    log, mark = [], None
    inner_clock = [0.0]

    def tick(inner_so_far, cols):
        nonlocal mark
        now = _time.perf_counter()
        if mark is not None:
            log.append((now - mark[0], inner_so_far - mark[1], mark[2], inner_clock[0] - mark[3]))
        mark = (now, inner_so_far, cols, inner_clock[0])

    def done(res):
        res.outer_log, res.setup_seconds = log, setup_s
        return res

    for _j in range(k):
        its_here = 0
        inner_here = 0
        locked = False
        while not locked:
            tick(sum(inner_its) + inner_here, U.shape[1] + V.shape[1])
            if outer >= max_outer or (time_budget is not None and _time.perf_counter() - t_start > time_budget):
                return done(_finish(L, evals, evecs, outer_its + [its_here], inner_its + [inner_here], i, dl,
                                    restarts, breakdowns, refreshes, history, partial=True))
            outer += 1
            its_here += 1
            # subspace extraction: all eigenpairs of H, ascending, unit eigenvectors
            theta, S = np.linalg.eigh(H)
            s1 = S[:, 0]
            y = U @ s1
            r = W @ s1 - theta[0] * y  # Ritz residual
            rn = np.linalg.norm(r)
            history.append(rn)
            if rn < tol:
                # acceptance: a fresh product with L (and the deflation term)
                ly = L @ y
                true_r = np.linalg.norm(ly - theta[0] * y)
                if true_r < tol:
                    evals.append(theta[0])
                    evecs.append(y)
                    locked = True
                    # eigenvector purging: drop the locked direction from the basis
                    U = U @ S[:, 1:]
                    W = W @ S[:, 1:]
                    H = np.diag(theta[1:])
                    V = np.column_stack([V, y])
                    if moving_shift and len(theta) > 1:
                        sigma = min(float(theta[1]), sigma_cap)
                    if U.shape[1] == 0:
                        U, W, H, draws, breakdowns = _reseed(L, V, dl, ones, n, seed, draws, breakdowns)
                    break
                # the carried W has drifted: recompute W = (L + delta V V^T) U and H
                refreshes += 1
                W = np.column_stack([L @ U[:, t] + dl * (V @ (V.T @ U[:, t])) for t in range(U.shape[1])])
                H = U.T @ W
                H = 0.5 * (H + H.T)
                continue
            if U.shape[1] == m:  # subspace restart
                restarts += 1
                U = U @ S[:, :q]
                W = W @ S[:, :q]
                H = np.diag(theta[:q])
            # subspace expansion: trimmed (deflated) inner solve and enlargement
            rr = r - np.mean(r)  # Lemma 2.1: the right-hand side must be orthogonal to 1
            t_in = _time.perf_counter()
            zstar, its, _ = inner_solve(L, dvec, rr, i, sigma, dl, V, inner_rtol, max_inner, minv_hat, Lhat,
                                        rank_one, "minres" if moving_shift else "pcg")
            inner_clock[0] += _time.perf_counter() - t_in
            inner_here += its
            # orthonormalize against U and V (and 1/sqrt(n))
            Q = np.column_stack([U, V, ones])
            z, before, after = cgs2(Q, zstar)
            while not (after > 1e-10 * before and after > 0.0):
                breakdowns += 1
                z, before, after = cgs2(Q, replacement_vector(n, seed, draws))
                draws += 1
            u = z / after
            # expand U, and W = (L + delta V V^T) U one column at a time
            w = L @ u + dl * (V @ (V.T @ u))
            h = U.T @ w
            alpha = u @ w
            kk = U.shape[1]
            Hn = np.zeros((kk + 1, kk + 1))
            Hn[:kk, :kk] = H
            Hn[:kk, kk] = h
            Hn[kk, :kk] = h
            Hn[kk, kk] = alpha
            H = Hn
            U = np.column_stack([U, u])
            W = np.column_stack([W, w])
        outer_its.append(its_here)
        inner_its.append(inner_here)
    tick(sum(inner_its), U.shape[1] + V.shape[1])
    return done(_finish(L, evals, evecs, outer_its, inner_its, i, dl, restarts, breakdowns, refreshes, history))


def _reseed(L, V, dl, ones, n, seed, draws, breakdowns):
    """An empty basis after purging: start again from one replacement vector."""
    Q = np.column_stack([V, ones])
    while True:
        z, before, after = cgs2(Q, replacement_vector(n, seed, draws))
        draws += 1
        if after > 1e-10 * before:
            break
        breakdowns += 1
    u = z / after
    w = L @ u + dl * (V @ (V.T @ u))
    return u[:, None], w[:, None], np.array([[u @ w]]), draws, breakdowns


def _finish(L, evals, evecs, outer_its, inner_its, i, dl, restarts, breakdowns, refreshes, history,
            partial=False):
    ev = np.array(evals, dtype=np.float64)
    X = np.column_stack(evecs) if evecs else np.zeros((L.shape[0], 0))
    X = np.array([sign_normalize(X[:, j]) for j in range(X.shape[1])]).T.reshape(L.shape[0], -1)
    res = np.array([np.linalg.norm(L @ X[:, j] - ev[j] * X[:, j]) for j in range(X.shape[1])])
    return IsiraResult(ev, X, res, len(evals), outer_its, inner_its, i, dl, restarts, breakdowns,
                       refreshes, history)


def sign_normalize(v: np.ndarray) -> np.ndarray:
    """Make the entry of largest magnitude positive (lowest index among ties)."""
    j = int(np.argmax(np.abs(v)))
    return -v if v[j] < 0 else v


# ----------------------------------------------------------------------------------------
# Plain definition of the result, for small graphs
# ----------------------------------------------------------------------------------------


def smallest_positive_eigenpairs_dense(g, k: int):
    """The k smallest positive eigenvalues of L (with multiplicity) by dense symmetric
    eigendecomposition; the single zero eigenvalue (Theorem 1.2) is skipped."""
    Ld = laplacian(g).toarray()
    lam, X = np.linalg.eigh(Ld)
    return lam[1:k + 1], X[:, 1:k + 1]
