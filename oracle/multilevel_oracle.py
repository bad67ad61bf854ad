"""Plain FP64 CPU oracle of the multilevel preconditioner for the inner systems of iSIRA.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link this
module: only the tests, the smoke check and the bench's CPU-baseline leg use it.  It shares
no code with the GPU library.

Section 3 of the paper names a multilevel solver (combinatorial multigrid) as a
preconditioner choice for the trimmed systems and leaves the choice open (Remark 3.2: any
SPD approximation M-hat_sigma of L-hat - sigma I, combined with eq. (3.5) for the deflation
term).  This module defines the one built here, an unsmoothed-aggregation multigrid
V-cycle for the trimmed Laplacian L-hat:

  * levels: A_0 = L-hat (the Laplacian with the trimmed vertex's row and column deleted,
    eq. (2.4)); A_{l+1} = P_l^T A_l P_l (Galerkin), P_l the 0/1 aggregation matrix of
    level l (row v has its one 1 in the column of v's aggregate);
  * aggregation of level l (greedy, on the graph of A_l's off-diagonal pattern):
      a vertex without neighbours (for instance a leaf of the trimmed vertex) belongs to
      no aggregate (its row of P is zero); the others are aggregated as follows;
      visiting order: decreasing number of neighbours, ties by increasing index;
      phase 1: a vertex that is unassigned and whose neighbours are all unassigned forms
               a new aggregate with all its neighbours (ids in order of creation);
      phase 2: every vertex still unassigned joins, among the phase-1 aggregates holding
               at least one of its neighbours, the one holding the most, ties by the
               smallest id.  (A vertex left after phase 1 always has such a neighbour:
               it was skipped because one of its neighbours was already assigned.)
    The rule uses no floating-point comparison, so any implementation that follows it
    forms the same aggregates;
  * a level with at most ``coarse_max`` vertices that have neighbours is the coarsest and
    is solved exactly (its vertices without neighbours decouple: each is one equation);
  * smoothing: one damped Jacobi sweep x <- x + S (b - A x), S = W D^-1, before and one
    after the coarse correction (D = diag(A_l), W = diag(w_v) with w_v = omega, or 1 for a
    vertex without neighbours, whose equation the sweep then solves exactly); pre- and
    post-smoother are the same symmetric operator, so the cycle is a symmetric linear
    operator, and positive definite for omega < 2 / lambda_max(D^-1 A) (at most 2 for these
    diagonally dominant levels).  Every aggregate has at least two members, so each level
    has at most half as many vertices with neighbours as the one before, and with
    ``coarse_max = 0`` the coarsening runs until no vertex has a neighbour.

Readings (listed in the design notes too): the hierarchy approximates L-hat^{-1}, without
the shift (the bench and the configurations use sigma = 0, where it is exactly the
trimmed operator of eq. (2.4)); the deflation term is handled by eq. (3.5) as for Jacobi;
the rank-one term of eq. (2.15) is left out of the preconditioner (Remark 3.1), as for
Jacobi.  Library primitives used as steps: scipy sparse products and sparse direct solve.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import isira_oracle as O


def _neighbours(A: sp.csr_matrix) -> List[np.ndarray]:
    """Off-diagonal column indices of each row of A (the level's graph)."""
    A = A.tocsr()
    out = []
    for v in range(A.shape[0]):
        cols = A.indices[A.indptr[v]:A.indptr[v + 1]]
        vals = A.data[A.indptr[v]:A.indptr[v + 1]]
        out.append(np.sort(cols[(cols != v) & (vals != 0.0)]))
    return out


def aggregate(A: sp.csr_matrix) -> np.ndarray:
    """Aggregate id of every vertex of the graph of A (phases 1 and 2 above); -1 for a
    vertex without neighbours."""
    nb = _neighbours(A)
    n = len(nb)
    rowlen = np.array([len(x) for x in nb], dtype=np.int64)
    order = np.argsort(-rowlen, kind="stable")  # decreasing row length, ties by index
    agg = -np.ones(n, dtype=np.int64)
    nagg = 0
    for v in order:  # phase 1
        if rowlen[v] > 0 and agg[v] < 0 and np.all(agg[nb[v]] < 0):
            agg[v] = nagg
            agg[nb[v]] = nagg
            nagg += 1
    phase1 = agg.copy()
    for v in range(n):  # phase 2 (reads phase-1 assignments only)
        if phase1[v] >= 0 or rowlen[v] == 0:
            continue
        ids = phase1[nb[v]]
        ids = ids[ids >= 0]
        assert ids.size > 0, "a vertex left after phase 1 has an assigned neighbour"
        agg[v] = int(np.argmax(np.bincount(ids)))  # most members; argmax takes the smallest id
    assert np.all((agg >= 0) == (rowlen > 0))
    return agg


def prolongation(agg: np.ndarray) -> sp.csr_matrix:
    """P with P[v, agg[v]] = 1 (row v zero when agg[v] = -1)."""
    n = agg.size
    v = np.flatnonzero(agg >= 0)
    return sp.csr_matrix((np.ones(v.size), (v, agg[v])), shape=(n, int(agg.max()) + 1))


def connected_count(A: sp.csr_matrix) -> int:
    """Number of vertices with at least one neighbour in the graph of A."""
    return int(sum(len(x) > 0 for x in _neighbours(A)))


def smoother_weights(A: sp.csr_matrix, omega: float) -> np.ndarray:
    """S = W D^-1 of the definition above, as a vector."""
    A = A.tocsr()
    has_nb = np.array([np.any((A.indices[A.indptr[v]:A.indptr[v + 1]] != v) &
                              (A.data[A.indptr[v]:A.indptr[v + 1]] != 0.0))
                       for v in range(A.shape[0])])
    return np.where(has_nb, omega, 1.0) / A.diagonal()


@dataclasses.dataclass
class Hierarchy:
    A: List[sp.csr_matrix]   # A_0 .. A_L (A_L the coarsest, solved exactly)
    P: List[sp.csr_matrix]   # P_0 .. P_{L-1}
    agg: List[np.ndarray]    # aggregate ids of levels 0 .. L-1
    omega: float
    trim: int                # trimmed vertex of the graph (caller label)


def setup(g, trim: int, omega: float = 0.9, coarse_max: int = 512,
          max_levels: int = 16) -> Hierarchy:
    """Hierarchy of A_0 = L-hat (vertex ``trim`` deleted) as defined above."""
    L = O.laplacian(g)
    A = O.trimmed_matrix(L, trim).tocsr()
    As, Ps, aggs = [A], [], []
    while connected_count(As[-1]) > coarse_max:
        if len(As) >= max_levels:
            raise ValueError("coarsest level still larger than coarse_max at max_levels")
        agg = aggregate(As[-1])
        P = prolongation(agg)
        Ac = (P.T @ As[-1] @ P).tocsr()
        Ac.sum_duplicates()
        aggs.append(agg)
        Ps.append(P)
        As.append(Ac)
    return Hierarchy(As, Ps, aggs, float(omega), int(trim))


def vcycle(h: Hierarchy, b: np.ndarray, level: int = 0) -> np.ndarray:
    """One V(1,1) cycle from x = 0 for A_level x = b."""
    A = h.A[level]
    if level == len(h.A) - 1:
        return spla.spsolve(A.tocsc(), b) if A.shape[0] > 1 else b / A.diagonal()
    s = smoother_weights(A, h.omega)
    P = h.P[level]
    x = s * b                                   # pre-smoothing from zero
    r = b - A @ x                               # residual
    ec = vcycle(h, P.T @ r, level + 1)          # restriction, coarse correction
    x = x + P @ ec                              # prolongation
    x = x + s * (b - A @ x)                     # post-smoothing
    return x


def preconditioner_factory(g, omega: float = 0.9, coarse_max: int = 512,
                           max_levels: int = 16) -> Callable:
    """For ``isira_oracle.isira(apply_minv_hat_factory=...)``: (trim, sigma) -> the V-cycle
    acting on trimmed (n-1)-vectors (the shift is not part of the hierarchy)."""

    def factory(trim: int, sigma: float):
        h = setup(g, trim, omega, coarse_max, max_levels)
        return lambda x: vcycle(h, x)

    return factory


def operator_matrix(h: Hierarchy, level: int = 0) -> np.ndarray:
    """Dense matrix of the V-cycle at ``level`` (columns = cycle applied to unit vectors);
    small levels only."""
    m = h.A[level].shape[0]
    return np.column_stack([vcycle(h, np.eye(m)[:, j], level) for j in range(m)])
