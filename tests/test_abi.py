"""CPU-side checks of the C ABI: the library loads, exports every declared entry point,
the host eigensolver works, and graph validation rejects bad input before any GPU call."""
import os
import re

import numpy as np
import pytest

import graphgen as gg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def P():
    import paper_1710_07080_amd as pkg

    pkg.load()
    return pkg


def declared_functions():
    text = open(os.path.join(ROOT, "include", "isira.h")).read()
    return sorted(set(re.findall(r"\b(isira_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(P):
    lib = P.load()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    assert sorted(P.isira.EXPORTS) == names


def test_defaults_and_strerror(P):
    o = P.isira.default_options()
    assert o.k0 == 4 and o.inner_rtol == 1e-1 and o.trim_index == -1 and o.check_every == 8
    lib = P.load()
    for code in [0, 1, -1, -2, -3, -4, -5, -6, -7, -8]:
        assert lib.isira_strerror(code) and lib.isira_strerror(code) != b"unknown error", code
    assert lib.isira_strerror(-99) == b"unknown error"


@pytest.mark.parametrize("k", [1, 2, 3, 7, 40, 120, 192])
def test_host_symeig(P, k):
    rng = np.random.default_rng(k)
    H = rng.standard_normal((k, k))
    H = H + H.T
    theta, S = P.symeig(H)
    lam = np.linalg.eigvalsh(H)
    scale = max(1.0, np.abs(lam).max())
    assert np.abs(theta - lam).max() <= 1e-13 * scale
    assert np.abs(H @ S - S * theta).max() <= 1e-12 * scale
    assert np.abs(S.T @ S - np.eye(k)).max() <= 1e-13
    assert np.all(np.diff(theta) >= 0)


def test_symeig_clustered_and_diagonal(P):
    H = np.diag([3.0, 1.0, 2.0, 1.0, 5.0])
    theta, S = P.symeig(H)
    assert np.allclose(theta, [1, 1, 2, 3, 5])
    H = np.diag(np.arange(1, 31) * 1e-3) + 1e-12 * np.ones((30, 30))
    theta, S = P.symeig(H)
    assert np.allclose(theta, np.linalg.eigvalsh(H), rtol=0, atol=1e-15)


def _bad(P, n, rp, col, w=None, code=None):
    with pytest.raises(P.IsiraError) as e:
        P.Context(n, np.asarray(rp), np.asarray(col), w, stream=0)
    assert e.value.code == code


def test_create_rejects_bad_graphs(P):
    E = P.isira
    _bad(P, 3, [0, 1, 2, 2], [1, 0], code=E.ISIRA_E_DISCONNECTED)   # isolated vertex 2
    _bad(P, 3, [0, 2, 3, 4], [0, 1, 0, 0], code=E.ISIRA_E_GRAPH)    # self loop
    _bad(P, 3, [0, 1, 2, 3], [1, 0, 5], code=E.ISIRA_E_GRAPH)       # index out of range
    _bad(P, 3, [0, 2, 3, 4], [2, 1, 0, 0], code=E.ISIRA_E_GRAPH)    # unsorted columns
    _bad(P, 3, [0, 1, 3, 4], [1, 0, 2, 0], code=E.ISIRA_E_GRAPH)    # asymmetric pattern
    g = gg.path_graph(5)
    w = np.ones(g.nnz)
    w[0] = 2.0
    _bad(P, 5, g.row_ptr, g.col, w, code=E.ISIRA_E_GRAPH)            # asymmetric weights
    w = np.ones(g.nnz)
    w[3] = -1.0
    _bad(P, 5, g.row_ptr, g.col, w, code=E.ISIRA_E_GRAPH)            # negative weight
    # two components: 0-1 and 2-3
    _bad(P, 4, [0, 1, 2, 3, 4], [1, 0, 3, 2], code=E.ISIRA_E_DISCONNECTED)
    _bad(P, 2, [0, 1, 2], [1, 0], code=E.ISIRA_E_ARG)                # n too small


def test_multilevel_defaults(P):
    o = P.isira.MlOptions()
    assert P.load().isira_ml_default_options(o) == 0
    assert o.omega == 0.9 and o.coarse_max == 512 and o.max_levels == 24
    assert o.trim_index == -1
    assert P.isira.PC_MULTILEVEL == 2


@pytest.mark.parametrize("case", ["random7", "random60", "random192", "clustered", "diagonal",
                                  "k1", "k2", "graded", "rayleigh_ritz"])
def test_host_symeig_lowest(P, case):
    """Eigenvalues and the lowest eigenvector against numpy's LAPACK eigensolver."""
    rng = np.random.default_rng(len(case))
    if case.startswith("random"):
        k = int(case[6:])
        H = rng.standard_normal((k, k))
        H = H + H.T
    elif case == "clustered":  # the two smallest eigenvalues 1e-13 apart
        k = 40
        Q = np.linalg.qr(rng.standard_normal((k, k)))[0]
        lam = np.concatenate([[1.0, 1.0 + 1e-13], np.linspace(2.0, 9.0, k - 2)])
        H = (Q * lam) @ Q.T
    elif case == "diagonal":
        H = np.diag([3.0, 1.0, 2.0, 5.0, 0.5])
    elif case == "k1":
        H = np.array([[2.5]])
    elif case == "k2":
        H = np.array([[2.0, 1.0], [1.0, 2.0]])
    elif case == "graded":  # eigenvalues spanning twelve orders of magnitude
        k = 30
        Q = np.linalg.qr(rng.standard_normal((k, k)))[0]
        H = (Q * np.logspace(-8, 4, k)) @ Q.T
    else:  # the projected matrix of a Laplacian on an orthonormal block orthogonal to 1
        import scipy.sparse as sp
        g = gg.rmat(10, 8, seed=3)
        A = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
        L = sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A
        U = rng.standard_normal((g.n, 60))
        U -= U.mean(axis=0)
        U = np.linalg.qr(U)[0]
        H = U.T @ (L @ U)
        H = 0.5 * (H + H.T)
    theta, s1 = P.isira.symeig_lowest(H)
    lam, V = np.linalg.eigh(H)
    scale = max(1.0, np.abs(lam).max())
    assert np.abs(theta - lam).max() <= 1e-13 * scale
    assert abs(np.linalg.norm(s1) - 1.0) <= 1e-14
    # an eigenvector of the smallest eigenvalue (within the cluster when it is not simple)
    assert np.linalg.norm(H @ s1 - theta[0] * s1) <= 1e-13 * scale
    # the angle to numpy's eigenvector within the Davis-Kahan bound eps ||H|| / gap
    gap = lam[1] - lam[0] if len(lam) > 1 else np.inf
    if gap > 1e-6 * scale:
        v0 = V[:, 0]
        sin = np.linalg.norm(s1 - (s1 @ v0) * v0)  # the part of s1 orthogonal to v0
        assert sin <= 64 * 2.0 ** -53 * scale / gap + 1e-14


def test_workspace_bytes_bound(P):
    wb = P.isira.workspace_bytes
    n, nnz = 100000, 1600000
    assert wb(2, 10, 4) == 0 and wb(n, nnz, 0) == 0 and wb(n, nnz, 65) == 0
    assert wb(n, nnz, 4, m=193) == 0  # m beyond ISIRA_MAX_BASIS
    a = wb(n, nnz, 10)
    # at least the basis U, W (n x m FP64, m = 2 (k + 10)) and the CSR column indices
    assert a >= 2 * n * 40 * 8 + nnz * 4
    assert wb(n, nnz, 20) > a  # more pairs: a larger basis and more deflation columns
    assert wb(n, nnz, 10, w_dtype=P.isira.W_F64) >= a + nnz * 12  # FP64 and FP32 weights
    assert wb(n, nnz, 10, flags=P.isira.WS_LEARNED) >= a + nnz * 12  # M's values and pruned copy
    assert wb(n, nnz, 10, q=30, m=60) > a
