"""The allocation-free orthonormalization (isira_orthonormalize_noalloc) against the
allocating one (isira_orthonormalize), through the C ABI: two calls in a row, the second
on a smaller input, each compared with the allocating entry point's result."""
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


def _orthonormal_rows(n, nc, seed):
    # nc orthonormal vectors orthogonal to 1 (the basis shape the solver orthogonalizes against)
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, nc))
    A -= A.mean(axis=0)
    Q, _ = np.linalg.qr(A)
    return np.ascontiguousarray(Q.T)


def _case(P, g, nc, seed, heavy):
    ctx = P.Context.from_graph(g)
    n = g.n
    Q = _orthonormal_rows(n, nc, seed)
    rng = np.random.default_rng(seed + 1)
    z = rng.standard_normal(n)
    if heavy and nc:
        z = z + 1e6 * (Q.T @ rng.standard_normal(nc))  # heavy cancellation: both passes matter
    Qd = torch.as_tensor(Q, device="cuda")
    zd = torch.as_tensor(z, device="cuda")
    print(f"no-alloc CGS2: n={n} ncols={nc} seed={seed}", flush=True)
    u_ref, norms_ref = ctx.orthonormalize(Qd if nc else None, zd)
    u = torch.full_like(zd, float("nan"))
    norms = ctx.orthonormalize_noalloc(Qd if nc else None, zd, u)
    torch.cuda.synchronize()
    assert torch.equal(zd, torch.as_tensor(z, device="cuda"))  # z is read only
    u, u_ref = u.cpu().numpy(), u_ref.cpu().numpy()
    # both are CGS2 in FP64 with sums taken in other orders (caller vs internal labels): the
    # results agree to a few units of rounding times the cancellation ||z|| / ||z_after||
    amp = norms_ref[0] / norms_ref[1]
    assert np.allclose(norms, norms_ref, rtol=2e-14 * amp, atol=0)
    assert np.linalg.norm(u - u_ref) <= 2e-14 * amp
    # the result itself: unit norm, orthogonal to Q and to 1
    assert abs(np.linalg.norm(u) - 1.0) <= 1e-14
    if nc:
        assert np.abs(Q @ u).max() <= 1e-14
    assert abs(u.sum()) <= 1e-14 * np.sqrt(n)
    # against the oracle's CGS2 as well
    Qo = np.column_stack([Q.T, np.ones(n) / np.sqrt(n)])
    zo, before, after = O.cgs2(Qo, z)
    assert np.linalg.norm(u - zo / after) <= 2e-14 * amp
    return ctx


def test_noalloc_orthonormalize_two_calls(P):
    # first call: n beyond 512 * 1024 rows (the full grid of the column-dot kernel) and the
    # maximal basis width; second call: a smaller graph and basis, on the same GPU's scratch
    big = gg.grid3d(90, 90, 90)
    _case(P, big, 192, 3, heavy=True)
    small = gg.random_connected(3001, 5000, seed=8)
    _case(P, small, 7, 4, heavy=False)


def test_noalloc_orthonormalize_rejects_wide_basis(P):
    g = gg.path_graph(500)
    ctx = P.Context.from_graph(g)
    z = torch.ones(500, dtype=torch.float64, device="cuda")
    u = torch.empty_like(z)
    Q = torch.zeros((193, 500), dtype=torch.float64, device="cuda")
    with pytest.raises(P.isira.IsiraError) as e:
        ctx.orthonormalize_noalloc(Q, z, u)
    assert e.value.code == P.isira.ISIRA_E_ARG
