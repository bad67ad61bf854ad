"""The boundary's workspace form (isira_workspace_bytes, isira_create_ws): a context whose
device memory is a caller-owned workspace computes exactly what a context with its own
allocations computes (same relabelling, same plan, same kernels), takes no device memory of
its own, accepts device-resident CSR, and reports a short workspace as ISIRA_E_WORKSPACE."""
import os

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1710_07080_amd as pkg

    pkg.load()
    return pkg


def _ws(P, g, k, flags=0, **opts):
    wdt = P.isira.W_NONE if g.w is None else P.isira.W_F64
    nbytes = P.isira.workspace_bytes(g.n, g.nnz, k, w_dtype=wdt, flags=flags, **opts)
    assert nbytes > 0
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def _same(a, b):
    ev_a, X_a, r_a, st_a = a
    ev_b, X_b, r_b, st_b = b
    assert st_a["n_converged"] == st_b["n_converged"] > 0
    assert st_a["outer_total"] == st_b["outer_total"] and st_a["inner_total"] == st_b["inner_total"]
    assert np.array_equal(ev_a, ev_b) and np.array_equal(r_a, r_b)
    assert torch.equal(X_a, X_b)


def test_workspace_context_is_bit_identical_and_allocates_nothing(P):
    g = gg.grid3d(90, 90, 90)
    k = 6
    U0 = gg.start_block(g.n, 4, 3)
    print(f"workspace context: grid 90^3 n={g.n} k={k}", flush=True)
    own = P.Context.from_graph(g)
    ref = own.solve(k, 0.0, 1e-8, u0=U0)
    own.close()
    torch.cuda.synchronize()
    ws = _ws(P, g, k)
    torch.cuda.synchronize()
    free0, res0 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
    ctx = P.Context.with_workspace(g.n, g.row_ptr, g.col, workspace=ws, k=k)
    got = ctx.solve(k, 0.0, 1e-8, u0=U0)
    y = ctx.laplacian_apply(torch.ones(g.n, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    free1, res1 = torch.cuda.mem_get_info()[0], torch.cuda.memory_reserved()
    _same(ref, got)
    assert float(y.abs().max()) == 0.0  # L 1 = 0 exactly for unit weights
    info = ctx.memory_info()
    assert 0 < info["peak"] <= info["capacity"] <= ws.numel()
    # the context's buffers (hundreds of MB here) all live in the workspace: beyond what torch
    # reserved for the outputs, the device's free memory moved by runtime bookkeeping at most
    assert ws.numel() > 256 << 20
    assert (free0 - free1) - (res1 - res0) < 16 << 20, (free0 - free1, res1 - res0, info)


def test_workspace_with_device_csr_and_weights(P):
    g = gg.grid3d(20, 17, 13, weights=(0.5, 1.5), seed=3)
    k = 5
    U0 = gg.start_block(g.n, 4, 4)
    ref = P.Context.from_graph(g).solve(k, 0.0, 1e-9, u0=U0, inner_prec=P.isira.FP32)
    ws = _ws(P, g, k)
    rp = torch.as_tensor(g.row_ptr, device="cuda")
    col = torch.as_tensor(g.col, device="cuda")
    w = torch.as_tensor(g.w, device="cuda")
    ctx = P.Context.with_workspace(g.n, rp, col, w, workspace=ws, k=k)
    _same(ref, ctx.solve(k, 0.0, 1e-9, u0=U0, inner_prec=P.isira.FP32))


def test_workspace_learned_preconditioner(P):
    from paper_1710_07080_amd import spai_train

    if not os.path.exists(spai_train.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    g = gg.rmat(14, 8, seed=9)
    k = 8
    U0 = gg.start_block(g.n, 4, 2)
    params = spai_train.load()
    own = P.Context.from_graph(g)
    own.spai_install(params, sigma=0.0)
    kept_a = own.spai_prune(0.02)
    ref = own.solve(k, 0.0, 1e-9, u0=U0, inner_prec=P.isira.FP32, precond=P.isira.PC_LEARNED)
    ws = _ws(P, g, k, flags=P.isira.WS_LEARNED)
    ctx = P.Context.with_workspace(g.n, g.row_ptr, g.col, workspace=ws, k=k)
    ctx.spai_install(params, sigma=0.0)
    assert ctx.spai_prune(0.02) == kept_a
    _same(ref, ctx.solve(k, 0.0, 1e-9, u0=U0, inner_prec=P.isira.FP32, precond=P.isira.PC_LEARNED))
    assert ctx.memory_info()["peak"] <= ws.numel()


def test_workspace_too_small(P):
    g = gg.rmat(12, 8, seed=3)
    k = 8
    full = P.isira.workspace_bytes(g.n, g.nnz, k)
    small = torch.empty(full // 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.isira.IsiraError) as e:
        P.Context.with_workspace(g.n, g.row_ptr, g.col, workspace=small, k=k)
    assert e.value.code == P.isira.ISIRA_E_WORKSPACE
    # sized for k = 8: a solve asking for more pairs (a larger basis) cannot grow into it
    ws = torch.empty(full, dtype=torch.uint8, device="cuda")
    ctx = P.Context.with_workspace(g.n, g.row_ptr, g.col, workspace=ws, k=k)
    with pytest.raises(P.isira.IsiraError) as e:
        ctx.solve(40, 0.0, 1e-8)
    assert e.value.code == P.isira.ISIRA_E_WORKSPACE
    ev, X, r, st = ctx.solve(k, 0.0, 1e-8)  # the sized solve still runs afterwards
    assert st["n_converged"] == k


def test_workspace_multilevel_hierarchy(P):
    """The multilevel hierarchy's buffers come from the workspace too: with room for them
    the cycle-preconditioned solve is bit-identical to an allocating context's; without it
    the set-up fails with ISIRA_E_WORKSPACE and the context keeps working with Jacobi."""
    g = gg.grid3d(24, 22, 20, weights=(0.5, 1.5), seed=6)
    k = 6
    U0 = gg.start_block(g.n, 4, 6)
    own = P.Context.from_graph(g)
    info = own.ml_setup()
    ref = own.solve(k, 0.0, 1e-9, u0=U0, inner_prec=P.isira.FP32, precond=P.isira.PC_MULTILEVEL)
    plain = own.solve(k, 0.0, 1e-9, u0=U0)
    own.close()
    base = P.isira.workspace_bytes(g.n, g.nnz, k, w_dtype=P.isira.W_F64)
    # room for the hierarchy: its device bytes plus one 256-byte block per buffer
    ws = torch.empty(base + info["device_bytes"] + (1 << 20), dtype=torch.uint8, device="cuda")
    rp, col, w = g.row_ptr, g.col, g.w
    ctx = P.Context.with_workspace(g.n, rp, col, w, workspace=ws, k=k)
    assert ctx.ml_setup()["rows"] == info["rows"]
    _same(ref, ctx.solve(k, 0.0, 1e-9, u0=U0, inner_prec=P.isira.FP32, precond=P.isira.PC_MULTILEVEL))
    assert ctx.memory_info()["peak"] <= ws.numel()
    ctx.close()
    tight = torch.empty(base, dtype=torch.uint8, device="cuda")
    ctx = P.Context.with_workspace(g.n, rp, col, w, workspace=tight, k=k)
    with pytest.raises(P.isira.IsiraError) as e:
        ctx.ml_setup()
    assert e.value.code == P.isira.ISIRA_E_WORKSPACE
    _same(plain, ctx.solve(k, 0.0, 1e-9, u0=U0))
