"""Training of the learned sparse-approximate-inverse (SPAI) preconditioner.

Data: the plain FP64 solver (Jacobi preconditioner) runs on seeded graphs with its capture
hook on; every inner solve contributes the pair (r', z) with r' = (L-hat - sigma I) z, the
pair an approximate inverse of L-hat - sigma I should map onto each other.
Training: minibatches of pairs go through libisira's network forward and hand-written
backward kernels (``isira_spai_loss_grad``) and its Adam kernel (``isira_adam_step``).
This module only orchestrates; tensors are torch CUDA tensors used as device memory.

Parameter layout (FP32 master copy; the kernels round to BF16):
    W1 (H x F), b1 (H), W2 (H x H), b2 (H), wd (2H), bd, We (H x (2H+1)), be (H), we (H), ce
with F = 8 vertex features and H = 16 hidden units.
"""
from __future__ import annotations

import math
import os
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from . import isira as I

F, H = 8, 16
E = 2 * H + 1
_LAYOUT = [("W1", H * F, F), ("b1", H, 0), ("W2", H * H, H), ("b2", H, 0), ("wd", 2 * H, 2 * H),
           ("bd", 1, 0), ("We", H * E, E), ("be", H, 0), ("we", H, H), ("ce", 1, 0)]
OFFSETS = {}
_o = 0
for _n, _sz, _fan in _LAYOUT:
    OFFSETS[_n] = (_o, _sz, _fan)
    _o += _sz
NPARAM = _o

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
DEFAULT_WEIGHTS = os.path.join(WEIGHTS_DIR, "spai_rmat_h16.npy")


def init_params(seed: int = 0):
    """Scaled-normal weights, zero biases; bd makes softplus(s) = 1 (the Jacobi diagonal)
    and ce = 0 with a small output layer starts the off-diagonal values near zero, so the
    untrained network is close to the Jacobi preconditioner."""
    import torch

    gen = torch.Generator().manual_seed(seed)
    p = torch.zeros(NPARAM, dtype=torch.float32)
    for name, (o, sz, fan) in OFFSETS.items():
        if fan:
            scale = 0.05 if name in ("wd", "we") else 1.0 / math.sqrt(fan)
            p[o:o + sz] = torch.randn(sz, generator=gen) * scale
    p[OFFSETS["bd"][0]] = math.log(math.e - 1.0)
    return p.cuda()


@dataclass
class PairSet:
    ctx: "I.Context"
    R: object  # torch float32 (count, n)
    Z: object
    sigma: float
    name: str = ""
    solve_s: float = 0.0


def generate_pairs(g, k: int = 20, sigma: float = 0.0, tol: float = 1e-8, cap: int = 400,
                   inner_rtol: float = 1e-4, seed: int = 1, name: str = "") -> PairSet:
    """Run the plain FP64 solver with the capture hook and keep the captured pairs."""
    import torch

    import graphgen as gg

    ctx = I.Context.from_graph(g)
    cr = torch.zeros((cap, g.n), dtype=torch.float64, device="cuda")
    cz = torch.zeros((cap, g.n), dtype=torch.float64, device="cuda")
    t = time.perf_counter()
    ev, X, res, st = ctx.solve(k, sigma, tol, u0=gg.start_block(g.n, 4, seed), capture=(cr, cz),
                               inner_rtol=inner_rtol)
    torch.cuda.synchronize()
    cnt = st["captured"]
    R = cr[:cnt].float().contiguous()
    Z = cz[:cnt].float().contiguous()
    del cr, cz
    return PairSet(ctx, R, Z, sigma, name or g.name, time.perf_counter() - t)


@dataclass
class TrainLog:
    steps: List[int] = field(default_factory=list)
    loss: List[float] = field(default_factory=list)
    seconds: float = 0.0


def train(sets: List[PairSet], steps: int = 600, batch: int = 16, lr: float = 3e-3,
          seed: int = 0, params=None, log_every: int = 50, verbose: bool = True):
    """Adam on minibatches of S pairs, cycling over the graphs."""
    import torch

    p = init_params(seed) if params is None else params.clone()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    gen = torch.Generator().manual_seed(seed + 17)
    logd = TrainLog()
    t0 = time.perf_counter()
    run = 0.0
    for step in range(1, steps + 1):
        ps = sets[(step - 1) % len(sets)]
        cnt = ps.R.shape[0]
        S = min(batch, cnt)
        idx = torch.randperm(cnt, generator=gen)[:S].cuda()
        R = ps.R.index_select(0, idx).contiguous()
        Z = ps.Z.index_select(0, idx).contiguous()
        loss, grad = ps.ctx.spai_loss_grad(p, R, Z, sigma=ps.sigma)
        ps.ctx.adam_step(p, grad, m, v, lr=lr, step=step)
        run = loss if step == 1 else 0.95 * run + 0.05 * loss
        if step % log_every == 0 or step == 1 or step == steps:
            logd.steps.append(step)
            logd.loss.append(run)
            if verbose:
                print(f"[spai] step {step} loss(ema) {run:.4f} graph {ps.name}", flush=True)
    torch.cuda.synchronize()
    logd.seconds = time.perf_counter() - t0
    return p, logd


def mean_loss(sets: List[PairSet], params, batch: int = 32) -> float:
    import torch

    tot = 0.0
    cnt = 0
    for ps in sets:
        n = ps.R.shape[0]
        for b in range(0, n, batch):
            S = min(batch, n - b)
            if S < 1:
                continue
            loss, _ = ps.ctx.spai_loss_grad(params, ps.R[b:b + S].contiguous(), ps.Z[b:b + S].contiguous(),
                                            sigma=ps.sigma)
            tot += loss * S
            cnt += S
    torch.cuda.synchronize()
    return tot / max(1, cnt)


def evaluate(g, params, k: int = 20, sigma: float = 0.0, tol: float = 1e-8, seed: int = 1,
             inner_rtol: float = 1e-4, repeats: int = 1) -> dict:
    """Time to k pairs on one graph: plain FP64 (Jacobi), FP32 inner (Jacobi) and FP32 inner
    with the learned preconditioner; every variant must reach the residual tolerance."""
    import numpy as np
    import torch

    import graphgen as gg

    ctx = I.Context.from_graph(g)
    u0 = gg.start_block(g.n, 4, seed)
    out = {"n": g.n, "nnz": g.nnz}
    ref = None
    t = time.perf_counter()
    ctx.spai_install(params, sigma=sigma)
    torch.cuda.synchronize()
    out["install_s"] = time.perf_counter() - t
    for name, prec, pc in [("fp64_jacobi", I.FP64, I.PC_JACOBI), ("fp32_jacobi", I.FP32, I.PC_JACOBI),
                           ("fp32_learned", I.FP32, I.PC_LEARNED), ("fp64_learned", I.FP64, I.PC_LEARNED)]:
        best = None
        for _ in range(repeats):
            ev, X, res, st = ctx.solve(k, sigma, tol, u0=u0, inner_prec=prec, precond=pc,
                                       inner_rtol=inner_rtol)
            best = st if best is None or st["ms_total"] < best["ms_total"] else best
        ev = np.sort(ev)
        row = {"s": best["ms_total"] / 1e3, "converged": best["n_converged"], "outer": best["outer_total"],
               "inner": best["inner_total"], "max_resid": float(np.max(res)) if len(res) else None}
        if ref is None:
            ref = ev
        elif len(ev) == len(ref):
            row["max_rel_eval_diff_vs_fp64_jacobi"] = float(np.max(np.abs(ev - ref) / ref))
        out[name] = row
    return out


def save(params, path: str = DEFAULT_WEIGHTS):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, params.detach().cpu().numpy().astype(np.float32), allow_pickle=False)


def load(path: str = DEFAULT_WEIGHTS):
    import torch

    a = np.load(path, allow_pickle=False)
    if a.shape != (NPARAM,) or a.dtype != np.float32:
        raise ValueError(f"{path}: expected float32[{NPARAM}]")
    return torch.as_tensor(a).cuda()


def main(argv: Optional[list] = None):
    """Train on seeded R-MAT graphs (scale 16 + seed mod 3, edge factor 8), save the weights,
    and optionally evaluate them on held-out R-MAT graphs."""
    import argparse
    import json

    import graphgen as gg

    ap = argparse.ArgumentParser()
    ap.add_argument("--graphs", type=int, default=64)
    ap.add_argument("--first-seed", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--k", type=int, default=20)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    ap.add_argument("--eval", default="", help="comma list of held-out graphs: rmatS[:EF[:seed]]")
    args = ap.parse_args(argv)
    I.load()
    sets = []
    t0 = time.perf_counter()
    for s in range(args.first_seed, args.first_seed + args.graphs):
        g = gg.rmat(16 + (s % 3), 8, seed=s)
        ps = generate_pairs(g, k=args.k, seed=s)
        print(f"[spai] graph seed {s}: n={g.n} nnz={g.nnz} pairs={ps.R.shape[0]} "
              f"solve {ps.solve_s:.2f} s", flush=True)
        sets.append(ps)
    print(f"[spai] data generation {time.perf_counter() - t0:.1f} s", flush=True)
    l0 = mean_loss(sets[:4], init_params(0))
    p, lg = train(sets, steps=args.steps, batch=args.batch, lr=args.lr)
    l1 = mean_loss(sets[:4], p)
    print(f"[spai] trained {args.steps} steps in {lg.seconds:.1f} s; loss {l0:.4f} -> {l1:.4f}", flush=True)
    save(p, args.out)
    print(f"[spai] saved {args.out}", flush=True)
    for spec in [x for x in args.eval.split(",") if x]:
        parts = spec[4:].split(":")
        scale = int(parts[0])
        ef = int(parts[1]) if len(parts) > 1 else 8
        seed = int(parts[2]) if len(parts) > 2 else 4000
        g = gg.rmat(scale, ef, seed=seed)
        res = evaluate(g, p, k=args.k)
        res["graph"] = spec
        print("[spai-eval] " + json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
