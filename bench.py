"""Benchmark of the iSIRA hot path on one MI355X.

One step = one full isira_solve (Algorithm 3.2: Rayleigh-Ritz, residual, trimmed deflated
PCG inner solve, enlargement, CGS2, expansion, restart/purge/lock) for the k smallest
positive eigenpairs of a seeded synthetic graph that is already resident in HBM.

Default workload: the learned preconditioner's held-out graph, R-MAT scale 22 with 16 * 2^22
edge samples ((0.57, 0.19, 0.19, 0.05), symmetrized, deduplicated, self loops removed,
largest connected component, unit weights; n = 2,394,541, 128 M stored entries), k = 20,
sigma = 0, tol = 1e-8.  The timed form is the metric's "learned + FP32": the trained network's
approximate inverse (pruned) as the inner preconditioner and FP32 inner solves, with FP64
outer steps.  The plain FP64 method (Jacobi) and FP32 Jacobi (the learned part's own gain)
are timed beside it the same way (median of the same number of solves).

Prints one JSON line: time to k eigenpairs (seconds, lower is better), the SpMV roofline
of the dominant kernel (measured live with HIP events on the library's stream, each launch
from HBM), and the FP64 CPU oracle timed on a bounded sample on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
DEFAULT_WORKLOAD = "rmat22e16"
WORKLOAD_TEXT = {
    "rmat22e16": "rmat22e16: held-out R-MAT scale 22, 16 * 2^22 edge samples, LCC, unit weights",
    "rmat20": "rmat20: R-MAT scale 20, edge factor 8, LCC, unit weights",
    "chunglu24": "chunglu24: Chung-Lu n = 2^24, exponent 2.1, mean degree 24, LCC, unit weights",
    "grid128w": "grid128w: 3-D 7-point grid 128^3, weights U[0.5, 1.5]",
    "grid64": "grid64: 2-D 5-point grid 64 x 64, unit weights",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import graphgen as gg

    if name == "rmat20":
        return gg.rmat(20, 8, seed=2), dict(k=20, sigma=0.0, tol=1e-8)
    if name == "grid64":
        return gg.grid2d(64, 64), dict(k=10, sigma=0.0, tol=1e-10)
    if name == "grid128w":
        return gg.grid3d(128, 128, 128, weights=(0.5, 1.5), seed=3), dict(k=20, sigma=0.0, tol=1e-8)
    if name == "chunglu24":  # n = 2^24, beta 2.1, mean degree 24 (sorted on the GPU)
        return gg.chung_lu(1 << 24, 2.1, 24.0, seed=5, device="cuda"), dict(k=50, sigma=0.0, tol=1e-8)
    if name == "rmat22e16":  # held-out graph of the learned preconditioner: scale 22, mean degree 32
        return gg.rmat(22, 16, seed=4000, device="cuda"), dict(k=20, sigma=0.0, tol=1e-8)
    if name.startswith("rmat"):
        s = int(name[4:])
        return gg.rmat(s, 8, seed=2), dict(k=20, sigma=0.0, tol=1e-8)
    raise KeyError(name)


SPAI_WEIGHTS = os.path.join(HERE, "paper_1710_07080_amd", "weights", "spai_rmat_h16.npy")
CAL_BYTES = 256 << 20  # size of the calibration copy in --probe runs
# pruning threshold of the learned M's variant: keeps off-diagonals with
# |m_ij| >= tau sqrt(M_ii M_jj), a few percent of them for the trained network
PRUNE_TAU = 0.02
# HBM traffic of the dominant kernel from rocprofv3 counter runs (FETCH_SIZE, WRITE_SIZE),
# with the sources it was measured on; it is reported only while those sources are unchanged.
PROFILES = os.path.join(HERE, "profiles")
CSRC = os.path.join(HERE, "paper_1710_07080_amd", "csrc")
# The product's sources: kernels.hip up to the PCG updates (the product and the reduction
# helpers it uses), internal.h, and the relabelling and work-unit plan of api.hip.
PRODUCT_SOURCES = [("kernels.hip", None, "// ------------------------------------------------------------------ PCG updates"),
                   ("internal.h", None, None),
                   ("api.hip", "// Power-law test on the degree-sorted labels", "void isira::free_spmv_plan")]


def sources_digest():
    """sha256 prefix of the product's sources (a traffic record is valid while they match)."""
    import hashlib

    h = hashlib.sha256()
    for name, begin, end in PRODUCT_SOURCES:
        with open(os.path.join(CSRC, name)) as f:
            text = f.read()
        a = text.index(begin) if begin else 0
        b = text.index(end) if end else len(text)
        h.update(text[a:b].encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, prec):
    """Bytes per launch of the product (prec "fp64" / "fp32") from the committed counter
    summary, or None when there is none for this workload or the kernel sources changed
    since it was taken."""
    path = os.path.join(PROFILES, f"k_spmv_{prec}_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("traffic_json: "):
                rec = json.loads(line[len("traffic_json: "):])
    if not rec or rec.get("workload") != workload or rec.get("sources_digest") != sources_digest():
        return None
    return rec


def golden(name):
    """Reference eigenvalues of the workload: the closed form for the 64x64 grid (the
    Laplacian of a product of two paths has the sums of the paths' eigenvalues
    2 - 2 cos(j pi / 64)), else the oracle's (written by tests/golden/make_golden.py)."""
    if name == "grid64":
        p = 2.0 - 2.0 * np.cos(np.arange(64) * np.pi / 64)
        return np.sort((p[:, None] + p[None, :]).ravel())[1:11]
    path = os.path.join(HERE, "tests", "golden", f"{name}_k20.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return np.array(json.load(f)["evals_sorted"])


def ref_key(name):
    return "rel_eval_err_vs_closed_form" if name == "grid64" else "rel_eval_err_vs_oracle"


def rel_err(ev, gold):
    """Per-eigenpair relative eigenvalue error against the oracle (sorted, max and list)."""
    ev = np.sort(np.asarray(ev))
    if len(ev) != len(gold):
        return None
    e = np.abs(ev - gold) / gold
    return {"max": float(e.max()), "per_pair": [float(f"{v:.3g}") for v in e]}


def spmv_bytes(g, s):
    """Algorithmic bytes of one Laplacian product: row pointers, column indices, weights
    (if any), x read once, the degree vector and y written (s bytes per scalar)."""
    sw = 0 if g.w is None else s
    return 4 * (g.n + 1) + g.nnz * (4 + sw) + 3 * g.n * s


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, cfg, ref_stats, u0, inner_rtol, budget):
    """The FP64 oracle (plain method, same graph, start block and tolerances) on one host
    core for a bounded sample, turned into an estimate of its time to k pairs.

    * Sample: the oracle's set-up, then outer iterations until `budget` seconds.  Each outer
      iteration logs its seconds, its inner iterations, the columns of U and V it worked
      with, and the seconds of its inner solve.
    * Inner solves: the sample gives the cost per inner iteration, referred to c = 0 locked
      pairs with the slope below (the sample usually locks none): a0.  The growth with c locked pairs (deflation columns) is
      timed apart: the oracle's own inner solve with c orthonormal columns, 7 iterations
      minus 2 iterations, at c = 0 and c = min(k - 1, 24), gives a1 per iteration and
      column.  Pair j
      of the GPU's plain FP64 solve is computed with j locked pairs, so its inner
      iterations cost a0 + a1 j each.
    * The rest of an outer iteration (Ritz residual, CGS2, the new W and H columns, the
      dense eigensolver) is fitted, by non-negative least squares, as b (columns of U and
      V) + e, and applied to the GPU solve's summed basis columns and outer iterations."""
    from scipy.optimize import nnls
    from threadpoolctl import threadpool_limits

    from oracle import isira_oracle as O

    k = cfg["k"]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        res = O.isira(g, k, cfg["sigma"], cfg["tol"], u0, inner_rtol=inner_rtol,
                      time_budget=budget)
        el = time.perf_counter() - t0
        rows = np.array(res.outer_log, dtype=np.float64).reshape(-1, 4)
        if len(rows) < 3:
            return {"value": None, "unit": "s", "cores": 1, "kind": "oracle", "cpu": cpu_model(),
                    "sample": f"too few outer iterations in {el:.1f} s"}
        a0 = float(rows[:, 3].sum() / max(1.0, rows[:, 1].sum()))
        # per-iteration growth of the oracle's inner solve with the deflation columns
        L = O.laplacian(g)
        d = O.degrees(g)
        i = O.trim_index(d)
        delta = 2.0 * float(d.max())
        Lhat = O.trimmed_matrix(L, i)
        rng = np.random.default_rng(11)
        r = rng.standard_normal(g.n)
        r -= r.mean()

        def per_it(c):
            V = np.linalg.qr(rng.standard_normal((g.n, c)))[0] if c else np.zeros((g.n, 0))
            ts = []
            for its in (2, 7):
                t = time.perf_counter()
                _, done_its, _ = O.inner_solve(L, d, r, i, cfg["sigma"], delta, V, 1e-30, its, None, Lhat)
                ts.append((time.perf_counter() - t, done_its))
            return (ts[1][0] - ts[0][0]) / max(1, ts[1][1] - ts[0][1])

        c_hi = max(1, min(k - 1, 24))
        p0, p1 = per_it(0), per_it(c_hi)
        a1 = max(0.0, (p1 - p0) / c_hi)
    dense = rows[:, 0] - rows[:, 3]
    A = np.column_stack([rows[:, 2], np.ones(len(rows))])
    (b, e), _ = nnls(A, dense)
    # the sample's inner iterations ran with 0, 1, ... locked pairs: refer a0 to c = 0
    smp = np.asarray(res.inner_its, dtype=np.float64)
    c_smp = float(np.sum(smp * np.arange(len(smp))) / max(1.0, smp.sum()))
    a0 = max(0.0, a0 - a1 * c_smp)
    per_pair = np.asarray(ref_stats["inner_per_pair"], dtype=np.float64)
    inner_est = float(np.sum(per_pair * (a0 + a1 * np.arange(len(per_pair)))))
    dense_est = b * ref_stats["basis_cols_total"] + e * ref_stats["outer_total"]
    est = res.setup_seconds + inner_est + dense_est
    return {
        "value": est, "unit": "s", "cores": 1, "kind": "oracle", "cpu": cpu_model(),
        "sample": (f"oracle iSIRA (plain FP64, numpy/scipy on 1 thread) on the same graph, start block and "
                   f"tolerances: set-up {res.setup_seconds:.1f} s, then {len(rows)} outer iterations in "
                   f"{el - res.setup_seconds:.1f} s ({int(rows[:, 1].sum())} inner iterations in "
                   f"{rows[:, 3].sum():.1f} s, {res.converged} pairs locked); inner iteration "
                   f"{a0:.3g} s + {a1:.3g} s per locked pair (the oracle's inner solve timed at 0 and "
                   f"{c_hi} deflation columns: {p0:.3g} / {p1:.3g} s per iteration); rest of an outer "
                   f"iteration {b:.3g} s per basis column + {e:.3g} s; applied to the GPU plain FP64 "
                   f"solve's inner iterations per pair (total {ref_stats['inner_total']}), "
                   f"{ref_stats['basis_cols_total']} basis columns and {ref_stats['outer_total']} outer "
                   f"iterations: inner {inner_est:.1f} s, rest {dense_est:.1f} s"),
    }


def trim_study(ctx, g, cfg, opts, args):
    """Time to k pairs for several trimmed vertices (Table 2 of the paper compares a
    degree-1 vertex, vertex 1 and the maximum-degree vertex; Remark 4.1 recommends the
    last).  Thm 2.4 makes the eigenpairs independent of the choice; the work is not."""
    d = g.counts() if g.w is None else None
    if d is None:
        d = np.zeros(g.n)
        np.add.at(d, np.repeat(np.arange(g.n), np.diff(g.row_ptr)), g.w)
    choices = [("max_degree", int(np.argmax(d))), ("min_degree", int(np.argmin(d))), ("vertex_0", 0)]
    rows, ref = [], None
    for name, trim in choices:
        ts = []
        for _ in range(max(1, args.steps)):
            ev, X, res, st = ctx.solve(cfg["k"], cfg["sigma"], cfg["tol"], trim_index=trim, **opts)
            ts.append(st["ms_total"] / 1e3)
        ev = np.sort(ev)
        ref = ev if ref is None else ref
        row = {"trim": name, "vertex": trim, "degree": float(d[trim]), "median_s": float(np.median(ts)),
               "outer_total": st["outer_total"], "inner_total": st["inner_total"],
               "converged": st["n_converged"], "max_resid": float(np.max(res)),
               "max_rel_eval_diff_vs_max_degree": float(np.max(np.abs(ev - ref) / ref))
               if len(ev) == len(ref) else None}
        rows.append(row)
        log(f"trim {row}")
    print(json.dumps({"study": "trim", "workload": args.workload, "n": g.n, "nnz": g.nnz,
                      "k": cfg["k"], "tol": cfg["tol"], "rows": rows}), flush=True)


def rank_one_study(ctx, g, cfg, opts, args):
    """Remark 3.1 ablation: with sigma = lambda_1 / 2 (lambda_1 from a sigma = 0 solve), the
    inner operator with and without (sigma/n) 1-hat 1-hat^T; iterations, time, fallbacks."""
    ev0, _, _, _ = ctx.solve(cfg["k"], 0.0, cfg["tol"], **opts)
    sigma = 0.5 * float(np.min(ev0))
    rows, ref = [], None
    for name, drop in [("kept", 0), ("dropped", 1)]:
        ts = []
        for _ in range(max(1, args.steps)):
            ev, X, res, st = ctx.solve(cfg["k"], sigma, cfg["tol"], drop_rank_one=drop, **opts)
            ts.append(st["ms_total"] / 1e3)
        ev = np.sort(ev)
        ref = ev if ref is None else ref
        rows.append({"rank_one_term": name, "median_s": float(np.median(ts)), "outer_total": st["outer_total"],
                     "inner_total": st["inner_total"], "inner_fallbacks": st["inner_fallbacks"],
                     "converged": st["n_converged"], "max_resid": float(np.max(res)),
                     "max_rel_eval_diff_vs_kept": float(np.max(np.abs(ev - ref) / ref))
                     if len(ev) == len(ref) else None})
        log(f"rank1 {rows[-1]}")
    print(json.dumps({"study": "rank1", "workload": args.workload, "n": g.n, "sigma": sigma,
                      "k": cfg["k"], "tol": cfg["tol"], "rows": rows}), flush=True)


def shift_study(ctx, g, cfg, opts, args, P):
    """Algorithm 3.2's purge step moves sigma to about theta_2; with the moving shift the
    inner systems can be indefinite and are solved by MINRES.  Fixed sigma (PCG) against
    moving sigma (MINRES), FP64 and FP32 inner solves."""
    rows, ref = [], None
    for name, mode, prec in [("fixed_fp64", P.isira.SHIFT_FIXED, P.isira.FP64),
                             ("moving_fp64", P.isira.SHIFT_MOVING, P.isira.FP64),
                             ("fixed_fp32", P.isira.SHIFT_FIXED, P.isira.FP32),
                             ("moving_fp32", P.isira.SHIFT_MOVING, P.isira.FP32)]:
        ts = []
        for _ in range(max(1, args.steps)):
            ev, X, res, st = ctx.solve(cfg["k"], cfg["sigma"], cfg["tol"], shift_mode=mode,
                                       inner_prec=prec, **opts)
            ts.append(st["ms_total"] / 1e3)
        ev = np.sort(ev)
        ref = ev if ref is None else ref
        row = {"variant": name, "median_s": float(np.median(ts)), "outer_total": st["outer_total"],
               "inner_total": st["inner_total"], "inner_fallbacks": st["inner_fallbacks"],
               "sigma_last": st["sigma_last"], "converged": st["n_converged"],
               "max_resid": float(np.max(res)) if len(res) else None,
               "max_rel_eval_diff_vs_fixed_fp64": float(np.max(np.abs(ev - ref) / ref))
               if len(ev) == len(ref) else None}
        gold = golden(args.workload)
        if gold is not None:
            row[ref_key(args.workload)] = rel_err(ev, gold)
        rows.append(row)
        log(f"shift {row}")
    print(json.dumps({"study": "shift", "workload": args.workload, "n": g.n, "k": cfg["k"],
                      "tol": cfg["tol"], "rows": rows}), flush=True)


def prune_setup(ctx) -> dict:
    """Prunes the installed learned M with PRUNE_TAU; the set-up's own cost, reported."""
    t = time.perf_counter()
    kept = ctx.spai_prune(PRUNE_TAU)
    return {"prune_tau": PRUNE_TAU, "kept_offdiag": kept, "kept_frac": kept / ctx.nnz,
            "prune_setup_s": time.perf_counter() - t}


def timed_solves(ctx, cfg, steps, **opts):
    """`steps` solves of one form; returns (per-solve seconds from HIP events on the
    context's stream, the last solve's outputs)."""
    import torch

    stream = torch.cuda.current_stream()
    times, last = [], None
    for _ in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        last = ctx.solve(cfg["k"], cfg["sigma"], cfg["tol"], **opts)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    return times, last


def form_row(times, out, gold, ref_ev=None):
    ev, X, res, st = out
    row = {"median_s": float(np.median(times)), "min_s": float(np.min(times)), "solves": len(times),
           "converged": st["n_converged"], "outer_total": st["outer_total"], "inner_total": st["inner_total"],
           "max_resid": float(np.max(res)) if len(res) else None}
    if gold is not None:
        row["rel_eval_err_vs_oracle"] = rel_err(ev, gold)
    if ref_ev is not None and len(ev) == len(ref_ev):
        a, b = np.sort(ev), np.sort(ref_ev)
        row["max_rel_eval_diff_vs_plain_fp64"] = float(np.max(np.abs(a - b) / b))
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD)
    ap.add_argument("--inner-rtol", type=float, default=1e-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=40.0)
    ap.add_argument("--no-variants", action="store_true",
                    help="time only the metric's two forms (learned + FP32 and plain FP64) and FP32 Jacobi")
    ap.add_argument("--variant-steps", type=int, default=3,
                    help="solves of each further variant (moving shift, multilevel, full learned M)")
    ap.add_argument("--precond", choices=["jacobi", "learned", "learned_pruned", "multilevel"],
                    default="learned_pruned",
                    help="preconditioner of the timed form (default: the pruned learned M)")
    ap.add_argument("--inner-prec", choices=["fp64", "fp32"], default="fp32",
                    help="precision of the timed form's inner solves (default FP32)")
    ap.add_argument("--probe", action="store_true",
                    help="only a 256 MiB device copy (counter calibration) and cold launches of the "
                         "FP64 and FP32 products, for rocprofv3 counter runs")
    ap.add_argument("--probe-reps", type=int, default=20)
    ap.add_argument("--study", choices=["trim", "rank1", "shift"], default=None,
                    help="trim: the paper's Table 2 comparison of trimmed vertices (maximum "
                         "degree, a minimum-degree vertex, vertex 0) on this workload; "
                         "rank1: sigma = lambda_1 / 2 with and without the (sigma/n) 1 1^T "
                         "term of the inner operator (Remark 3.1); shift: fixed sigma = 0 (PCG) "
                         "against the purge step's moving shift (MINRES)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this solver is a design note, not an implemented path", file=sys.stderr)
        sys.exit(2)
    import torch

    import graphgen as gg
    import paper_1710_07080_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    P.load()
    t = time.perf_counter()
    g, cfg = workload(args.workload)
    log(f"graph {args.workload}: n={g.n} nnz={g.nnz} maxdeg={int(g.counts().max())} "
        f"({time.perf_counter() - t:.1f} s)")
    t = time.perf_counter()
    ctx = P.Context.from_graph(g)
    log(f"context created ({time.perf_counter() - t:.1f} s): {ctx.info()}")
    if args.probe:
        a = torch.ones(CAL_BYTES // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # the calibration copy: CAL_BYTES read, CAL_BYTES written
        torch.cuda.synchronize()
        del a, b
        ms64 = ctx.time_spmv(P.isira.FP64, reps=args.probe_reps, cold=True)
        ms32 = ctx.time_spmv(P.isira.FP32, reps=args.probe_reps, cold=True)
        print(json.dumps({"probe": args.workload, "calibration_copy_bytes": CAL_BYTES,
                          "spmv64_ms": ms64, "spmv64_bytes": spmv_bytes(g, 8),
                          "spmv32_ms": ms32, "spmv32_bytes": spmv_bytes(g, 4),
                          "reps": args.probe_reps, "cold": True}), flush=True)
        return
    u0 = gg.start_block(g.n, 4, 1)
    opts = dict(u0=u0, inner_rtol=args.inner_rtol)
    if args.study == "trim":
        trim_study(ctx, g, cfg, opts, args)
        return
    if args.study == "rank1":
        rank_one_study(ctx, g, cfg, opts, args)
        return
    if args.study == "shift":
        shift_study(ctx, g, cfg, opts, args, P)
        return
    gold = golden(args.workload)
    # ---- the timed form (default: the metric's learned + FP32)
    main_pc = {"jacobi": P.isira.PC_JACOBI, "learned": P.isira.PC_LEARNED,
               "learned_pruned": P.isira.PC_LEARNED, "multilevel": P.isira.PC_MULTILEVEL}[args.precond]
    main_prec = P.isira.FP32 if args.inner_prec == "fp32" else P.isira.FP64
    setup = {}
    if main_pc == P.isira.PC_MULTILEVEL:
        setup = ctx.ml_setup()
    elif main_pc == P.isira.PC_LEARNED:
        from paper_1710_07080_amd import spai_train

        t = time.perf_counter()
        ctx.spai_install(spai_train.load(SPAI_WEIGHTS), sigma=cfg["sigma"])
        torch.cuda.synchronize()
        setup = {"network_forward_s": time.perf_counter() - t}
        if args.precond == "learned_pruned":
            setup.update(prune_setup(ctx))
    log(f"set-up of the timed form: {setup}")
    main_opts = dict(opts, inner_prec=main_prec, precond=main_pc)
    for w in range(args.warmup):
        ev, X, res, st = ctx.solve(cfg["k"], cfg["sigma"], cfg["tol"], **main_opts)
        log(f"warmup {w}: {st['ms_total'] / 1e3:.3f} s, converged {st['n_converged']}")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    wall0 = time.perf_counter()
    step_s, stats = [], []
    for s_ in range(args.steps):
        t = time.perf_counter()
        ev, X, res, st = ctx.solve(cfg["k"], cfg["sigma"], cfg["tol"], **main_opts)
        step_s.append(time.perf_counter() - t)
        stats.append(st)
        log(f"step {s_}: {st['ms_total'] / 1e3:.3f} s, outer {st['outer_total']}, "
            f"inner {st['inner_total']}, converged {st['n_converged']}")
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sec_per_step = e0.elapsed_time(e1) / 1e3 / args.steps
    st = stats[-1]
    ok = st["n_converged"] == cfg["k"] and float(np.max(res)) < cfg["tol"]
    main_out = (ev, X, res, st)
    # ---- the plain FP64 method and FP32 Jacobi, the same number of solves, median
    ref_steps = max(1, args.steps)
    t64, out64 = timed_solves(ctx, cfg, ref_steps, inner_prec=P.isira.FP64, precond=P.isira.PC_JACOBI, **opts)
    plain = form_row(t64, out64, gold)
    log(f"plain_fp64: {plain}")
    t32, out32 = timed_solves(ctx, cfg, ref_steps, inner_prec=P.isira.FP32, precond=P.isira.PC_JACOBI, **opts)
    j32 = form_row(t32, out32, gold, out64[0])
    log(f"fp32_jacobi: {j32}")
    main_row = form_row(step_s, main_out, gold, out64[0])
    # ---- dominant kernel of the timed form: its Laplacian product (FP32 inner solves ->
    # the FP32 product), every launch timed from HBM (cold), and back to back (warm)
    kprec = "fp32" if main_prec == P.isira.FP32 else "fp64"
    kp = P.isira.FP32 if main_prec == P.isira.FP32 else P.isira.FP64
    ms_cold = ctx.time_spmv(kp, reps=100, cold=True)
    ms_warm = ctx.time_spmv(kp, reps=100, cold=False)
    kb = spmv_bytes(g, 4 if kprec == "fp32" else 8)
    achieved = kb / (ms_cold * 1e-3) / 1e9
    ms64_cold = ctx.time_spmv(P.isira.FP64, reps=100, cold=True)
    trec = measured_traffic(args.workload, kprec)
    form = (f"{args.precond} M + SMW, {args.inner_prec.upper()} inner PCG, FP64 outer"
            if main_pc == P.isira.PC_LEARNED else f"{args.precond} + SMW, {args.inner_prec.upper()} inner PCG")
    out = {
        "metric": "time to k eigpairs @ resid 1e-8 (learned+FP32 vs plain FP64); SpMV HBM GB/s",
        "value": sec_per_step,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec_per_step * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 inner, f64 outer" if main_prec == P.isira.FP32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD_TEXT.get(args.workload, args.workload),
            "n": g.n, "nnz": g.nnz, "k": cfg["k"], "sigma": cfg["sigma"], "tol": cfg["tol"],
            "form": form, "inner_rtol": args.inner_rtol,
        },
        "converged": bool(ok),
        "max_resid": float(np.max(res)),
        "outer_total": st["outer_total"],
        "inner_total": st["inner_total"],
        "median_s": main_row["median_s"],
        "phases_ms": {k: round(st[k], 2) for k in ("ms_total", "ms_inner", "ms_ortho", "ms_rr_host",
                                                  "ms_residual", "ms_restart")},
        "wall_s_per_step": wall / args.steps,
        "setup": setup,
        "plain_fp64": plain,
        "fp32_jacobi": j32,
        "learned_fp32_vs_plain_fp64": {
            "speedup_median": plain["median_s"] / main_row["median_s"],
            "learned_fp32_median_s": main_row["median_s"], "plain_fp64_median_s": plain["median_s"]},
        "learned_vs_fp32_jacobi": {"speedup_median": j32["median_s"] / main_row["median_s"]},
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": trec["bytes_per_launch"] if trec else None,
            "kernel": f"k_spmv<{'float' if kprec == 'fp32' else 'double'}, ..., TAG=1, ...> main dispatch of the "
                      f"{kprec.upper()} Laplacian product (isira_time_spmv, each launch after a 512 MiB flush)",
            "bytes_per_launch": kb, "ms_per_launch": ms_cold, "ms_per_launch_warm": ms_warm,
        },
        "spmv_fp64_cold": {"ms_per_launch": ms64_cold, "bytes_per_launch": spmv_bytes(g, 8),
                           "achieved_GBs": spmv_bytes(g, 8) / (ms64_cold * 1e-3) / 1e9},
    }
    if gold is not None:
        out[ref_key(args.workload)] = main_row.get("rel_eval_err_vs_oracle") or rel_err(ev, gold)
    out["max_rel_eval_diff_vs_plain_fp64"] = main_row.get("max_rel_eval_diff_vs_plain_fp64")
    if not args.no_variants:
        fixed, moving = P.isira.SHIFT_FIXED, P.isira.SHIFT_MOVING
        variants = [("moving_shift_fp64", P.isira.FP64, P.isira.PC_JACOBI, moving, None),
                    ("moving_shift_fp32", P.isira.FP32, P.isira.PC_JACOBI, moving, None)]
        if os.path.exists(SPAI_WEIGHTS):
            from paper_1710_07080_amd import spai_train

            def full_m():
                ctx.spai_install(spai_train.load(SPAI_WEIGHTS), sigma=cfg["sigma"])
                return {}

            variants.append(("fp32_learned_full_M", P.isira.FP32, P.isira.PC_LEARNED, fixed, full_m))
        mlinfo = ctx.ml_setup()
        out["multilevel_setup"] = {k: mlinfo[k] for k in ("levels", "rows", "connected", "coarsest_dense",
                                                          "stored_nnz", "device_bytes", "setup_ms")}
        variants += [("multilevel_fp64", P.isira.FP64, P.isira.PC_MULTILEVEL, fixed, None),
                     ("multilevel_fp32", P.isira.FP32, P.isira.PC_MULTILEVEL, fixed, None)]
        for name, prec, pc, mode, prep in variants:
            extra = prep() if prep is not None else {}
            tv, outv = timed_solves(ctx, cfg, max(1, args.variant_steps), inner_prec=prec, precond=pc,
                                    shift_mode=mode, **opts)
            row = dict(form_row(tv, outv, gold, out64[0]), **extra)
            row["speedup_vs_plain_fp64"] = plain["median_s"] / row["median_s"]
            out[name] = row
            log(f"{name}: {row}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(g, cfg, out64[3], u0, args.inner_rtol, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
