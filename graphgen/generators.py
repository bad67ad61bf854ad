"""Seeded generators of simple, connected, undirected graphs in CSR form.

Every generator returns a :class:`CSRGraph` holding only the off-diagonal pattern of
the adjacency (or weight) matrix W: ``row_ptr`` (int32, n+1), ``col`` (int32, sorted
and unique within each row, no self loops, symmetric pattern) and ``w`` (float64
weights > 0, symmetric) or ``None`` for unit weights.  The Laplacian L = D - W is
never formed here.  Random numbers come from ``numpy.random.default_rng(seed)``
(PCG64), so a (generator, arguments, seed) triple names one graph on any machine.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclasses.dataclass
class CSRGraph:
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[nnz]
    w: Optional[np.ndarray]  # float64[nnz] or None (unit weights)
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def counts(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))


def _csr_from_undirected(n, u, v, w=None, *, lcc=True, relabel_seed=None, name="", meta=None,
                         device=None):
    """Symmetrize, drop self loops and duplicates, keep the largest component,
    optionally apply a seeded random relabelling, and return sorted CSR.
    ``device`` (a torch device name) runs the same steps with torch sorts on that device
    (large graphs); the CSR it returns is identical."""
    if device is not None:
        return _csr_from_undirected_torch(n, u, v, w, lcc=lcc, relabel_seed=relabel_seed, name=name,
                                          meta=meta, device=device)
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    if w is not None:
        w = np.asarray(w, dtype=np.float64)[keep]
    # canonical undirected key (min, max); duplicates collapse to the first occurrence
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    key = a * n + b
    _, first = np.unique(key, return_index=True)
    a, b = a[first], b[first]
    if w is not None:
        w = w[first]
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    vals = None if w is None else np.concatenate([w, w])
    mat = sp.csr_matrix(
        (np.ones(rows.size) if vals is None else vals, (rows, cols)), shape=(n, n)
    )
    mat.sort_indices()
    if lcc:
        ncomp, labels = connected_components(mat, directed=False)
        if ncomp > 1:
            big = np.argmax(np.bincount(labels))
            keepv = np.flatnonzero(labels == big)
            mat = mat[keepv][:, keepv]
            n = keepv.size
    if relabel_seed is not None:
        perm = np.random.default_rng(relabel_seed).permutation(n)  # new label of old vertex
        inv = np.empty(n, dtype=np.int64)
        inv[perm] = np.arange(n)
        mat = mat[inv][:, inv]
    mat = sp.csr_matrix(mat)
    mat.sort_indices()
    row_ptr = mat.indptr.astype(np.int32)
    col = mat.indices.astype(np.int32)
    wout = None if w is None else mat.data.astype(np.float64)
    g = CSRGraph(int(n), row_ptr, col, wout, name=name, meta=dict(meta or {}))
    g.meta.update(n=int(n), nnz=g.nnz)
    return g


def _csr_from_undirected_torch(n, u, v, w, *, lcc, relabel_seed, name, meta, device):
    """The steps of _csr_from_undirected with torch on ``device``: the same edge set (the
    first occurrence of each undirected edge keeps its weight), the largest component by
    minimum-label propagation (ties: the component with the smallest vertex, as the scipy
    labelling gives), the same seeded permutation, and rows and columns sorted."""
    import torch

    dev = torch.device(device)
    u = torch.as_tensor(np.asarray(u, dtype=np.int64), device=dev)
    v = torch.as_tensor(np.asarray(v, dtype=np.int64), device=dev)
    keep = u != v
    u, v = u[keep], v[keep]
    wt = None
    if w is not None:
        wt = torch.as_tensor(np.asarray(w, dtype=np.float64), device=dev)[keep]
    del keep
    a = torch.minimum(u, v)
    b = torch.maximum(u, v)
    del u, v
    key, order = torch.sort(a * n + b, stable=True)
    first = torch.ones_like(key, dtype=torch.bool)
    first[1:] = key[1:] != key[:-1]
    del key
    pick = order[first]  # first occurrence of each edge, in increasing key order
    del order, first
    a, b = a[pick], b[pick]
    if wt is not None:
        wt = wt[pick]
    del pick
    if lcc:
        rows = torch.cat([a, b])
        cols = torch.cat([b, a])
        lab = torch.arange(n, device=dev, dtype=torch.int64)
        while True:
            nl = lab.clone()
            nl.scatter_reduce_(0, rows, lab[cols], reduce="amin", include_self=True)
            nl = nl[nl]
            if torch.equal(nl, lab):
                break
            lab = nl
        del rows, cols
        big = int(torch.argmax(torch.bincount(lab, minlength=n)))
        inlcc = lab == big
        if not bool(inlcc.all()):
            rank = torch.cumsum(inlcc.to(torch.int64), 0) - 1
            sel = inlcc[a]
            a, b = rank[a[sel]], rank[b[sel]]
            if wt is not None:
                wt = wt[sel]
            n = int(inlcc.sum())
    if relabel_seed is not None:
        perm = torch.as_tensor(np.random.default_rng(relabel_seed).permutation(n), device=dev)
        a, b = perm[a], perm[b]
    rows = torch.cat([a, b])
    cols = torch.cat([b, a])
    del a, b
    _, order = torch.sort(rows * n + cols)
    col = cols[order].to(torch.int32).cpu().numpy()
    counts = torch.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = torch.cumsum(counts, 0).cpu().numpy()
    wout = None if wt is None else torch.cat([wt, wt])[order].cpu().numpy()
    del rows, cols, order
    g = CSRGraph(int(n), row_ptr.astype(np.int32), col, wout, name=name, meta=dict(meta or {}))
    g.meta.update(n=int(n), nnz=g.nnz)
    return g


def path_graph(n: int) -> CSRGraph:
    i = np.arange(n - 1)
    return _csr_from_undirected(n, i, i + 1, lcc=False, name=f"path{n}")


def cycle_graph(n: int) -> CSRGraph:
    i = np.arange(n)
    return _csr_from_undirected(n, i, (i + 1) % n, lcc=False, name=f"cycle{n}")


def grid2d(nx: int, ny: int, weights: Optional[tuple] = None, seed: int = 0) -> CSRGraph:
    """nx-by-ny 5-point grid; vertex (x, y) -> x + nx*y; edges +x then +y per vertex."""
    return _grid([nx, ny], weights, seed, f"grid{nx}x{ny}")


def grid3d(nx: int, ny: int, nz: int, weights: Optional[tuple] = None, seed: int = 0) -> CSRGraph:
    """7-point grid; v = x + nx*y + nx*ny*z.  With ``weights=(lo, hi)`` the edge
    weights are drawn uniform(lo, hi) in the order of (v, direction in +x,+y,+z)."""
    return _grid([nx, ny, nz], weights, seed, f"grid{nx}x{ny}x{nz}")


def _grid(dims, weights, seed, name):
    dims = [int(d) for d in dims]
    n = int(np.prod(dims))
    v = np.arange(n, dtype=np.int64)
    coords = []
    rem = v.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    stride = 1
    us, vs, ds = [], [], []
    for axis, d in enumerate(dims):
        ok = coords[axis] < d - 1
        src = v[ok]
        us.append(src)
        vs.append(src + stride)
        ds.append(np.full(src.size, axis, dtype=np.int64))
        stride *= d
    u = np.concatenate(us)
    t = np.concatenate(vs)
    dirn = np.concatenate(ds)
    order = np.lexsort((dirn, u))  # vertex-major, direction-minor enumeration
    u, t = u[order], t[order]
    w = None
    if weights is not None:
        lo, hi = weights
        w = np.random.default_rng(seed).uniform(lo, hi, size=u.size)
    return _csr_from_undirected(n, u, t, w, lcc=False, name=name, meta=dict(dims=dims))


def complete_graph(n: int) -> CSRGraph:
    a, b = np.triu_indices(n, 1)
    return _csr_from_undirected(n, a, b, lcc=False, name=f"K{n}")


def star_graph(n: int) -> CSRGraph:
    """Star with n vertices: centre 0 joined to 1..n-1."""
    leaves = np.arange(1, n)
    return _csr_from_undirected(n, np.zeros(n - 1, dtype=np.int64), leaves, lcc=False, name=f"star{n}")


def hypercube(d: int) -> CSRGraph:
    n = 1 << d
    v = np.arange(n)
    us, ts = [], []
    for bit in range(d):
        nb = v ^ (1 << bit)
        m = v < nb
        us.append(v[m])
        ts.append(nb[m])
    return _csr_from_undirected(n, np.concatenate(us), np.concatenate(ts), lcc=False, name=f"Q{d}")


def spider(p: int, length: int) -> CSRGraph:
    """Centre 0 with p pendant paths of ``length`` vertices each."""
    n = 1 + p * length
    us, ts = [], []
    for leg in range(p):
        base = 1 + leg * length
        us.append(0)
        ts.append(base)
        for s in range(length - 1):
            us.append(base + s)
            ts.append(base + s + 1)
    return _csr_from_undirected(n, us, ts, lcc=False, name=f"spider{p}x{length}")


def whiskered_clique(m: int = 12) -> CSRGraph:
    """The complete graph on vertices 0..m-1 with two leaves (m, m+1) and two 2-paths
    (0-(m+2)-(m+3), 0-(m+4)-(m+5)) hanging from vertex 0: R-MAT's whiskers in miniature."""
    us = [i for i in range(m) for j in range(i + 1, m)]
    ts = [j for i in range(m) for j in range(i + 1, m)]
    us += [0, 0, 0, m + 2, 0, m + 4]
    ts += [m, m + 1, m + 2, m + 3, m + 4, m + 5]
    return _csr_from_undirected(m + 6, us, ts, lcc=False, name=f"whiskered_clique{m}")


def random_connected(n: int, extra: int, seed: int, weights: Optional[tuple] = None) -> CSRGraph:
    """Random spanning tree plus ``extra`` random edges (duplicates/self loops dropped)."""
    rng = np.random.default_rng(seed)
    order = rng.permutation(n)
    parents = order[(rng.random(n - 1) * np.arange(1, n)).astype(np.int64)]
    u = np.concatenate([order[1:], rng.integers(0, n, extra)])
    t = np.concatenate([parents, rng.integers(0, n, extra)])
    w = None
    if weights is not None:
        w = rng.uniform(weights[0], weights[1], size=u.size)
    return _csr_from_undirected(n, u, t, w, lcc=False, name=f"rand{n}_{extra}_{seed}")


def rmat(scale: int, edge_factor: int, seed: int, probs=(0.57, 0.19, 0.19, 0.05),
         relabel: bool = True, device=None) -> CSRGraph:
    """R-MAT graph: edge_factor * 2**scale edge samples, no per-level noise, then
    symmetrized, deduplicated, self loops removed, largest connected component,
    and a seeded random relabelling.  ``device``: see _csr_from_undirected."""
    a, b, c, _ = probs
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = edge_factor * n
    u = np.zeros(m, dtype=np.int64)
    v = np.zeros(m, dtype=np.int64)
    chunk = 1 << 22
    xp = np
    if device is not None:  # the same draws, with the bit arithmetic on the device
        import torch as xp
    for lo in range(0, m, chunk):
        hi = min(m, lo + chunk)
        uu = xp.zeros(hi - lo, dtype=xp.int64)
        vv = xp.zeros(hi - lo, dtype=xp.int64)
        if device is not None:
            uu, vv = uu.to(device), vv.to(device)
        for _ in range(scale):
            r = rng.random(hi - lo)
            if device is not None:
                r = xp.as_tensor(r, device=device)
            ubit = r >= a + b
            vbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
            uu = (uu << 1) | ubit
            vv = (vv << 1) | vbit
        if device is not None:
            uu, vv = uu.cpu().numpy(), vv.cpu().numpy()
        u[lo:hi] = uu
        v[lo:hi] = vv
    return _csr_from_undirected(
        n, u, v, lcc=True, relabel_seed=seed + 7919 if relabel else None,
        name=f"rmat{scale}_ef{edge_factor}_s{seed}",
        meta=dict(scale=scale, edge_factor=edge_factor, seed=seed, probs=list(probs)), device=device,
    )


def chung_lu(n: int, beta: float, avg_deg: float, seed: int, pairs_per_vertex: int = 12,
             device=None) -> CSRGraph:
    """Chung-Lu graph: expected-degree weights w_i ~ (i+1)^(-1/(beta-1)) scaled to mean
    avg_deg and capped at sqrt(sum w); pairs_per_vertex*n endpoint pairs drawn
    proportionally to w; then the largest component and a seeded relabelling.
    ``device``: see _csr_from_undirected (the endpoint search runs there too)."""
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.float64)
    wt = (i + 1.0) ** (-1.0 / (beta - 1.0))
    wt *= avg_deg / wt.mean()
    wt = np.minimum(wt, np.sqrt(wt.sum()))
    cdf = np.cumsum(wt)
    cdf /= cdf[-1]
    m = pairs_per_vertex * n
    if device is None:
        u = np.searchsorted(cdf, rng.random(m), side="right")
        v = np.searchsorted(cdf, rng.random(m), side="right")
    else:
        import torch

        cdf_t = torch.as_tensor(cdf, device=device)
        u = torch.searchsorted(cdf_t, torch.as_tensor(rng.random(m), device=device), right=True).cpu().numpy()
        v = torch.searchsorted(cdf_t, torch.as_tensor(rng.random(m), device=device), right=True).cpu().numpy()
    return _csr_from_undirected(
        n, np.minimum(u, n - 1), np.minimum(v, n - 1), lcc=True, relabel_seed=seed + 7919,
        name=f"chunglu{n}_b{beta}_d{avg_deg}_s{seed}",
        meta=dict(beta=beta, avg_deg=avg_deg, seed=seed), device=device,
    )


def start_block(n: int, k0: int, seed: int) -> np.ndarray:
    """k0 seeded N(0,1) start columns (n-by-k0, Fortran order).  The solvers remove
    the column means and orthonormalize these themselves."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((k0, n)).T)


def config_graph(name: str) -> CSRGraph:
    """The named benchmark workloads (synthetic stand-ins for the paper's networks)."""
    if name == "grid64":
        return grid2d(64, 64)
    if name == "rmat20":
        return rmat(20, 8, seed=2)
    if name == "grid128w":
        return grid3d(128, 128, 128, weights=(0.5, 1.5), seed=3)
    if name.startswith("rmat-train-"):
        s = int(name.rsplit("-", 1)[1])
        return rmat(16 + (s % 3), 8, seed=s)
    if name == "rmat22":
        return rmat(22, 16, seed=4000)
    if name == "chunglu24":
        return chung_lu(1 << 24, 2.1, 24.0, seed=5)
    raise KeyError(name)
