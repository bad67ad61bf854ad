"""FP64 CPU oracle of the learned sparse-approximate-inverse (SPAI) preconditioner.

TEST INFRASTRUCTURE ONLY (imported by the tests and never by the GPU library).

The paper leaves the M-hat_sigma slot of Remark 3.2 / eq. (3.5) open (it used a
combinatorial multigrid there); this module defines the learned replacement: a per-vertex
and per-edge network over the sparsity pattern of L-hat whose output M is symmetric and
strictly diagonally dominant with a positive diagonal (hence SPD) and approximates
(L-hat - sigma I)^{-1}.  Parameter layout (flat, F = 8, H = 16, E = 2H + 1):
    W1 (H x F), b1 (H), W2 (H x H), b2 (H), wd (2H), bd (1), We (H x E), be (H), we (H), ce (1)
Forward, with weights rounded to BF16 (round to nearest even) before use:
    t = tanh(W1 f + b1);  h = tanh(W2 t + b2);  a_i = mean_{j in N(i)} h_j
    s_i = wd . [h_i; a_i] + bd;  M_ii = softplus(s_i) / (d_i - sigma)   (0 at the trimmed vertex)
    e_ij = [h_i + h_j, h_i * h_j, w_ij / sqrt(d_i d_j)];  u = tanh(We e + be);  g = we . u + ce
    m_ij = (1 - eps) tanh(g) min(M_ii, M_jj) / max(n_i, n_j),  eps = 0.05
Features f_i = [1, log d_i, log n_i, mean_j log d_j, max_j log d_j, sigma/d_i, 1/n_i,
                [i adjacent to the trimmed vertex]].
Loss over samples (r_s, z_s):  (1/S) sum_s ||M r_s - z_s||^2 / ||z_s||^2, with the row of the
trimmed vertex of M r forced to 0.  The backward pass below is written out by hand and is
pinned by central finite differences in the tests.
Pruning (optional, after the forward pass): an off-diagonal m_ij is kept when it is nonzero
and |m_ij| >= tau sqrt(M_ii M_jj); the others become 0.  The rule is symmetric in (i, j) and
only removes off-diagonal weight, so the pruned M stays symmetric and strictly diagonally
dominant with a positive diagonal, hence SPD.
"""
from __future__ import annotations

import numpy as np

F, H = 8, 16
E = 2 * H + 1
EPS = 0.05
_sizes = [("W1", H * F), ("b1", H), ("W2", H * H), ("b2", H), ("wd", 2 * H), ("bd", 1),
          ("We", H * E), ("be", H), ("we", H), ("ce", 1)]
OFF = {}
_o = 0
for _name, _sz in _sizes:
    OFF[_name] = (_o, _sz)
    _o += _sz
NPARAM = _o


def bf16_round(p) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even); returns float64."""
    x = np.asarray(p, dtype=np.float32).copy()
    u = x.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    u = np.where(finite, r, u).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def unpack(p):
    P = {}
    for name, (o, sz) in OFF.items():
        v = np.asarray(p[o:o + sz], dtype=np.float64)
        if name == "W1":
            v = v.reshape(H, F)
        elif name == "W2":
            v = v.reshape(H, H)
        elif name == "We":
            v = v.reshape(H, E)
        elif name in ("bd", "ce"):
            v = float(v[0])
        P[name] = v
    return P


def pack(P) -> np.ndarray:
    out = np.zeros(NPARAM)
    for name, (o, sz) in OFF.items():
        out[o:o + sz] = np.ravel(P[name])
    return out


def init_params(seed: int = 0) -> np.ndarray:
    """Small random weights; bd makes softplus(s) = 1 (the Jacobi diagonal) at start."""
    rng = np.random.default_rng(seed)
    P = {
        "W1": rng.standard_normal((H, F)) * 0.3, "b1": np.zeros(H),
        "W2": rng.standard_normal((H, H)) * 0.3, "b2": np.zeros(H),
        "wd": rng.standard_normal(2 * H) * 0.05, "bd": float(np.log(np.e - 1.0)),
        "We": rng.standard_normal((H, E)) * 0.3, "be": np.zeros(H),
        "we": rng.standard_normal(H) * 0.1, "ce": 0.5,
    }
    return pack(P).astype(np.float32)


def _graph_arrays(g):
    rp = g.row_ptr.astype(np.int64)
    col = g.col.astype(np.int64)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    w = np.ones(g.nnz) if g.w is None else np.asarray(g.w, dtype=np.float64)
    d = np.zeros(g.n)
    np.add.at(d, rows, w)
    cnt = np.diff(rp).astype(np.float64)
    return rp, col, rows, w, d, cnt


def features(g, sigma: float, trim: int) -> np.ndarray:
    rp, col, rows, w, d, cnt = _graph_arrays(g)
    ld = np.log(d)
    f = np.zeros((g.n, F))
    f[:, 0] = 1.0
    f[:, 1] = ld
    f[:, 2] = np.log(cnt)
    s = np.zeros(g.n)
    np.add.at(s, rows, ld[col])
    f[:, 3] = s / cnt
    mx = np.full(g.n, -np.inf)
    np.maximum.at(mx, rows, ld[col])
    f[:, 4] = mx
    f[:, 5] = sigma / d
    f[:, 6] = 1.0 / cnt
    adj = np.zeros(g.n)
    adj[rows[col == trim]] = 1.0
    f[:, 7] = adj
    return f


def softplus(x):
    return np.maximum(x, 0) + np.log1p(np.exp(-np.abs(x)))


def forward(g, params, sigma: float, trim: int, round_bf16: bool = True):
    """Returns a dict with M's diagonal ("diag") and stored off-diagonal values ("offd", in
    the CSR order of g) plus the intermediates used by the backward pass."""
    p = bf16_round(params) if round_bf16 else np.asarray(params, dtype=np.float64)
    P = unpack(p)
    rp, col, rows, w, d, cnt = _graph_arrays(g)
    f = features(g, sigma, trim)
    t = np.tanh(f @ P["W1"].T + P["b1"])
    h = np.tanh(t @ P["W2"].T + P["b2"])
    a = np.zeros((g.n, H))
    np.add.at(a, rows, h[col])
    a /= cnt[:, None]
    s = h @ P["wd"][:H] + a @ P["wd"][H:] + P["bd"]
    diag = softplus(s) / (d - sigma)
    diag[trim] = 0.0
    e = np.concatenate([h[rows] + h[col], h[rows] * h[col], (w / np.sqrt(d[rows] * d[col]))[:, None]], axis=1)
    u = np.tanh(e @ P["We"].T + P["be"])
    gg = u @ P["we"] + P["ce"]
    th = np.tanh(gg)
    mn = np.minimum(diag[rows], diag[col])
    mx = np.maximum(cnt[rows], cnt[col])
    offd = (1 - EPS) * th * mn / mx
    return dict(P=P, f=f, t=t, h=h, a=a, s=s, diag=diag, e=e, u=u, th=th, mn=mn, mx=mx,
                offd=offd, rows=rows, col=col, d=d, cnt=cnt)


def apply(g, diag, offd, trim: int, X: np.ndarray) -> np.ndarray:
    """Y = M X (columns of X are vectors); row `trim` of the result is 0."""
    rp, col, rows, w, d, cnt = _graph_arrays(g)
    X2 = X if X.ndim == 2 else X[:, None]
    Y = diag[:, None] * X2
    np.add.at(Y, rows, offd[:, None] * X2[col])
    Y[trim] = 0.0
    return Y if X.ndim == 2 else Y[:, 0]


def prune(g, diag, offd, tau: float) -> np.ndarray:
    """Off-diagonal values after pruning with threshold tau (rule in the module docstring),
    in the CSR order of g; the decision is taken in FP64 from the values given."""
    rp, col, rows, w, d, cnt = _graph_arrays(g)
    diag = np.asarray(diag, dtype=np.float64)
    offd = np.asarray(offd, dtype=np.float64)
    keep = (offd != 0.0) & (np.abs(offd) >= tau * np.sqrt(diag[rows] * diag[col]))
    return np.where(keep, offd, 0.0)


def dense_M(g, diag, offd) -> np.ndarray:
    rp, col, rows, w, d, cnt = _graph_arrays(g)
    M = np.diag(diag)
    M[rows, col] = offd
    return M


def loss(g, params, sigma, trim, R, Z, round_bf16=True) -> float:
    """R, Z: n-by-S (column s = sample s; entry `trim` of each column is 0)."""
    fw = forward(g, params, sigma, trim, round_bf16)
    Y = apply(g, fw["diag"], fw["offd"], trim, R)
    S = R.shape[1]
    zz = np.sum(Z * Z, axis=0)
    return float(np.sum(np.sum((Y - Z) ** 2, axis=0) / zz) / S)


def loss_grad(g, params, sigma, trim, R, Z, round_bf16=True):
    """Loss and its gradient with respect to the (rounded) parameters, by hand."""
    fw = forward(g, params, sigma, trim, round_bf16)
    P = fw["P"]
    rows, col, d, cnt = fw["rows"], fw["col"], fw["d"], fw["cnt"]
    n = g.n
    Y = apply(g, fw["diag"], fw["offd"], trim, R)
    S = R.shape[1]
    zz = np.sum(Z * Z, axis=0)
    L = float(np.sum(np.sum((Y - Z) ** 2, axis=0) / zz) / S)
    G = 2.0 * (Y - Z) / (S * zz)[None, :]  # dL/dY; row trim: Y = Z = 0 there
    G[trim] = 0.0
    # dL/d(stored value m_ij) = sum_s G_is R_js; the shared value m_ij = m_ji collects both
    g_dir = np.sum(G[rows] * R[col], axis=1)
    # map each stored entry to its transpose
    key = rows * n + col
    tkey = col * n + rows
    order = np.argsort(key)
    tpos = order[np.searchsorted(key[order], tkey)]
    dm = g_dir + g_dir[tpos]
    own = rows < col  # each undirected edge once
    dM = np.sum(G * R, axis=1)  # direct diagonal term
    # through m = (1 - eps) th mn / mx
    th, mn, mx, u = fw["th"], fw["mn"], fw["mx"], fw["u"]
    dg = dm * (1 - EPS) * (1 - th ** 2) * mn / mx
    dmn = dm * (1 - EPS) * th / mx
    Mi, Mj = fw["diag"][rows], fw["diag"][col]
    share_i = np.where(Mi < Mj, 1.0, np.where(Mi == Mj, 0.5, 0.0))
    np.add.at(dM, rows, np.where(own, dmn * share_i, 0.0))
    np.add.at(dM, col, np.where(own, dmn * (1.0 - share_i), 0.0))
    # edge head
    dpre = (dg[:, None] * P["we"][None, :]) * (1 - u ** 2)
    grads = {}
    grads["we"] = np.sum(np.where(own[:, None], dg[:, None] * u, 0.0), axis=0)
    grads["ce"] = float(np.sum(np.where(own, dg, 0.0)))
    grads["We"] = np.where(own[:, None], dpre, 0.0).T @ fw["e"]
    grads["be"] = np.sum(np.where(own[:, None], dpre, 0.0), axis=0)
    de = np.where(own[:, None], dpre, 0.0) @ P["We"]  # (nnz, E)
    h = fw["h"]
    dh = np.zeros((n, H))
    np.add.at(dh, rows, de[:, :H] + de[:, H:2 * H] * h[col])
    np.add.at(dh, col, de[:, :H] + de[:, H:2 * H] * h[rows])
    # diagonal head
    sig = 1.0 / (1.0 + np.exp(-fw["s"]))
    ds = dM * sig / (d - sigma)
    ds[trim] = 0.0
    grads["wd"] = np.concatenate([ds @ h, ds @ fw["a"]])
    grads["bd"] = float(np.sum(ds))
    dh += ds[:, None] * P["wd"][None, :H]
    da = ds[:, None] * P["wd"][None, H:]
    # aggregation a_i = mean_j h_j  ->  dh_j += da_i / n_i
    np.add.at(dh, col, da[rows] / cnt[rows][:, None])
    # vertex MLP
    dpre2 = dh * (1 - h ** 2)
    grads["W2"] = dpre2.T @ fw["t"]
    grads["b2"] = np.sum(dpre2, axis=0)
    dt = dpre2 @ P["W2"]
    dpre1 = dt * (1 - fw["t"] ** 2)
    grads["W1"] = dpre1.T @ fw["f"]
    grads["b1"] = np.sum(dpre1, axis=0)
    return L, pack(grads)
