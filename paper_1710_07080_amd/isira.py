"""ctypes binding of libisira (the gfx950 iSIRA library declared in include/isira.h).

Argument marshalling only: every step of the solver runs in the library's HIP kernels.
PyTorch supplies device memory (CUDA tensors on ROCm) and the stream.  The binding
refuses to run without the built library; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisira.so")

ISIRA_OK = 0
ISIRA_NOT_CONVERGED = 1
ISIRA_E_ARG = -1
ISIRA_E_GRAPH = -2
ISIRA_E_DISCONNECTED = -3
ISIRA_E_HIP = -4
ISIRA_E_PRECOND = -5
ISIRA_E_STATE = -6
ISIRA_E_WORKSPACE = -7
ISIRA_E_HOST = -8
WS_LEARNED = 1
W_NONE, W_F32, W_F64 = 0, 1, 2
FP64, FP32 = 0, 1
PC_JACOBI, PC_LEARNED, PC_MULTILEVEL = 0, 1, 2
SOLVER_PCG, SOLVER_MINRES = 0, 1
SHIFT_FIXED, SHIFT_MOVING = 0, 1
MAX_K = 64
STATS_MAX = 64
ML_MAX_LEVELS = 32

_c_double_p = ctypes.POINTER(ctypes.c_double)
_c_int32_p = ctypes.POINTER(ctypes.c_int32)


class IsiraError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"isira error {code}: {message}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int32), ("q", ctypes.c_int32), ("k0", ctypes.c_int32),
        ("inner_rtol", ctypes.c_double), ("max_inner", ctypes.c_int32),
        ("max_outer", ctypes.c_int32), ("inner_prec", ctypes.c_int32),
        ("precond", ctypes.c_int32), ("trim_index", ctypes.c_int64), ("delta", ctypes.c_double),
        ("seed", ctypes.c_uint64), ("u0", _c_double_p), ("check_every", ctypes.c_int32),
        ("verbose", ctypes.c_int32), ("capture_r", _c_double_p), ("capture_z", _c_double_p),
        ("capture_cap", ctypes.c_int32), ("capture_count", _c_int32_p),
        ("drop_rank_one", ctypes.c_int32), ("shift_mode", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_converged", ctypes.c_int32), ("outer_total", ctypes.c_int32),
        ("inner_total", ctypes.c_int64), ("spmv_total", ctypes.c_int64),
        ("restarts", ctypes.c_int32), ("breakdowns", ctypes.c_int32),
        ("refreshes", ctypes.c_int32), ("inner_fallbacks", ctypes.c_int32),
        ("inner_capped", ctypes.c_int32),
        ("outer_per_pair", ctypes.c_int32 * STATS_MAX), ("inner_per_pair", ctypes.c_int32 * STATS_MAX),
        ("ms_total", ctypes.c_double), ("ms_inner", ctypes.c_double), ("ms_ortho", ctypes.c_double),
        ("ms_rr_host", ctypes.c_double), ("ms_residual", ctypes.c_double),
        ("ms_restart", ctypes.c_double), ("trim_index", ctypes.c_int64), ("delta", ctypes.c_double),
        ("sigma_last", ctypes.c_double), ("basis_cols_total", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        k = self.n_converged
        d = {f: getattr(self, f) for f, _ in self._fields_ if f not in ("outer_per_pair", "inner_per_pair")}
        d["outer_per_pair"] = list(self.outer_per_pair)[:k]
        d["inner_per_pair"] = list(self.inner_per_pair)[:k]
        return d


class Info(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("trim_index", ctypes.c_int64),
        ("max_degree", ctypes.c_double), ("min_degree", ctypes.c_double),
        ("delta_default", ctypes.c_double), ("norm1", ctypes.c_double),
        ("n_spmv_units", ctypes.c_int32), ("n_spmv_blocks", ctypes.c_int32),
        ("n_split_rows", ctypes.c_int32), ("has_learned", ctypes.c_int32),
    ]


class MlOptions(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("coarse_max", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("trim_index", ctypes.c_int64)]


class MlInfo(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("rows", ctypes.c_int64 * ML_MAX_LEVELS),
        ("offdiag_nnz", ctypes.c_int64 * ML_MAX_LEVELS), ("connected", ctypes.c_int64 * ML_MAX_LEVELS),
        ("coarsest_dense", ctypes.c_int64), ("stored_nnz", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64), ("setup_ms", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        L = self.levels
        return dict(levels=L, rows=list(self.rows[:L]), offdiag_nnz=list(self.offdiag_nnz[:L]),
                    connected=list(self.connected[:L]), coarsest_dense=self.coarsest_dense,
                    stored_nnz=self.stored_nnz, device_bytes=self.device_bytes, setup_ms=self.setup_ms)


EXPORTS = [
    "isira_default_options", "isira_create", "isira_create_ws", "isira_workspace_bytes",
    "isira_memory_info", "isira_destroy", "isira_get_info", "isira_solve",
    "isira_laplacian_apply", "isira_laplacian_apply_f32", "isira_time_spmv", "isira_inner_solve",
    "isira_orthonormalize", "isira_orthonormalize_noalloc", "isira_symeig", "isira_symeig_lowest", "isira_spai_nparam", "isira_spai_install",
    "isira_spai_prune", "isira_spai_export", "isira_spai_loss_grad", "isira_adam_step", "isira_ml_default_options",
    "isira_ml_setup", "isira_ml_get_info", "isira_ml_apply", "isira_ml_shape", "isira_ml_level_matrix", "isira_strerror",
    "isira_last_error",
]

_lib = None


def load() -> ctypes.CDLL:
    """Load libisira.so from the package directory (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with paper_1710_07080_amd/build.py "
                          "(or __graft_entry__.build())")
    # torch's HIP runtime must be the one in the process before the library binds to it:
    # device memory and streams come from torch, and a second runtime loaded first may not
    # see the device
    import torch  # noqa: F401

    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "isira_default_options": (i32, [ctypes.POINTER(Options)]),
        "isira_create": (i32, [ctypes.POINTER(vp), i64, i64, vp, vp, vp, i32, vp, i32]),
        "isira_destroy": (None, [vp]),
        "isira_create_ws": (i32, [ctypes.POINTER(vp), i64, i64, vp, vp, vp, i32, i32, vp, ctypes.c_size_t,
                                  i32, ctypes.POINTER(Options), vp, i32]),
        "isira_workspace_bytes": (ctypes.c_size_t, [i64, i64, i32, i32, ctypes.POINTER(Options), i32]),
        "isira_memory_info": (i32, [vp, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.POINTER(ctypes.c_size_t)]),
        "isira_get_info": (i32, [vp, ctypes.POINTER(Info)]),
        "isira_solve": (i32, [vp, i32, dbl, dbl, ctypes.POINTER(Options), vp, vp, vp,
                              ctypes.POINTER(Stats)]),
        "isira_laplacian_apply": (i32, [vp, vp, vp]),
        "isira_laplacian_apply_f32": (i32, [vp, vp, vp]),
        "isira_time_spmv": (i32, [vp, i32, i32, i32, _c_double_p]),
        "isira_inner_solve": (i32, [vp, vp, vp, i32, dbl, dbl, i64, dbl, i32, i32, i32, i32, vp,
                                    _c_int32_p, _c_double_p]),
        "isira_orthonormalize": (i32, [vp, vp, i32, vp, vp, _c_double_p]),
        "isira_orthonormalize_noalloc": (i32, [vp, vp, i32, vp, vp, _c_double_p]),
        "isira_symeig": (i32, [i32, vp, vp, vp]),
        "isira_symeig_lowest": (i32, [i32, vp, vp, vp]),
        "isira_spai_nparam": (i32, []),
        "isira_spai_install": (i32, [vp, vp, dbl, i64]),
        "isira_spai_prune": (i32, [vp, dbl, ctypes.POINTER(i64)]),
        "isira_spai_export": (i32, [vp, vp, vp]),
        "isira_spai_loss_grad": (i32, [vp, vp, dbl, i64, vp, vp, i32, vp, _c_double_p]),
        "isira_adam_step": (i32, [vp, vp, vp, vp, vp, i32, ctypes.c_float, ctypes.c_float,
                                  ctypes.c_float, ctypes.c_float, i32]),
        "isira_ml_default_options": (i32, [ctypes.POINTER(MlOptions)]),
        "isira_ml_setup": (i32, [vp, ctypes.POINTER(MlOptions), ctypes.POINTER(MlInfo)]),
        "isira_ml_get_info": (i32, [vp, ctypes.POINTER(MlInfo)]),
        "isira_ml_apply": (i32, [vp, i32, vp, vp]),
        "isira_ml_shape": (i32, [i64, vp, vp, vp, i64, ctypes.POINTER(MlOptions), ctypes.POINTER(MlInfo)]),
        "isira_ml_level_matrix": (i32, [i64, vp, vp, vp, i64, ctypes.POINTER(MlOptions), i32,
                                        ctypes.POINTER(i64), ctypes.POINTER(i64), vp, vp, vp, vp, vp]),
        "isira_strerror": (ctypes.c_char_p, [i32]),
        "isira_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, allow_not_converged: bool = False) -> int:
    if rc == ISIRA_OK or (allow_not_converged and rc == ISIRA_NOT_CONVERGED):
        return rc
    lib = load()
    raise IsiraError(rc, lib.isira_last_error().decode() or lib.isira_strerror(rc).decode())


def _ptr(t) -> int:
    """Device pointer of a torch tensor, or host pointer of a numpy array."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _require_cuda(t, dtype, numel, name):
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous CUDA tensor of dtype {dtype}")
    if t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, needs {numel}")


def workspace_bytes(n: int, nnz: int, k: int, w_dtype: int = W_NONE, flags: int = 0, **opts) -> int:
    """isira_workspace_bytes: device bytes of a context made by Context.with_workspace."""
    o = default_options()
    for key, val in opts.items():
        setattr(o, key, val)
    return int(load().isira_workspace_bytes(int(n), int(nnz), int(w_dtype), int(k), ctypes.byref(o), int(flags)))


def default_options() -> Options:
    o = Options()
    _check(load().isira_default_options(ctypes.byref(o)))
    return o


def symeig(H: np.ndarray):
    """All eigenpairs of a symmetric matrix with the library's host eigensolver."""
    H = np.asfortranarray(H, dtype=np.float64)
    k = H.shape[0]
    theta = np.zeros(k)
    S = np.zeros((k, k), order="F")
    _check(load().isira_symeig(k, _ptr(H), _ptr(theta), _ptr(S)))
    return theta, S


def ml_shape(g, trim: int, omega: float = 0.9, coarse_max: int = 512, max_levels: int = 24) -> dict:
    """Host-only shape of the multilevel hierarchy for graph g (caller labels)."""
    o = MlOptions()
    o.omega, o.coarse_max, o.max_levels, o.trim_index = float(omega), int(coarse_max), int(max_levels), int(trim)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w, dtype=np.float64)
    inf = MlInfo()
    _check(load().isira_ml_shape(int(g.n), rp.ctypes.data, col.ctypes.data,
                                 None if w is None else w.ctypes.data, int(trim), ctypes.byref(o),
                                 ctypes.byref(inf)))
    return inf.as_dict()


def ml_level_matrix(g, trim: int, level: int, omega: float = 0.9, coarse_max: int = 512,
                    max_levels: int = 24):
    """Host-only level `level` of the multilevel hierarchy for graph g (caller labels):
    (scipy CSR of the off-diagonal weights, diagonal, aggregation map into the next level)."""
    import scipy.sparse as sp

    o = MlOptions()
    o.omega, o.coarse_max, o.max_levels, o.trim_index = float(omega), int(coarse_max), int(max_levels), int(trim)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w, dtype=np.float64)
    lib = load()
    rows, nnz = ctypes.c_int64(), ctypes.c_int64()
    args = (int(g.n), rp.ctypes.data, col.ctypes.data, None if w is None else w.ctypes.data, int(trim),
            ctypes.byref(o), int(level), ctypes.byref(rows), ctypes.byref(nnz))
    _check(lib.isira_ml_level_matrix(*args, None, None, None, None, None))
    m, e = rows.value, nnz.value
    orp = np.zeros(m + 1, dtype=np.int32)
    ocol = np.zeros(max(e, 1), dtype=np.int32)
    ow = np.zeros(max(e, 1))
    od = np.zeros(m)
    oagg = np.zeros(m, dtype=np.int32)
    _check(lib.isira_ml_level_matrix(*args, orp.ctypes.data, ocol.ctypes.data, ow.ctypes.data, od.ctypes.data,
                                     oagg.ctypes.data))
    W = sp.csr_matrix((ow[:e], ocol[:e], orp), shape=(m, m))
    return W, od, oagg


def symeig_lowest(H: np.ndarray):
    """All eigenvalues and a unit eigenvector of the smallest, with the library's host
    routine for outer iterations that lock nothing."""
    H = np.asfortranarray(H, dtype=np.float64)
    k = H.shape[0]
    theta = np.zeros(k)
    s1 = np.zeros(k)
    _check(load().isira_symeig_lowest(k, _ptr(H), _ptr(theta), _ptr(s1)))
    return theta, s1


def current_stream() -> int:
    import torch

    return torch.cuda.current_stream().cuda_stream


class Context:
    """One graph on one GPU (``isira_create``)."""

    def __init__(self, n: int, row_ptr: np.ndarray, col: np.ndarray, w: Optional[np.ndarray] = None,
                 stream: Optional[int] = None, validate: bool = True):
        lib = load()
        self._lib = lib
        self.n = int(n)
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        wdt = W_NONE
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w)
            if w.dtype == np.float32:
                wdt = W_F32
            else:
                w = w.astype(np.float64, copy=False)
                wdt = W_F64
            wp = _ptr(w)
        self.nnz = int(row_ptr[-1])
        handle = ctypes.c_void_p()
        s = current_stream() if stream is None else stream
        _check(lib.isira_create(ctypes.byref(handle), self.n, self.nnz, _ptr(row_ptr), _ptr(col), wp,
                                wdt, s, 1 if validate else 0))
        self._h = handle

    @classmethod
    def with_workspace(cls, n: int, row_ptr, col, w=None, *, workspace, k: int, stream: Optional[int] = None,
                       validate: bool = True, **opts) -> "Context":
        """isira_create_ws: every device buffer of the context is carved from `workspace` (a
        CUDA uint8 tensor the caller keeps alive); row_ptr/col/w may be numpy arrays (host) or
        CUDA tensors (device).  opts size the solve workspace (m, q) as for solve()."""
        import torch

        lib = load()
        self = cls.__new__(cls)
        self._lib = lib
        self.n = int(n)
        on_dev = isinstance(row_ptr, torch.Tensor)
        if on_dev:
            for t, dt in ((row_ptr, torch.int32), (col, torch.int32)):
                _require_cuda(t, dt, 1, "CSR array")
            self.nnz = int(col.numel())
        else:
            row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
            col = np.ascontiguousarray(col, dtype=np.int32)
            self.nnz = int(row_ptr[-1])
        wdt = W_NONE
        if w is not None:
            if on_dev:
                wdt = W_F32 if w.dtype == torch.float32 else W_F64
            else:
                w = np.ascontiguousarray(w)
                if w.dtype != np.float32:
                    w = w.astype(np.float64, copy=False)
                wdt = W_F32 if w.dtype == np.float32 else W_F64
        if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda):
            raise TypeError("workspace must be a CUDA tensor")
        o = default_options()
        for key, val in opts.items():
            setattr(o, key, val)
        self._workspace = workspace  # the context's memory lives there
        handle = ctypes.c_void_p()
        s = current_stream() if stream is None else stream
        _check(lib.isira_create_ws(ctypes.byref(handle), self.n, self.nnz, _ptr(row_ptr), _ptr(col), _ptr(w), wdt,
                                   1 if on_dev else 0, workspace.data_ptr(),
                                   workspace.numel() * workspace.element_size(), int(k), ctypes.byref(o), s,
                                   1 if validate else 0))
        self._h = handle
        return self

    def memory_info(self) -> dict:
        a, b, c = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(self._lib.isira_memory_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"in_use": a.value, "peak": b.value, "capacity": c.value}

    @classmethod
    def from_graph(cls, g, weights_dtype=None, **kw) -> "Context":
        w = g.w
        if w is not None and weights_dtype is not None:
            w = w.astype(weights_dtype)
        return cls(g.n, g.row_ptr, g.col, w, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.isira_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = Info()
        _check(self._lib.isira_get_info(self._h, ctypes.byref(inf)))
        return {f: getattr(inf, f) for f, _ in inf._fields_}

    def solve(self, k: int, sigma: float = 0.0, tol: float = 1e-8, *, u0: Optional[np.ndarray] = None,
              capture=None, **opts):
        """Algorithm 3.2.  Returns (evals, evecs, resid, stats): evals/resid numpy, evecs a
        CUDA tensor of shape (k, n) (row j is eigenvector j)."""
        import torch

        o = default_options()
        for key, val in opts.items():
            if not hasattr(o, key):
                raise KeyError(key)
            setattr(o, key, val)
        if u0 is not None:
            u0 = np.asfortranarray(u0, dtype=np.float64)
            if u0.shape[0] != self.n:
                raise ValueError("u0 must be n-by-k0")
            o.k0 = u0.shape[1]
            o.u0 = u0.ctypes.data_as(_c_double_p)
        count = ctypes.c_int32(0)
        if capture is not None:
            cr, cz = capture
            _require_cuda(cr, torch.float64, self.n, "capture_r")
            _require_cuda(cz, torch.float64, self.n, "capture_z")
            o.capture_r = ctypes.cast(cr.data_ptr(), _c_double_p)
            o.capture_z = ctypes.cast(cz.data_ptr(), _c_double_p)
            o.capture_cap = cr.numel() // self.n
            o.capture_count = ctypes.pointer(count)
        evals = np.zeros(k)
        resid = np.zeros(k)
        evecs = torch.zeros((k, self.n), dtype=torch.float64, device="cuda")
        st = Stats()
        rc = self._lib.isira_solve(self._h, int(k), float(sigma), float(tol), ctypes.byref(o), _ptr(evals),
                                   _ptr(evecs), _ptr(resid), ctypes.byref(st))
        _check(rc, allow_not_converged=True)
        stats = st.as_dict()
        stats["return_code"] = rc
        stats["captured"] = count.value
        kc = st.n_converged
        return evals[:kc], evecs[:kc], resid[:kc], stats

    def laplacian_apply(self, x):
        import torch

        _require_cuda(x, torch.float64, self.n, "x")
        y = torch.empty_like(x)
        _check(self._lib.isira_laplacian_apply(self._h, _ptr(x), _ptr(y)))
        return y

    def laplacian_apply_f32(self, x):
        import torch

        _require_cuda(x, torch.float32, self.n, "x")
        y = torch.empty_like(x)
        _check(self._lib.isira_laplacian_apply_f32(self._h, _ptr(x), _ptr(y)))
        return y

    def time_spmv(self, prec: int = FP64, reps: int = 50, cold: bool = False) -> float:
        """Average ms per launch of the product's main dispatch (cold: each launch from HBM)."""
        ms = ctypes.c_double(0)
        _check(self._lib.isira_time_spmv(self._h, int(prec), int(reps), 1 if cold else 0, ctypes.byref(ms)))
        return ms.value

    def inner_solve(self, r, V=None, sigma: float = 0.0, delta: float = 0.0, trim: int = -1,
                    rtol: float = 1e-10, max_it: int = 5000, prec: int = FP64,
                    precond: int = PC_JACOBI, solver: int = SOLVER_PCG):
        """Trimmed, shifted, deflated solve (2.15) + enlargement (2.5).  r: CUDA float64 (n),
        V: CUDA float64 (c, n) rows = deflation vectors.  Returns (z, iters, relres)."""
        import torch

        _require_cuda(r, torch.float64, self.n, "r")
        c = 0
        vp = None
        if V is not None and V.numel() > 0:
            _require_cuda(V, torch.float64, V.shape[0] * self.n, "V")
            c = V.shape[0]
            vp = _ptr(V)
        z = torch.empty_like(r)
        its = ctypes.c_int32(0)
        rel = ctypes.c_double(0)
        _check(self._lib.isira_inner_solve(self._h, _ptr(r), vp, c, float(sigma), float(delta), int(trim),
                                           float(rtol), int(max_it), int(prec), int(precond), int(solver),
                                           _ptr(z),
                                           ctypes.byref(its), ctypes.byref(rel)))
        return z, its.value, rel.value

    def orthonormalize(self, Q, z):
        """CGS2 of z against the rows of Q (CUDA float64 (ncols, n)) and 1/sqrt(n)."""
        import torch

        _require_cuda(z, torch.float64, self.n, "z")
        nc = 0 if Q is None else Q.shape[0]
        if nc:
            _require_cuda(Q, torch.float64, nc * self.n, "Q")
        u = torch.empty_like(z)
        norms = np.zeros(2)
        _check(self._lib.isira_orthonormalize(self._h, _ptr(Q) if nc else None, nc, _ptr(z), _ptr(u),
                                              norms.ctypes.data_as(_c_double_p)))
        return u, norms

    def orthonormalize_noalloc(self, Q, z, u):
        """The same CGS2 through the allocation-free entry point, into the caller's u."""
        import torch

        _require_cuda(z, torch.float64, self.n, "z")
        _require_cuda(u, torch.float64, self.n, "u")
        nc = 0 if Q is None else Q.shape[0]
        if nc:
            _require_cuda(Q, torch.float64, nc * self.n, "Q")
        norms = np.zeros(2)
        _check(self._lib.isira_orthonormalize_noalloc(self._h, _ptr(Q) if nc else None, nc, _ptr(z),
                                                      _ptr(u), norms.ctypes.data_as(_c_double_p)))
        return norms

    # ---- multilevel preconditioner ----
    def ml_setup(self, omega: Optional[float] = None, coarse_max: Optional[int] = None,
                 max_levels: Optional[int] = None, trim: int = -1) -> dict:
        """Build the aggregation-multigrid hierarchy of L-hat; returns its statistics."""
        o = MlOptions()
        _check(self._lib.isira_ml_default_options(ctypes.byref(o)))
        if omega is not None:
            o.omega = float(omega)
        if coarse_max is not None:
            o.coarse_max = int(coarse_max)
        if max_levels is not None:
            o.max_levels = int(max_levels)
        o.trim_index = int(trim)
        inf = MlInfo()
        _check(self._lib.isira_ml_setup(self._h, ctypes.byref(o), ctypes.byref(inf)))
        return inf.as_dict()

    def ml_info(self) -> dict:
        inf = MlInfo()
        _check(self._lib.isira_ml_get_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    def ml_apply(self, x, prec: int = FP64):
        """One V-cycle on the trimmed x (CUDA float64, n); the trimmed entry of the result is 0."""
        import torch

        _require_cuda(x, torch.float64, self.n, "x")
        y = torch.empty_like(x)
        _check(self._lib.isira_ml_apply(self._h, int(prec), _ptr(x), _ptr(y)))
        return y

    # ---- learned preconditioner ----
    def spai_install(self, params, sigma: float = 0.0, trim: int = -1):
        import torch

        _require_cuda(params, torch.float32, spai_nparam(), "params")
        _check(self._lib.isira_spai_install(self._h, _ptr(params), float(sigma), int(trim)))

    def spai_prune(self, tau: float) -> int:
        """Prune the installed learned M (isira_spai_prune); returns the kept off-diagonal
        count."""
        kept = ctypes.c_int64(0)
        _check(self._lib.isira_spai_prune(self._h, float(tau), ctypes.byref(kept)))
        return int(kept.value)

    def spai_export(self):
        import torch

        diag = torch.empty(self.n, dtype=torch.float32, device="cuda")
        offd = torch.empty(self.nnz, dtype=torch.float32, device="cuda")
        _check(self._lib.isira_spai_export(self._h, _ptr(diag), _ptr(offd)))
        return diag, offd

    def spai_loss_grad(self, params, r, z, sigma: float = 0.0, trim: int = -1):
        """r, z: CUDA float32 (S, n) (row s = sample s).  Returns (loss, grad)."""
        import torch

        S = r.shape[0]
        _require_cuda(params, torch.float32, spai_nparam(), "params")
        _require_cuda(r, torch.float32, S * self.n, "r")
        _require_cuda(z, torch.float32, S * self.n, "z")
        grad = torch.empty_like(params)
        loss = ctypes.c_double(0)
        _check(self._lib.isira_spai_loss_grad(self._h, _ptr(params), float(sigma), int(trim), _ptr(r), _ptr(z),
                                              int(S), _ptr(grad), ctypes.byref(loss)))
        return loss.value, grad

    def adam_step(self, param, grad, m, v, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, step=1):
        _check(self._lib.isira_adam_step(self._h, _ptr(param), _ptr(grad), _ptr(m), _ptr(v), param.numel(),
                                         lr, beta1, beta2, eps, int(step)))


def spai_nparam() -> int:
    return int(load().isira_spai_nparam())
