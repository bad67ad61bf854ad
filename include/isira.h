/*
 * isira.h -- C ABI of the MI355X (gfx950) implementation of iSIRA, the integrated
 * shift-invert residual Arnoldi method for the smallest positive eigenpairs of a graph
 * Laplacian (Huang, Lin, Lu, Yau, arXiv 1710.07080).
 *
 * Problem (Section 1.1, Algorithm 3.2): given a simple, connected, undirected graph with
 * positive edge weights W (Remark 1.3), find the k smallest positive eigenvalues of
 * L = D - W (eq. (1.1)) and orthonormal eigenvectors, all orthogonal to the null vector 1
 * (Theorem 1.2).
 *
 * Conventions shared by every entry point:
 *   - Return value: ISIRA_OK (0), ISIRA_NOT_CONVERGED (1), or a negative ISIRA_E_* code.
 *     No exception crosses the ABI.  isira_strerror() names a code; isira_last_error()
 *     gives the message of the last failure on this thread.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP device memory
 *     of the GPU the context was created on (e.g. torch CUDA tensors on ROCm).  The caller
 *     owns every pointer it passes; the library copies what it keeps.
 *   - Vectors passed to or returned from a context use the caller's vertex labels.
 *     Internally the library relabels vertices (by decreasing row length, or in reverse
 *     Cuthill-McKee order when no row is longer than a product work unit and the gathers do
 *     not concentrate on a few hubs) and maps back.
 *   - Dense n-by-c blocks are column-major with leading dimension n unless stated.
 *   - A context is not thread-safe; calls on one context must not overlap.
 *   - All GPU work of a context runs on the stream given at creation (NULL = default).
 */
#ifndef ISIRA_H
#define ISIRA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define ISIRA_OK 0
#define ISIRA_NOT_CONVERGED 1   /* max_outer reached: the first stats->n_converged pairs are valid */
#define ISIRA_E_ARG (-1)        /* bad argument (k, sigma, tol, m, q, sizes, null pointers) */
#define ISIRA_E_GRAPH (-2)      /* CSR not simple/undirected: bad index, self loop, unsorted or
                                   duplicate column, asymmetric pattern or weight, weight <= 0 */
#define ISIRA_E_DISCONNECTED (-3) /* the graph has more than one connected component */
#define ISIRA_E_HIP (-4)        /* a HIP runtime call failed (allocation, launch, copy) */
#define ISIRA_E_PRECOND (-5)    /* the learned preconditioner is missing or not usable */
#define ISIRA_E_STATE (-6)      /* entry point called in the wrong state */
#define ISIRA_E_WORKSPACE (-7)  /* the caller's workspace is too small for this call */
#define ISIRA_E_HOST (-8)       /* host-side failure, e.g. host memory exhausted (no C++ exception
                                   crosses an entry point) */

/* ---- weight dtypes ---- */
#define ISIRA_W_NONE 0 /* unit weights (plain adjacency A) */
#define ISIRA_W_F32 1
#define ISIRA_W_F64 2

/* ---- inner-solve precision ---- */
#define ISIRA_FP64 0
#define ISIRA_FP32 1

/* ---- inner preconditioner ---- */
#define ISIRA_PC_JACOBI 0  /* M-hat_sigma = diag(d - sigma), Remark 3.2, with eq. (3.5) */
#define ISIRA_PC_LEARNED 1 /* learned sparse approximate inverse, with eq. (3.5) */
#define ISIRA_PC_MULTILEVEL 2 /* aggregation multigrid V-cycle for L-hat (the multilevel
                                 slot of Section 3), with eq. (3.5); set up by isira_ml_setup */

/* ---- inner solver ---- */
#define ISIRA_SOLVER_PCG 0    /* preconditioned conjugate gradients (SPD systems) */
#define ISIRA_SOLVER_MINRES 1 /* preconditioned MINRES (symmetric, possibly indefinite) */

/* ---- shift strategy ---- */
#define ISIRA_SHIFT_FIXED 0   /* sigma stays the caller's value (inner solver PCG) */
#define ISIRA_SHIFT_MOVING 1  /* Algorithm 3.2's purge step: sigma <- theta_2 after each locked
                                 pair, capped at half the minimum degree (inner solver MINRES) */

#define ISIRA_MAX_K 64        /* at most 64 wanted pairs per solve */
#define ISIRA_MAX_BASIS 192   /* m (maximal search-space dimension) is at most 192 */

typedef struct isira_ctx isira_ctx;

/* Options of one solve.  Zero / negative fields select the documented default. */
typedef struct {
  int32_t m;            /* maximal search-space dimension (Algorithm 3.2); default 2*q */
  int32_t q;            /* restart size; default k + 10 */
  int32_t k0;           /* start-block columns; default 4 */
  double inner_rtol;    /* inner PCG stop: ||r_hat - K_hat z|| <= inner_rtol ||r_hat||; default 1e-1 */
  int32_t max_inner;    /* PCG iteration cap per inner solve; default 1000 */
  int32_t max_outer;    /* cap on outer iterations of the whole solve; default 20000 */
  int32_t inner_prec;   /* ISIRA_FP64 (default) or ISIRA_FP32 */
  int32_t precond;      /* ISIRA_PC_JACOBI (default), ISIRA_PC_LEARNED or ISIRA_PC_MULTILEVEL */
  int64_t trim_index;   /* trimmed vertex (caller label); -1 = max degree, lowest label on ties */
  double delta;         /* deflation shift; <= 0 selects 2 * max diag(L) (Remark 4.1(ii)) */
  uint64_t seed;        /* seed of the SplitMix64 replacement vectors (breakdowns, default start) */
  const double* u0;     /* host, n-by-k0 column-major start block (caller labels), or NULL:
                           then column j is SplitMix64(seed) at counters (j*n + l) */
  int32_t check_every;  /* PCG iterations launched between convergence read-backs; default 8 */
  int32_t verbose;      /* 1: print one line per locked pair to stderr */
  /* optional capture of inner-solve pairs (device, caller labels), for preconditioner
     training: column j of capture_z (n-by-capture_cap, FP64) receives the solution z_hat
     of inner solve j (trimmed entry 0) and column j of capture_r receives
     (L-hat - sigma I) z_hat, i.e. the pair an approximate inverse of L-hat - sigma I
     should map onto each other; *capture_count (host) is the number written. */
  double* capture_r;
  double* capture_z;
  int32_t capture_cap;
  int32_t* capture_count;
  int32_t drop_rank_one;  /* 1: leave the rank-one term (sigma/n) 1-hat 1-hat^T out of the inner
                             operator (the simplification Remark 3.1 allows for large n);
                             default 0 keeps the exact operator of eq. (2.15) */
  int32_t shift_mode;     /* ISIRA_SHIFT_FIXED (default) or ISIRA_SHIFT_MOVING; the moving shift
                             is not combined with the learned preconditioner (ISIRA_E_PRECOND) */
} isira_options;

#define ISIRA_STATS_MAX 64
typedef struct {
  int32_t n_converged;
  int32_t outer_total;                 /* outer (Rayleigh-Ritz) iterations */
  int64_t inner_total;                 /* PCG iterations */
  int64_t spmv_total;                  /* Laplacian applications (all precisions) */
  int32_t restarts, breakdowns, refreshes, inner_fallbacks, inner_capped;
  int32_t outer_per_pair[ISIRA_STATS_MAX];
  int32_t inner_per_pair[ISIRA_STATS_MAX];
  /* wall time (ms) of the whole solve and of its phases: inner solves (with the first batch
     of each, queued behind the Ritz residual), orthonormalization and expansion, host
     Rayleigh-Ritz, the Ritz residual kernels (HIP events), restarts and purges */
  double ms_total, ms_inner, ms_ortho, ms_rr_host, ms_residual, ms_restart;
  int64_t trim_index;                  /* caller label of the trimmed vertex */
  double delta;
  double sigma_last;                   /* the shift of the last inner solve */
  int64_t basis_cols_total;            /* sum over outer iterations of the basis width plus
                                          the locked pairs (the columns its dense steps read) */
} isira_stats;

typedef struct {
  int64_t n, nnz;
  int64_t trim_index;    /* caller label of the default trim vertex */
  double max_degree, min_degree, delta_default, norm1; /* norm1 = ||L||_1 = 2 max diag(L) */
  int32_t n_spmv_units, n_spmv_blocks, n_split_rows;
  int32_t has_learned;   /* 1 once learned preconditioner values are installed */
} isira_info;

/* Fill *opt with the defaults. */
int isira_default_options(isira_options* opt);

/* Create a context for one graph.  row_ptr (n+1), col (nnz) and w (nnz, or NULL when
 * w_dtype == ISIRA_W_NONE) are HOST arrays of the off-diagonal adjacency in CSR form:
 * sorted unique columns, no self loops, symmetric pattern and weights, weights > 0.
 * The library validates the graph (E_GRAPH), checks connectivity (E_DISCONNECTED),
 * relabels it, uploads its own copy, and computes on the GPU the weighted degrees,
 * the trim index (Remark 4.1(i)) and delta (Remark 4.1(ii)).
 * stream: a hipStream_t (NULL = default stream).  validate: 0 skips the O(nnz log d)
 * symmetry check (the caller vouches for the input). */
int isira_create(isira_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                 const int32_t* col, const void* w, int32_t w_dtype, void* stream,
                 int32_t validate);

/* ---- caller-owned device memory (the boundary's workspace form) ----
 * isira_workspace_bytes: an upper bound of the device bytes one context needs for a graph of
 * n vertices and nnz stored off-diagonal entries (weights of dtype w_dtype) to run
 * isira_create_ws and then isira_solve for up to k pairs with the options opt (NULL: the
 * defaults; m and k size the basis U, W of Algorithm 3.2 and the deflation blocks).  flags:
 * ISIRA_WS_LEARNED adds the learned preconditioner's buffers (isira_spai_install and
 * isira_spai_prune).  The multilevel hierarchy (isira_ml_setup) and the training entry points
 * need more, which their sizes decide; on a workspace context they take it from the
 * workspace and fail with ISIRA_E_WORKSPACE when it is short.  Returns 0 for invalid sizes. */
#define ISIRA_WS_LEARNED 1
size_t isira_workspace_bytes(int64_t n, int64_t nnz, int32_t w_dtype, int32_t k,
                             const isira_options* opt, int32_t flags);
/* isira_create with caller-owned device memory: every device buffer of the context (the
 * relabelled CSR, degrees, the SpMV plan, reduction buffers, and the solve workspace for k
 * pairs with options opt, sized here at creation) is carved from `workspace` (device,
 * ws_bytes bytes, owned by the caller and kept alive until isira_destroy); the library makes
 * no device allocation.  csr_on_device: 0 = row_ptr/col/w are host arrays as for
 * isira_create, 1 = they are device arrays (read once into a host copy for validation and
 * relabelling).  Pinned host buffers (a few KB plus a 1 MiB upload ring) are still the
 * library's.  Errors as isira_create, plus ISIRA_E_WORKSPACE when ws_bytes is short (take
 * isira_workspace_bytes).  A later solve with a larger k or m than sized here, or any call
 * that needs more device memory, fails with ISIRA_E_WORKSPACE instead of allocating. */
int isira_create_ws(isira_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                    const int32_t* col, const void* w, int32_t w_dtype, int32_t csr_on_device,
                    void* workspace, size_t ws_bytes, int32_t k, const isira_options* opt,
                    void* stream, int32_t validate);
/* Device bytes of the context now in use and at most (both contexts), and the workspace's
 * usable size (0 for a context that allocates its own memory); any pointer may be NULL. */
int isira_memory_info(const isira_ctx* ctx, size_t* in_use, size_t* peak, size_t* capacity);

void isira_destroy(isira_ctx* ctx);
int isira_get_info(const isira_ctx* ctx, isira_info* info);

/* Algorithm 3.2: the k smallest positive eigenpairs (1 <= k <= min(ISIRA_MAX_K, n-2)).
 * sigma: fixed shift of the inner systems, 0 <= sigma < min degree (the caller
 *   promises sigma < lambda_1 so the trimmed system (2.15) stays positive definite).
 * tol: outer tolerance on ||W s_1 - theta_1 U s_1||_2; a pair is locked only when the
 *   fresh FP64 residual ||L y - theta y||_2 also satisfies it.
 * evals: host, k, ascending order of locking.  evecs: device, n-by-k column-major FP64,
 *   caller labels, unit norm, orthogonal to 1, largest-magnitude entry positive.
 * resid: host, k, ||L v - lambda v||_2 in FP64.  stats: host, may be NULL.
 * Returns ISIRA_OK, ISIRA_NOT_CONVERGED (max_outer hit), or an error. */
int isira_solve(isira_ctx* ctx, int32_t k, double sigma, double tol, const isira_options* opt,
                double* evals, double* evecs, double* resid, isira_stats* stats);

/* ---- operator-level entry points (kernel parity and measurement) ---- */

/* y = L x in FP64 (eq. (1.1)); x, y device, n, caller labels. */
int isira_laplacian_apply(isira_ctx* ctx, const double* x, double* y);
/* y = L x with FP32 vectors and FP32 weights (the inner-solve operator precision). */
int isira_laplacian_apply_f32(isira_ctx* ctx, const float* x, float* y);
/* Time `reps` launches of the main dispatch of the FP64 (prec 0) or FP32 (prec 1) Laplacian
 * product (kernel symbol k_spmv<..., TAG = 1, ...>) on internal vectors, with HIP events on
 * the context stream; *ms_per = average ms per launch.  cold = 0: back-to-back launches
 * (the graph may stay in the 256 MB memory-side cache between them); cold = 1: before each
 * launch a 512 MiB device buffer (taken from the context's memory and released afterwards)
 * is read and written, and each launch is timed on its own, so every launch starts from
 * HBM.  The finishing dispatch of rows split into chunks (a few of the longest rows) is left
 * out, so the probe's output is not a complete product and is not used. */
int isira_time_spmv(isira_ctx* ctx, int32_t prec, int32_t reps, int32_t cold, double* ms_per);

/* One inner solve of Algorithm 3.2's expansion step: solve the trimmed, shifted,
 * deflated system (2.15) for r_hat = r with entry `trim` deleted, by PCG with the
 * Remark 3.2 preconditioner (Jacobi or learned, with eq. (3.5) when c > 0), then enlarge
 * by eq. (2.5).  r: device n FP64 (must be orthogonal to 1), V: device n-by-c FP64
 * (orthonormal, orthogonal to 1; c <= ISIRA_MAX_K), trim: caller label or -1,
 * delta <= 0 selects the default.  z: device n FP64 output.  *iters, *relres: host. */
int isira_inner_solve(isira_ctx* ctx, const double* r, const double* V, int32_t c,
                      double sigma, double delta, int64_t trim, double rtol, int32_t max_it,
                      int32_t prec, int32_t precond, int32_t solver, double* z,
                      int32_t* iters, double* relres);

/* Classical Gram-Schmidt applied twice against the ncols orthonormal columns of Q and
 * the unit vector 1/sqrt(n), then normalization (the orthonormalization step of
 * Algorithm 3.2).  Q: device n-by-ncols (ld n), z: device n input, u: device n output;
 * norms (host, 2): ||z|| before and after.  Returns ISIRA_OK even on breakdown (u is then
 * z scaled by 1/after, possibly inf); the caller inspects norms. */
int isira_orthonormalize(isira_ctx* ctx, const double* Q, int32_t ncols, const double* z,
                         double* u, double* norms);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same orthonormalization as
 * isira_orthonormalize -- classical Gram-Schmidt applied twice against the ncols columns of
 * Q and 1/sqrt(n), then u = z_after / ||z_after|| (u = 0 when that norm is 0) -- that calls
 * no hipMalloc, hipFree or allocating routine.  Q: device n-by-ncols (ld n), z: device n
 * (read only), u: device n output (must not overlap z or Q), norms (host, 2): ||z|| before
 * and after; all in the caller's labels.  Intermediates live in a fixed device array of the
 * library (2 MiB, one per GPU, held until the process ends): ncols is limited to
 * 0..ISIRA_MAX_BASIS (E_ARG beyond).  Calls that overlap on one GPU (other streams or
 * threads) share that array and race; the call returns after its stream has finished. */
int isira_orthonormalize_noalloc(isira_ctx* ctx, const double* Q, int32_t ncols,
                                 const double* z, double* u, double* norms);

/* Host-only: all eigenpairs of a symmetric k-by-k matrix H (column-major), eigenvalues
 * ascending in theta (k), unit eigenvectors in the columns of S (k-by-k column-major)
 * -- the Rayleigh-Ritz step of Algorithm 3.2.  Householder tridiagonalization followed
 * by the implicit QL iteration.  No GPU needed. */
int isira_symeig(int32_t k, const double* H, double* theta, double* S);
/* Host-only: all eigenvalues of the same kind of matrix (theta, k, ascending) and a unit
 * eigenvector s1 (k) of the smallest -- what an outer iteration of Algorithm 3.2 needs when
 * no pair is locked and no restart follows.  The same tridiagonalization, the QL iteration
 * without eigenvectors, then inverse iteration with the tridiagonal matrix shifted by
 * theta[0] (Gaussian elimination with partial pivoting), mapped back through the
 * Householder reflections.  No GPU needed. */
int isira_symeig_lowest(int32_t k, const double* H, double* theta, double* s1);

/* ---- learned sparse approximate inverse (SPAI) preconditioner ---- */
/* The network maps per-vertex features through a vertex MLP, one mean-aggregation over
 * neighbours, a diagonal head and a symmetric edge head to the values of a matrix M on
 * the pattern of L-hat that is symmetric and strictly diagonally dominant with a
 * positive diagonal, hence SPD; M approximates (L-hat - sigma I)^{-1}.
 * Parameters are one flat FP32 vector of ISIRA_SPAI_NPARAM values (layout in the
 * binding); the forward pass rounds them to BF16 and accumulates in FP32. */
#define ISIRA_SPAI_F 8   /* vertex features */
#define ISIRA_SPAI_H 16  /* hidden width */
int32_t isira_spai_nparam(void);
/* Compute M for (graph, sigma, trim) from params (device FP32) and install it in the
 * context as the ISIRA_PC_LEARNED preconditioner. */
int isira_spai_install(isira_ctx* ctx, const float* params, double sigma, int64_t trim);
/* Prune the installed M: an off-diagonal m_ij is kept when it is nonzero and
 * |m_ij| >= tau * sqrt(M_ii * M_jj) (decided in FP64 from the stored FP32 values); the
 * others become 0.  The rule is symmetric in (i, j) and removes only off-diagonal weight,
 * so M stays symmetric and strictly diagonally dominant with a positive diagonal (SPD), a
 * valid M-hat_sigma for Remark 3.2.  tau = 0 keeps every nonzero.  Afterwards every apply
 * of M (inner PCG, the Y = M V-hat columns of eq. (3.5), isira_spai_export) uses the pruned
 * matrix; the PCG step then applies it by one thread per row, fused with the dots of the
 * Jacobi form, which pays off when few entries per row are kept (tau around 0.01-0.1 for
 * the trained network).  Install again to undo (pruning a pruned M starts from the pruned
 * values).  *kept (host, may be NULL): the number of stored off-diagonal entries kept.
 * While it runs it holds host copies of the pattern and the values (about 9 bytes per
 * stored entry, 8 more per kept one).  Errors: ISIRA_E_ARG (tau < 0 or not finite),
 * ISIRA_E_PRECOND (no learned M installed, or values found not symmetric), ISIRA_E_HIP (a
 * failed upload leaves no learned M installed). */
int isira_spai_prune(isira_ctx* ctx, double tau, int64_t* kept);
/* Export the installed M: diag (device n FP32, caller labels) and off-diagonal values
 * (device nnz FP32) in the caller's CSR order. */
int isira_spai_export(isira_ctx* ctx, float* diag, float* offd);
/* Loss and gradient for a batch of samples: loss = (1/S) sum_s ||M r_s - z_s||^2 /
 * ||z_s||^2 with r_s, z_s device n-by-S FP32 column-major (caller labels, trimmed entry
 * 0).  grad: device FP32 (nparam), overwritten.  *loss: host. */
int isira_spai_loss_grad(isira_ctx* ctx, const float* params, double sigma, int64_t trim,
                         const float* r, const float* z, int32_t S, float* grad,
                         double* loss);
/* One Adam step on device FP32 vectors (param, grad, m, v of length count). */
int isira_adam_step(isira_ctx* ctx, float* param, const float* grad, float* m, float* v,
                    int32_t count, float lr, float beta1, float beta2, float eps,
                    int32_t step);

/* ---- multilevel preconditioner (the multilevel solver slot of Section 3) ----
 * An unsmoothed-aggregation multigrid V-cycle approximating L-hat^{-1}, L-hat the
 * Laplacian with the trimmed vertex deleted (eq. (2.4)); Remark 3.2 allows any SPD
 * approximation of the trimmed operator, and eq. (3.5) adds the deflation term as for
 * Jacobi.  The shift is not part of the hierarchy, which is built once per trim index.
 *   Levels: A_0 = L-hat, A_{l+1} = P_l^T A_l P_l with P_l the 0/1 aggregation matrix.
 *   Aggregation, on the graph of A_l's off-diagonal pattern: a vertex without neighbours
 *   belongs to no aggregate; the others are visited by decreasing number of neighbours
 *   (ties: caller label on the finest level, index on coarser ones); a visited vertex
 *   that is unassigned with all neighbours unassigned forms an aggregate with them (ids in
 *   order of creation); each vertex left then joins, among these aggregates holding one of
 *   its neighbours, the one holding the most (ties: smallest id).
 *   A level with at most coarse_max vertices that have neighbours is the coarsest and is
 *   solved exactly (dense Cholesky inverse; 1/A_vv for a vertex without neighbours).
 *   Cycle: one damped Jacobi sweep, weight omega (1 for a vertex without neighbours),
 *   before and after the coarse correction, from x = 0: symmetric positive definite for
 *   0 < omega < 1.
 * The set-up runs on the host (O(nnz) per level) and uploads the matrices of each level's
 * two sparse products; it replaces any previous hierarchy of the context. */
#define ISIRA_ML_MAX_LEVELS 32
typedef struct {
  double omega;        /* smoothing weight, 0 < omega < 1; default 0.9 */
  int32_t coarse_max;  /* 0..2048; default 512 (0: coarsen until no vertex has a neighbour) */
  int32_t max_levels;  /* 1..ISIRA_ML_MAX_LEVELS; default 24 (E_PRECOND if not enough) */
  int64_t trim_index;  /* caller label of the trimmed vertex; -1 = the default trim vertex */
} isira_ml_options;
typedef struct {
  int32_t levels;                            /* including the finest and the coarsest */
  int64_t rows[ISIRA_ML_MAX_LEVELS];         /* vertices per level (finest: n - 1) */
  int64_t offdiag_nnz[ISIRA_ML_MAX_LEVELS];  /* stored off-diagonal entries of A_l */
  int64_t connected[ISIRA_ML_MAX_LEVELS];    /* vertices with at least one neighbour */
  int64_t coarsest_dense;                    /* order of the coarsest level's dense inverse */
  int64_t stored_nnz;                        /* entries of all transfer-product matrices */
  int64_t device_bytes;                      /* device memory held by the hierarchy */
  double setup_ms;                           /* host wall time of isira_ml_setup */
} isira_ml_info;
int isira_ml_default_options(isira_ml_options* opt);
/* Build the hierarchy for opt->trim_index (opt may be NULL: defaults).  info: host, may be
 * NULL.  E_ARG for options out of range, E_PRECOND if max_levels does not suffice. */
int isira_ml_setup(isira_ctx* ctx, const isira_ml_options* opt, isira_ml_info* info);
int isira_ml_get_info(const isira_ctx* ctx, isira_ml_info* info);
/* Host-only: the shape (levels, rows, stored entries, connected vertices, coarsest dense
 * order, transfer-matrix entries) of the hierarchy that isira_ml_setup builds, for host CSR
 * arrays in the caller's labels (no relabelling; the rule breaks ties by label either way),
 * off-diagonal weights w (n nnz doubles, or NULL for unit weights) and the trimmed vertex
 * trim (caller label); opt must be given.  No GPU is touched; device_bytes and setup_ms
 * stay 0. */
int isira_ml_shape(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* w,
                   int64_t trim, const isira_ml_options* opt, isira_ml_info* info);
/* Host-only: level `level` (0 = L-hat) of the hierarchy isira_ml_shape describes, for the
 * parity of its Galerkin products A_{l+1} = P_l^T A_l P_l: rows (*rows) and stored
 * off-diagonal entries (*nnz) of A_l; when rp_out is not NULL also its CSR (rp_out rows+1,
 * col_out / w_out nnz, where w_out holds the positive weights w_ij and the matrix entry is
 * -w_ij), its diagonal (diag_out, rows) and the aggregate of each vertex on the next level
 * (agg_out, rows; -1 for a vertex in no aggregate and on the coarsest level).  Level 0 is in
 * the caller's labels with the trimmed vertex's row empty and its diagonal 0; a coarse level
 * numbers its vertices in the order of their aggregates' first members on the finer level.
 * All outputs are host arrays; no GPU is touched. */
int isira_ml_level_matrix(int64_t n, const int32_t* row_ptr, const int32_t* col, const double* w,
                          int64_t trim, const isira_ml_options* opt, int32_t level, int64_t* rows,
                          int64_t* nnz, int32_t* rp_out, int32_t* col_out, double* w_out,
                          double* diag_out, int32_t* agg_out);
/* y = cycle(x-hat) enlarged by a zero at the trimmed vertex; x, y device n FP64, caller
 * labels (x's trimmed entry is ignored).  prec: ISIRA_FP64, or ISIRA_FP32 (the cycle in
 * FP32 vectors and matrix values, as inside FP32 inner solves).  E_STATE before set-up. */
int isira_ml_apply(isira_ctx* ctx, int32_t prec, const double* x, double* y);

const char* isira_strerror(int code);
const char* isira_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ISIRA_H */
