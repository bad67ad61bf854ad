// Internal declarations of the gfx950 iSIRA library: device state, SpMV plan, launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "isira.h"

namespace isira {

// Device memory of one context.  By default each block is its own hipMalloc; once a
// caller's workspace is attached (isira_create_ws) every block is carved from that one range
// instead (first fit, 256-byte aligned, freed blocks merged with their neighbours), and the
// library makes no device allocation of its own.
class DevMem {
 public:
  static constexpr size_t kAlign = 256;
  void attach(void* base, size_t bytes);
  bool external() const { return base_ != nullptr; }
  // ISIRA_OK; ISIRA_E_WORKSPACE when the attached workspace has no free range that large;
  // ISIRA_E_HIP when hipMalloc fails.  *p is nullptr on failure.
  int alloc(void** p, size_t bytes);
  void release(void* p);
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }
  size_t capacity() const { return cap_; }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0;
  std::map<size_t, size_t> free_;           // offset -> bytes of the free ranges
  std::unordered_map<void*, size_t> live_;  // block -> bytes
  size_t in_use_ = 0, peak_ = 0;
};

// Typed helpers: count elements of T (at least one); the error text goes to the thread's
// last-error message.
int dev_alloc_bytes(DevMem& m, void** p, size_t bytes);
template <typename T>
int dalloc(DevMem& m, T** p, size_t count) {
  return dev_alloc_bytes(m, (void**)p, (count == 0 ? 1 : count) * sizeof(T));
}
template <typename T>
void dfree(DevMem& m, T*& p) {
  if (p) m.release((void*)p);
  p = nullptr;
}
inline size_t dev_round(size_t bytes) {
  return ((bytes == 0 ? 1 : bytes) + DevMem::kAlign - 1) / DevMem::kAlign * DevMem::kAlign;
}

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
#ifndef ISIRA_STREAM_GRID
#define ISIRA_STREAM_GRID 1024
#endif
// max workgroups of grid-stride streaming kernels (compile-time tunable)
constexpr int kStreamGrid = ISIRA_STREAM_GRID;
constexpr int kSpmvGrid = 2048;       // max workgroups of the persistent SpMV grid
#ifndef ISIRA_UNIT_NNZ
#define ISIRA_UNIT_NNZ 2048
#define ISIRA_UNIT_ROWS 512
#endif
constexpr int kUnitNnz = ISIRA_UNIT_NNZ;    // nonzeros per SpMV unit (stream unit or long-row chunk)
constexpr int kUnitRows = ISIRA_UNIT_ROWS;  // rows per stream unit at most
// hub-cached shape for power-law graphs: two 512-thread workgroups per CU, each with x of
// the highest-degree labels in LDS (about 78 KB of LDS per workgroup in either precision)
#ifndef ISIRA_HUB_THREADS
#define ISIRA_HUB_THREADS 512
#define ISIRA_HUB_GRID 512
#endif
constexpr int kHubThreads = ISIRA_HUB_THREADS;
#ifndef ISIRA_HUB_UNNZ
#define ISIRA_HUB_UNNZ 4096
#define ISIRA_HUB_UROWS 1024
#define ISIRA_HUB_X64 4352
#define ISIRA_HUB_X32 13312
#endif
constexpr int kHubUnitNnz = ISIRA_HUB_UNNZ;
constexpr int kHubUnitRows = ISIRA_HUB_UROWS;
constexpr int kHubX64 = ISIRA_HUB_X64;  // FP64 x entries staged in LDS
constexpr int kHubX32 = ISIRA_HUB_X32;  // FP32 x entries staged in LDS
constexpr int kHubGrid = ISIRA_HUB_GRID;
// the hub-cached shape is chosen when a quarter of the gathers hit the kHubTestCols
// highest-degree labels
constexpr int kHubTestCols = 8192;
constexpr int kMaxC = ISIRA_MAX_K;     // deflation columns in the inner solve
constexpr int kTile = 512;             // rows per tile of the column-dot kernels
constexpr int kMaxCols = 2 * ISIRA_MAX_BASIS + 2;  // columns of one multi-dot
constexpr size_t kUploadRing = 1 << 20;            // pinned bytes for small uploads
// Values x workgroups of the largest reduction in the learned-preconditioner backward pass.
constexpr int kSpaiRedValues = 600;
constexpr int kSpaiRedGrid = 512;
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
// workgroups of a grid-stride streaming kernel over n rows (one partial per workgroup)
inline int stream_grid(int n) {
  int g = (n + kBlock - 1) / kBlock;
  return g < 1 ? 1 : (g > kStreamGrid ? kStreamGrid : g);
}

// The PCG kernels process the c deflation columns in whole groups: c rounded up to the next
// of these sizes.  The columns past c are allocated, finite (zeroed once) and weighted by 0.
inline int pick_cm(int c) {
  if (c <= 0) return 0;
  if (c <= 24) return (c + 3) / 4 * 4;
  if (c <= 48) return (c + 7) / 8 * 8;
  return 64;
}

// Capacity (doubles) of the shared partials buffer: every reducing kernel writes at most
// values x workgroups of it, each checked against this bound at compile time.  The
// product's own partials sit after the p-update's, which its finishing dispatch reads.
constexpr size_t kSpmvPartOff = (size_t)(1 + kMaxC) * kStreamGrid;
constexpr size_t kPartialsElems =
    cmax(cmax((size_t)kMaxCols * kStreamGrid, kSpmvPartOff + (size_t)4 * kSpmvGrid),
         (size_t)kSpaiRedValues * kSpaiRedGrid);

// SpMV work units (int4, device), built on the host from the relabelled CSR:
//   stream unit  {r0, j0, j1, rows << 8 | G}: rows [r0, r0 + rows) holding nonzeros
//                [j0, j1) (at most the unit size); their products are staged in LDS and
//                each row is summed by G lanes;
//   chunk unit   {row, j0, j1, -(p + 1)}: nonzeros [j0, j1) of a row longer than the unit
//                size, whose sum goes to split_part[p] and is finished by the second
//                dispatch.

// Scalars of the inner PCG and of the outer reductions, living in device memory.
struct DevState {
  double alpha, beta, rho, pq, rr, rr0, rmr, thresh2, rtol2, sump, sumx;
  double red[4];  // generic reduction outputs
  int32_t it, done, status, maxit;
  double t1[kMaxC];  // V-hat^T p
  double t2[kMaxC + 1];  // V-hat^T (M^-1 r); learned variant: [V-hat^T y, r^T y]
  double g[kMaxC];   // G^{-1} t2
  // MINRES: gamma_{j-1}, c_j, c_{j-1}, s_j, s_{j-1}, eta, eta_0, alpha_1, alpha_2, alpha_3
  // (gamma_j in rho, delta_j in pq, c_{j+1} eta in alpha); last_it: the iteration whose
  // solution update still runs after the test has stopped the iteration
  double mr[10];
  int32_t last_it;
  int32_t cgs_skip;  // 1: the second Gram-Schmidt pass is not needed (see launch_dgks_decide)
};

enum PcgStatus { kPcgOk = 0, kPcgCapped = 1, kPcgBreakdown = 2 };

// Reduction scratch shared by kernels on one stream (kernels run one after another): each
// reducing kernel writes one partial per workgroup and value, and a finishing dispatch
// sums them in a fixed order.
struct RedBuf {
  double* partials;   // max(kMaxCols * kStreamGrid, 4 * kSpmvGrid) doubles
  unsigned* counters; // 64 counters (setup kernels only), zeroed at creation
};

// SpMV execution plan (device arrays for split rows).
struct SpmvPlan {
  int hub = 0;  // 1: hub-cached shape
  int4* units = nullptr;
  int32_t n_units = 0;
  int32_t grid = 0;
  int32_t n_split_units = 0, n_split_rows = 0;
  int32_t* split_rowof = nullptr;  // per split row slot: the row
  int32_t* split_base = nullptr;   // per split row slot: first chunk partial index
  int32_t* split_nchunk = nullptr; // per split row slot: number of chunks
  double* split_part = nullptr;    // per chunk partial neighbour sums
  double* split_red = nullptr;     // per split row slot: reduction contribution
};

// Work units of the sparse product for a CSR matrix of n rows (host arrays); the plan's
// device arrays are allocated from mem here and released by free_spmv_plan.
int build_spmv_plan(DevMem& mem, int n, const int32_t* rp, const int32_t* col, SpmvPlan& P);
void free_spmv_plan(DevMem& mem, SpmvPlan& P);
// Upper bound of the bytes build_spmv_plan allocates for a matrix of n rows and nnz entries.
size_t spmv_plan_bytes_bound(int64_t n, int64_t nnz);

// Value mode of the sparse product y = diag .* x + sgn * sum_j v_ij x_j.
enum ValMode { kUnitNeg = 0, kF32Neg = 1, kF64Neg = 2, kF32Pos = 3, kF64Pos = 4 };

// Arguments of the fused sparse product.
template <typename T>
struct SpmvArgs {
  const int32_t* rp;
  const int32_t* col;
  const void* vals;    // weights (kF32Neg/kF64Neg) or learned values (kF32Pos)
  const T* x;
  T* y;
  const T* diag;
  int32_t n;
  int32_t trim;        // row forced to zero (-1: none)
  double sigma;        // y -= sigma x
  double sig_over_n;   // y += sig_over_n * st->sump
  const T* V;          // y += delta * V t, t = st->t1 (inner) or tvec
  int64_t ldv;
  int32_t c;
  const double* tvec;
  double delta;
  int32_t red;         // 0 none; 1 PCG p^T q -> alpha; 2 ||y - theta x||^2 -> st->red[0];
                       // 3 x^T y -> st->red[1]; 4 MINRES z^T q -> st->pq only
  double theta;
  DevState* st;
  int32_t check_done;  // return at once when st->done
  // PCG product (red 1) only: the deflation term delta V-hat (V-hat^T p) and the rank-one
  // term (sigma/n) 1-hat (1-hat^T p) of the operator are applied by the residual update;
  // the finishing dispatch first reduces the p-update's partial sums of p (fold_nblk
  // workgroups) into st->sump, and folds delta ||st->t1(0:fold_c)||^2 and
  // fold_sig_over_n * sump^2 into p^T q.
  int32_t fold_c;
  int32_t fold_nblk;
  const double* fold_partials;
  double fold_sig_over_n;
};

// ---- launchers (kernels.hip) ----
void launch_degree(const int32_t* rp, const void* w, int wdt, int n, double* d, float* d32,
                   hipStream_t s);
void launch_argmax_degree(const double* d, const int32_t* perm, int n, DevState* st,
                          RedBuf rb, double* out3, hipStream_t s);

template <typename T>
void launch_spmv(const SpmvPlan& plan, int valmode, const SpmvArgs<T>& a, RedBuf rb,
                 hipStream_t s);
// the same product under a separate kernel symbol, for bandwidth measurement (red = 0)
template <typename T>
void launch_spmv_probe(const SpmvPlan& plan, int valmode, const SpmvArgs<T>& a, double* partials,
                       hipStream_t s);

template <typename T>
void launch_pcg_update1(int n, T* x, T* r, const T* p, const T* q, const T* dinv, const T* V,
                        int64_t ldv, int c, const double* Ginv, double delta, int trim,
                        double sig_over_n, int init, DevState* st, RedBuf rb, hipStream_t s);
template <typename T>
void launch_pcg_update2(int n, const T* r, T* p, const T* dinv, const T* V, int64_t ldv,
                        int c, double delta, int init, DevState* st, RedBuf rb, hipStream_t s);
// learned preconditioner variants: update1 without the Jacobi dots; apply y = M r with
// the SMW dots; update2 with z = y - delta Y g.
// preconditioned MINRES for the indefinite inner systems of a moving shift
template <typename T>
void launch_minres_a(int n, const T* q, const T* vcur, T* vprev, const T* dinv, const T* V,
                     int64_t ldv, int c, const double* Ginv, double delta, int trim,
                     double sig_over_n, int init, DevState* st, RedBuf rb, hipStream_t s);
template <typename T>
void launch_minres_b(int n, T* z, T* wprev, T* wcur, T* x, const T* v, T* vzero, const T* dinv,
                     const T* V, int64_t ldv, int c, double delta, int init, int jit,
                     DevState* st, RedBuf rb, hipStream_t s);
// with_fin = false leaves the convergence test to the dispatch that follows (pruned M)
template <typename T>
void launch_pcg_update1_plain(int n, T* x, T* r, const T* p, const T* q, const T* V,
                              int64_t ldv, int c, double delta, int trim, double sig_over_n,
                              int init, DevState* st, RedBuf rb, hipStream_t s,
                              bool with_fin = true);
// Pruned learned M (diagonal mdiag plus the kept off-diagonal CSR prp/pcol/pval):
// u = M r with the partials ||r||^2, r^T u, V-hat^T u, then k_pcg_fin1 (eq. (3.5)).  Rows
// with more than kSpLongRow kept entries (listed in plong, n_long of them) are summed first,
// one wave per row; the thread-per-row pass reads their u.
constexpr int kSpLongRow = 32;
template <typename T>
void launch_spai_sparse_step(int n, const T* r, T* u, const int32_t* prp, const int32_t* pcol,
                             const float* pval, const T* mdiag, const int32_t* plong, int n_long,
                             const T* V, int64_t ldv, int c, const double* Ginv, double delta,
                             int init, DevState* st, RedBuf rb, hipStream_t s);
// y = M x for the pruned M; returns at once when skip_if_done is set and done.
template <typename T>
void launch_spai_sparse_mv(int n, const T* x, T* y, const int32_t* prp, const int32_t* pcol,
                           const float* pval, const T* mdiag, const int32_t* plong, int n_long,
                           const DevState* skip_if_done, hipStream_t s);
template <typename T>
void launch_pcg_update2_learned(int n, const T* y, T* p, const T* Y, int64_t ldv, int c,
                                const T* V, double delta, int init, DevState* st, RedBuf rb,
                                hipStream_t s);
void launch_spai_finish_rho(int c, const double* Ginv, double delta, int init, DevState* st,
                            hipStream_t s);

template <typename T>
void launch_rhs_prep(int n, const double* r64, double mean, const double* mean_sum,
                     double inv_n, int trim, T* rin, T* x, hipStream_t s);
template <typename T>
void launch_enlarge(int n, const T* x, double* z, DevState* st, RedBuf rb, hipStream_t s);

// Column dots h_j = sum_l A[l,j] * (w_l * z_l), j < na, then B, then (optional) sum z,
// then (optional) z^T z.  Result into h (device).  skip: both dispatches return at once
// when *skip is nonzero on the device (inside an inner solve: &st->done).
template <typename T>
void launch_multidot(int n, const T* A, int64_t lda, int na, const T* B, int64_t ldb, int nb,
                     const T* z, const T* wz, int with_sum, int with_self, double* h,
                     RedBuf rb, hipStream_t s, const int32_t* skip = nullptr);
// z -= A hA + B hB + (with_sum ? h_sum/n : 0); optional ||z||^2 into st->red[2].  skip as
// for launch_multidot.
void launch_gemv_sub(int n, const double* A, int64_t lda, int na, const double* B,
                     int64_t ldb, int nb, const double* h, int with_sum, double* z,
                     int with_norm, DevState* st, RedBuf rb, hipStream_t s,
                     const int32_t* skip = nullptr);
// Second-pass test of Gram-Schmidt (Daniel, Gragg, Kaufman and Stewart, 1976): with
// ||z||^2 before the first pass in h0sq (device) and after it in st->red[2], sets
// st->cgs_skip = 1 when ||z_after|| >= ||z_before|| / sqrt(2), i.e. when the first pass
// removed too little for cancellation to have spoiled orthogonality, else 0.
void launch_dgks_decide(const double* h0sq, DevState* st, hipStream_t s);
void launch_scale(int n, const double* z, double scale, double* u, hipStream_t s);
void launch_scale_dev(int n, const double* z, const double* nrm2, double* u, hipStream_t s);
void launch_pcg_reset(DevState* st, double rtol2, int maxit, hipStream_t s);
void launch_ritz_residual(int n, const double* U, const double* W, int64_t ld, int k,
                          const double* svec, double theta, double* r, DevState* st, RedBuf rb,
                          hipStream_t s);
void launch_ritz_vector(int n, const double* U, int64_t ld, int k, const double* svec,
                        double* y, hipStream_t s);
void launch_tsgemm_inplace(int n, double* U, int64_t ld, int k, const double* S, int q,
                           hipStream_t s);
template <typename T>
void launch_masked_copy(int n, const double* src, int trim, T* dst, hipStream_t s);
template <typename T>
void launch_dinv(int n, const double* d, double sigma, int trim, T* dinv, hipStream_t s);
template <typename Ts, typename Td>
void launch_gather(int n, const Ts* src, const int32_t* idx, Td* dst, hipStream_t s);
void launch_fill_replacement(int n, uint64_t seed, uint64_t draw, const int32_t* perm,
                             double* out, hipStream_t s);
// out[label] = sign * v[iperm[label]], sign making the largest-magnitude entry positive
// (lowest caller label among ties); scal4: device scratch of 4 doubles.
void launch_signed_gather(int n, const double* v, const int32_t* perm, const int32_t* iperm,
                          double* out, double* scal4, RedBuf rb, hipStream_t s);
int set_error(int code, const char* msg);

}  // namespace isira
