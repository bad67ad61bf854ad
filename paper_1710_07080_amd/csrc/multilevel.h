// Multilevel preconditioner of the inner systems: an unsmoothed-aggregation multigrid
// V-cycle for the trimmed Laplacian L-hat (the multilevel slot of Section 3; Remark 3.2
// combines it with eq. (3.5) for the deflation term).
#pragma once
#include <vector>

#include "internal.h"

namespace isira {
namespace ml {

// One level l that has a coarser level l+1.  The cycle at this level, one damped Jacobi
// sweep (S = W D^-1) before and after the coarse correction from x = 0, is applied as two
// sparse products over precomputed matrices:
//   down: b_{l+1} = Q^T b_l,              Q = (I - S A_l) P_l   (n_{l+1} rows)
//   up:   x_l = M b_l + Q x_{l+1},        M = 2S - S A_l S      (n_l rows)
// The level buffer holds b_l at [0, n) and x_{l+1} at [ld, ld + nc), so the up product
// is one product of [M | Q] with the buffer (columns of Q shifted by ld).
struct Level {
  int n = 0, ld = 0, nc = 0;
  SpmvPlan down, up;
  int32_t *down_rp = nullptr, *down_col = nullptr, *up_rp = nullptr, *up_col = nullptr;
  double *down_v64 = nullptr, *up_v64 = nullptr, *up_diag64 = nullptr;
  float *down_v32 = nullptr, *up_v32 = nullptr, *up_diag32 = nullptr;
  double* buf64 = nullptr;
  float* buf32 = nullptr;
};

struct Hierarchy {
  DevMem* mem = nullptr;  // the context's device memory (set at context creation)
  bool ready = false;
  int trim = -1;  // internal index of the trimmed vertex
  double omega = 0.0;
  int coarse_max = 0;
  std::vector<Level> lv;
  // coarsest level: dense inverse over its vertices with neighbours, 1/diag elsewhere
  int nL = 0, mL = 0;
  int32_t* cidx = nullptr;   // mL rows of the dense part
  int32_t* cpos = nullptr;   // nL: position in the dense part, or -1
  double* Ainv = nullptr;    // mL x mL, row-major
  double* cdinv = nullptr;   // nL: 1/diag outside the dense part, 0 for the trimmed row
  double* bufL64 = nullptr;  // nL
  float* bufL32 = nullptr;
  double* zero64 = nullptr;  // zero diagonal of the down products
  float* zero32 = nullptr;
  // statistics
  std::vector<int64_t> rows, offnnz, connected;
  int64_t stored_nnz = 0, device_bytes = 0;
  double setup_ms = 0.0;
};

struct Params {
  double omega;
  int coarse_max;
  int max_levels;
};

// Builds the hierarchy on the host from the relabelled graph (host CSR rp/col of n rows,
// weights w or NULL for unit weights, perm[internal] = caller label, which breaks ties of
// the aggregation order) with vertex `trim` (internal) deleted, and uploads it.
int setup(Hierarchy& H, int n, const int32_t* rp, const int32_t* col, const double* w,
          const int32_t* perm, int trim, const Params& prm);
void release(Hierarchy& H);

// out = cycle(in) on internal vectors of length n (in's trimmed entry is ignored, out's is
// 0).  check_done: every launch returns at once when st->done is set (inside PCG).
// in_place: `in` serves as the finest level's buffer, so it must have room for the second
// level's vector at [lv[0].ld, lv[0].ld + lv[0].nc), which the cycle overwrites; otherwise
// `in` is copied into the level's own buffer first.
template <typename T>
void apply(const Hierarchy& H, const T* in, T* out, int check_done, DevState* st, RedBuf rb,
           hipStream_t s, bool in_place = false);

}  // namespace ml
}  // namespace isira
