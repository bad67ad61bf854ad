// Learned sparse approximate inverse (SPAI) preconditioner: device buffers, the
// preconditioner apply used by the inner PCG, and the network kernels.
#pragma once
#include "internal.h"

namespace isira {
namespace spai {

struct SpaiWork {
  DevMem* mem = nullptr;     // the context's device memory (set at context creation)
  int64_t n = 0, nnz = 0;
  float* diag32 = nullptr;   // M_ii (internal order)
  double* diag64 = nullptr;  // M_ii in FP64 for the FP64 inner solve
  float* offd = nullptr;     // m_ij on the relabelled CSR pattern
  // network buffers (allocated on first use)
  float* feat = nullptr;     // n x F
  float* t1 = nullptr;       // n x H  first hidden layer of the vertex MLP
  float* h = nullptr;        // n x H  vertex embedding
  float* agg = nullptr;      // n x H  neighbour mean of h
  float* sdiag = nullptr;    // n      diagonal head pre-activation
  int32_t* rowidx = nullptr; // nnz    row of each stored entry
  float* nm_part = nullptr;  // neighbour mean: H sums per piece of a long row
  float* scratch = nullptr;  // training scratch
  size_t scratch_elems = 0;
  double* gpart = nullptr;   // gradient partials
  size_t gpart_elems = 0;
  // pruned form (isira_spai_prune): the kept off-diagonal entries of M as CSR in internal
  // order; while set, every apply of M uses it (the dropped entries of offd are 0 as well)
  bool pruned = false;
  int64_t pnnz = 0;
  int32_t* prp = nullptr;   // n + 1
  int32_t* pcol = nullptr;  // pnnz
  float* pval = nullptr;    // pnnz
  int32_t* plong = nullptr; // rows with more than kSpLongRow kept entries (one wave each)
  int64_t n_long = 0;
};

void free_work(SpaiWork& w);
void free_pruned(SpaiWork& w);

// y = M x with the trimmed row zeroed (x carries 0 at `trim`), followed by the dots
// st->t2[0..c) = V-hat^T y and st->t2[c] = x^T y used by eq. (3.5) in the PCG.
template <typename T>
void apply(SpaiWork& w, const SpmvPlan& plan, const int32_t* rp, const int32_t* col,
           const T* x, T* y, int n, int trim, const T* V, int64_t ldv, int c, DevState* st,
           RedBuf rb, hipStream_t s);
// y = M x only.
template <typename T>
void apply_plain(SpaiWork& w, const SpmvPlan& plan, const int32_t* rp, const int32_t* col,
                 const T* x, T* y, int n, int trim, hipStream_t s);
// Pruned M only (w.pruned): u = M r with the partials of one PCG step, finished by the
// Jacobi path's dispatch (see launch_spai_sparse_step).
template <typename T>
void sparse_step(const SpaiWork& w, int n, const T* r, T* u, const T* V, int64_t ldv, int c,
                 const double* Ginv, double delta, int init, DevState* st, RedBuf rb,
                 hipStream_t s);

int32_t nparam();
int ensure(SpaiWork& w, int64_t n, int64_t nnz);
size_t work_bytes(int64_t n, int64_t nnz);  // device bytes ensure() allocates
// Network forward: fills diag32 / diag64 / offd (internal order) for (sigma, trim).
int forward(SpaiWork& w, const int32_t* rp, const int32_t* col, const void* wts, int wdt,
            const double* deg, int n, int64_t nnz, double sigma, int trim, const float* params,
            hipStream_t s);
// Loss over S samples (caller-ordered r, z, sample-major) and its gradient (FP32, nparam).
int loss_grad(SpaiWork& w, const int32_t* rp, const int32_t* col, const void* wts, int wdt,
              const double* deg, int n, int64_t nnz, double sigma, int trim, const float* params,
              const int32_t* perm, const float* r, const float* z, int S, float* grad,
              double* loss_host, RedBuf rb, hipStream_t s);
void adam(float* p, const float* g, float* m, float* v, int count, float lr, float b1, float b2,
          float eps, int step, hipStream_t s);
void scatter_offd(int64_t nnz, const float* src, const int32_t* map, float* dst, hipStream_t s);

}  // namespace spai
}  // namespace isira
