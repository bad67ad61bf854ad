// Preconditioner apply of the learned sparse approximate inverse M (values on the pattern
// of L-hat plus its diagonal), reusing the binned SpMV of the Laplacian.
#include "spai.h"

namespace isira {
namespace spai {

void free_work(SpaiWork& w) {
  if (!w.mem) return;  // nothing was ever allocated
  for (float** p : {&w.diag32, &w.offd, &w.feat, &w.t1, &w.h, &w.agg, &w.sdiag, &w.scratch, &w.nm_part})
    dfree(*w.mem, *p);
  dfree(*w.mem, w.diag64);
  dfree(*w.mem, w.rowidx);
  dfree(*w.mem, w.gpart);
  w.scratch_elems = w.gpart_elems = 0;
  free_pruned(w);
}

void free_pruned(SpaiWork& w) {
  if (w.mem) {
    dfree(*w.mem, w.prp);
    dfree(*w.mem, w.pcol);
    dfree(*w.mem, w.pval);
    dfree(*w.mem, w.plong);
  }
  w.n_long = 0;
  w.pruned = false;
  w.pnnz = 0;
}

template <typename T>
static SpmvArgs<T> m_args(SpaiWork& w, const int32_t* rp, const int32_t* col, const T* x, T* y,
                          int n, int trim) {
  SpmvArgs<T> a{};
  a.rp = rp;
  a.col = col;
  a.vals = w.offd;
  a.x = x;
  a.y = y;
  if constexpr (sizeof(T) == 8) {
    a.diag = w.diag64;
  } else {
    a.diag = w.diag32;
  }
  a.n = n;
  a.trim = trim;
  return a;
}

template <typename T>
static const T* mdiag(const SpaiWork& w) {
  if constexpr (sizeof(T) == 8) {
    return w.diag64;
  } else {
    return w.diag32;
  }
}

template <typename T>
void apply(SpaiWork& w, const SpmvPlan& plan, const int32_t* rp, const int32_t* col,
           const T* x, T* y, int n, int trim, const T* V, int64_t ldv, int c, DevState* st,
           RedBuf rb, hipStream_t s) {
  if (w.pruned) {
    launch_spai_sparse_mv<T>(n, x, y, w.prp, w.pcol, w.pval, mdiag<T>(w), w.plong, (int)w.n_long, st, s);
  } else {
    SpmvArgs<T> a = m_args<T>(w, rp, col, x, y, n, trim);
    a.st = st;
    a.check_done = 1;
    launch_spmv<T>(plan, kF32Pos, a, rb, s);
  }
  // [V-hat^T y, x^T y] -> st->t2[0..c]
  launch_multidot<T>(n, V, ldv, c, x, ldv, 1, y, nullptr, 0, 0, st->t2, rb, s, &st->done);
}

template <typename T>
void apply_plain(SpaiWork& w, const SpmvPlan& plan, const int32_t* rp, const int32_t* col,
                 const T* x, T* y, int n, int trim, hipStream_t s) {
  if (w.pruned) {
    launch_spai_sparse_mv<T>(n, x, y, w.prp, w.pcol, w.pval, mdiag<T>(w), w.plong, (int)w.n_long, nullptr, s);
    return;
  }
  SpmvArgs<T> a = m_args<T>(w, rp, col, x, y, n, trim);
  RedBuf none{nullptr, nullptr};
  launch_spmv<T>(plan, kF32Pos, a, none, s);
}

template <typename T>
void sparse_step(const SpaiWork& w, int n, const T* r, T* u, const T* V, int64_t ldv, int c,
                 const double* Ginv, double delta, int init, DevState* st, RedBuf rb,
                 hipStream_t s) {
  launch_spai_sparse_step<T>(n, r, u, w.prp, w.pcol, w.pval, mdiag<T>(w), w.plong, (int)w.n_long, V,
                             ldv, c, Ginv, delta, init, st, rb, s);
}
template void sparse_step<double>(const SpaiWork&, int, const double*, double*, const double*,
                                  int64_t, int, const double*, double, int, DevState*, RedBuf,
                                  hipStream_t);
template void sparse_step<float>(const SpaiWork&, int, const float*, float*, const float*,
                                 int64_t, int, const double*, double, int, DevState*, RedBuf,
                                 hipStream_t);

template void apply<double>(SpaiWork&, const SpmvPlan&, const int32_t*, const int32_t*,
                            const double*, double*, int, int, const double*, int64_t, int,
                            DevState*, RedBuf, hipStream_t);
template void apply<float>(SpaiWork&, const SpmvPlan&, const int32_t*, const int32_t*,
                           const float*, float*, int, int, const float*, int64_t, int,
                           DevState*, RedBuf, hipStream_t);
template void apply_plain<double>(SpaiWork&, const SpmvPlan&, const int32_t*, const int32_t*,
                                  const double*, double*, int, int, hipStream_t);
template void apply_plain<float>(SpaiWork&, const SpmvPlan&, const int32_t*, const int32_t*,
                                 const float*, float*, int, int, hipStream_t);

}  // namespace spai
}  // namespace isira
