// Multilevel preconditioner: host-side hierarchy set-up (aggregation, Galerkin coarse
// matrices, the composite transfer matrices of the V-cycle, the coarsest-level inverse)
// and the device-side cycle.
//
// Definition of the cycle (the multilevel slot of Section 3, with Remark 3.2):
//   A_0 = L-hat (vertex `trim` deleted), A_{l+1} = P_l^T A_l P_l, P_l the 0/1 aggregation
//   matrix.  Aggregation of a level, on the graph of A_l's off-diagonal pattern: a vertex
//   without neighbours belongs to no aggregate; the others are visited by decreasing
//   number of neighbours (ties: caller label on level 0, index on coarser levels); phase 1:
//   a visited vertex that is unassigned and whose neighbours are all unassigned forms a new
//   aggregate with them (ids in order of creation); phase 2: each vertex left joins, among
//   the phase-1 aggregates holding a neighbour, the one holding the most, ties by the
//   smallest id.  No floating-point value enters the rule.  A level with at most coarse_max
//   vertices that have neighbours is the coarsest and is solved exactly.  Smoothing: one
//   damped Jacobi sweep with S = W D^-1 (w_v = omega, or 1 for a vertex without neighbours)
//   before and after the coarse correction, from x = 0.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <string>
#include <thread>
#include <vector>

#include "guard.h"
#include "multilevel.h"

namespace isira {
namespace ml {
namespace {

int err(int code, const std::string& m) { return set_error(code, m.c_str()); }

#define MLCK(expr)                                                                   \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return err(ISIRA_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

template <typename T>
int dal(DevMem& m, T** p, size_t count, int64_t& bytes) {
  const int rc = dalloc(m, p, count);
  if (rc == ISIRA_OK) bytes += (int64_t)dev_round((count == 0 ? 1 : count) * sizeof(T));
  return rc;
}

template <typename T>
int put(T* d, const std::vector<T>& h) {
  if (!h.empty()) MLCK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return ISIRA_OK;
}

template <typename T>
void dfr(DevMem& m, T*& p) {
  dfree(m, p);
}

// Host threads for the set-up: up to 16, one for small inputs.
int setup_threads(int64_t items) {
  unsigned hc = std::thread::hardware_concurrency();
  return items < 65536 ? 1 : (hc == 0 ? 1 : (hc > 16 ? 16 : (int)hc));
}

// f(t, begin, end) over nt contiguous ranges of [0, n), one thread each (a range whose
// thread cannot be started runs on the calling thread).  An exception in any range is
// rethrown here after every thread has joined.
template <typename F>
void run_ranges(int n, int nt, F f) {
  const int chunk = (n + nt - 1) / nt;
  if (nt == 1) {
    f(0, 0, n);
    return;
  }
  std::vector<std::exception_ptr> ex(nt);
  std::vector<std::thread> th;
  th.reserve(nt);
  for (int t = 0; t < nt; ++t) {
    auto job = [&, t] {
      try {
        f(t, t * chunk, std::min(n, t * chunk + chunk));
      } catch (...) {
        ex[t] = std::current_exception();
      }
    };
    try {
      th.emplace_back(job);
    } catch (...) {
      job();
    }
  }
  for (auto& x : th) x.join();
  for (auto& e : ex)
    if (e) std::rethrow_exception(e);
}

// f(begin, end) over chunks of [0, n) (64 per thread), which the threads take in turn.
template <typename F>
void for_chunks(int n, int nt, F f) {
  const int nchunk = nt == 1 ? 1 : std::min(n, 64 * nt);
  const int csize = nchunk ? (n + nchunk - 1) / nchunk : 0;
  std::atomic<int> next(0);
  run_ranges(nt, nt, [&](int, int, int) {
    for (int c = next++; c < nchunk; c = next++) f(c * csize, std::min(n, c * csize + csize));
  });
}

// Rows [0, nrows) of a CSR matrix built by up to 16 host threads.  The rows are cut into
// chunks of consecutive rows (many more than threads, since a few rows near the hubs carry
// much of the work); threads take chunks in turn from a shared counter and emit each
// chunk's rows into the chunk's own buffers through emit(row, cols, vals), a worker made
// per thread by make() that holds the thread's scratch.  The chunks are then concatenated in
// order.  Each row depends only on its own inputs, so the result is the serial build's, bit
// for bit.
template <typename V, typename Make>
void build_rows(int nrows, std::vector<int32_t>& rp, std::vector<int32_t>& col,
                std::vector<V>& val, Make make) {
  const int nt = setup_threads(nrows);
  const int nchunk = nt == 1 ? 1 : std::min(nrows, 64 * nt);
  const int csize = (nrows + nchunk - 1) / nchunk;
  std::vector<std::vector<int32_t>> cs(nchunk);
  std::vector<std::vector<V>> vs(nchunk);
  rp.assign((size_t)nrows + 1, 0);
  std::atomic<int> next(0);
  run_ranges(nt, nt, [&](int, int, int) {
    auto emit = make();
    for (int c = next++; c < nchunk; c = next++) {
      const int b = c * csize, e = std::min(nrows, b + csize);
      for (int r = b; r < e; ++r) {
        emit(r, cs[c], vs[c]);
        rp[r + 1] = (int32_t)cs[c].size();  // offset within the chunk; made global below
      }
    }
  });
  std::vector<size_t> base(nchunk + 1, 0);
  for (int c = 0; c < nchunk; ++c) base[c + 1] = base[c] + cs[c].size();
  col.resize(base[nchunk]);
  val.resize(base[nchunk]);
  std::atomic<int> next2(0);
  run_ranges(nt, nt, [&](int, int, int) {
    for (int c = next2++; c < nchunk; c = next2++) {
      std::copy(cs[c].begin(), cs[c].end(), col.begin() + base[c]);
      std::copy(vs[c].begin(), vs[c].end(), val.begin() + base[c]);
      const int b = c * csize, e = std::min(nrows, b + csize);
      for (int r = b; r < e; ++r) rp[r + 1] += (int32_t)base[c];
      std::vector<int32_t>().swap(cs[c]);
      std::vector<V>().swap(vs[c]);
    }
  });
}

// Accumulates a row's entries by column; flush() appends them in increasing column order.
template <typename V>
struct RowAccumulator {
  std::vector<int32_t> pos, touched;
  std::vector<V> acc;
  explicit RowAccumulator(int ncols) : pos(ncols, -1) {}
  void add(int b, V v) {
    if (pos[b] < 0) {
      pos[b] = (int)touched.size();
      touched.push_back(b);
      acc.push_back(V(0));
    }
    acc[pos[b]] += v;
  }
  void flush(std::vector<int32_t>& col, std::vector<V>& val) {
    std::vector<int32_t> idx(touched.size());
    for (size_t t = 0; t < idx.size(); ++t) idx[t] = (int32_t)t;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return touched[x] < touched[y]; });
    for (int t : idx) {
      col.push_back(touched[t]);
      val.push_back(acc[t]);
    }
    for (int b : touched) pos[b] = -1;
    touched.clear();
    acc.clear();
  }
};

// One level on the host: A_ij = -w for the stored off-diagonal entries, A_ii = diag.
struct HostLevel {
  int n = 0;
  std::vector<int32_t> rp, col;
  std::vector<double> w, diag;
  std::vector<uint8_t> active;  // 0 only for the trimmed vertex of level 0
  int rowlen(int i) const { return rp[i + 1] - rp[i]; }
};

// Aggregate ids (creation order) of the vertices of A; -1 for a vertex without
// neighbours.  by_key lists the vertices in increasing tie-break key.  Returns the count.
int aggregate(const HostLevel& A, const std::vector<int32_t>& by_key, std::vector<int32_t>& agg) {
  const int n = A.n;
  int maxlen = 0;
  for (int i = 0; i < n; ++i) maxlen = std::max(maxlen, A.rowlen(i));
  // visiting order: decreasing row length, ties by key (stable counting sort of by_key)
  std::vector<int32_t> start((size_t)maxlen + 2, 0), order;
  order.reserve(n);
  for (int v : by_key)
    if (A.rowlen(v) > 0) start[maxlen - A.rowlen(v) + 1]++;
  for (int b = 1; b <= maxlen + 1; ++b) start[b] += start[b - 1];
  order.assign(start[maxlen + 1], 0);
  for (int v : by_key) {
    const int l = A.rowlen(v);
    if (l > 0) order[start[maxlen - l]++] = v;
  }
  agg.assign(n, -1);
  int nagg = 0;
  for (int v : order) {  // phase 1
    if (agg[v] >= 0) continue;
    bool free_nb = true;
    for (int e = A.rp[v]; e < A.rp[v + 1] && free_nb; ++e) free_nb = agg[A.col[e]] < 0;
    if (!free_nb) continue;
    agg[v] = nagg;
    for (int e = A.rp[v]; e < A.rp[v + 1]; ++e) agg[A.col[e]] = nagg;
    ++nagg;
  }
  std::vector<int32_t> phase1 = agg, ids;
  for (int v = 0; v < n; ++v) {  // phase 2
    if (phase1[v] >= 0 || A.rowlen(v) == 0) continue;
    ids.clear();
    for (int e = A.rp[v]; e < A.rp[v + 1]; ++e)
      if (phase1[A.col[e]] >= 0) ids.push_back(phase1[A.col[e]]);
    std::sort(ids.begin(), ids.end());
    int best = -1, best_cnt = 0;
    for (size_t a = 0; a < ids.size();) {
      size_t b = a;
      while (b < ids.size() && ids[b] == ids[a]) ++b;
      if ((int)(b - a) > best_cnt) {  // ascending ids: the first maximum is the smallest id
        best_cnt = (int)(b - a);
        best = ids[a];
      }
      a = b;
    }
    agg[v] = best;  // >= 0: a vertex skipped in phase 1 has a phase-1 neighbour
  }
  return nagg;
}

// Galerkin coarse level P^T A P for the aggregation agg (nc aggregates).
HostLevel coarsen(const HostLevel& A, const std::vector<int32_t>& agg, int nc) {
  HostLevel C;
  C.n = nc;
  std::vector<int32_t> mptr((size_t)nc + 1, 0), mem;
  for (int i = 0; i < A.n; ++i)
    if (agg[i] >= 0) mptr[agg[i] + 1]++;
  for (int a = 0; a < nc; ++a) mptr[a + 1] += mptr[a];
  mem.assign(mptr[nc], 0);
  {
    std::vector<int32_t> fill(mptr.begin(), mptr.end() - 1);
    for (int i = 0; i < A.n; ++i)
      if (agg[i] >= 0) mem[fill[agg[i]]++] = i;
  }
  C.diag.assign(nc, 0.0);
  C.active.assign(nc, 1);
  build_rows<double>(nc, C.rp, C.col, C.w, [&] {
    return [&, ra = RowAccumulator<double>(nc)](int a, std::vector<int32_t>& col,
                                                std::vector<double>& val) mutable {
      double dg = 0.0;
      for (int k = mptr[a]; k < mptr[a + 1]; ++k) {
        const int i = mem[k];
        dg += A.diag[i];
        for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) {
          const int b = agg[A.col[e]];
          if (b == a)
            dg -= A.w[e];
          else
            ra.add(b, A.w[e]);
        }
      }
      C.diag[a] = dg;
      ra.flush(col, val);
    };
  });
  return C;
}

// In-place inverse of an SPD row-major m x m matrix by Cholesky (A = L L^T, X = L^-1,
// A^-1 = X^T X).  Returns false when a pivot is not positive.
bool spd_inverse_rowmajor(int m, std::vector<double>& A) {
  std::vector<double> L((size_t)m * m, 0.0), X((size_t)m * m, 0.0);
  for (int j = 0; j < m; ++j) {
    double s = A[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) s -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    L[(size_t)j * m + j] = ljj;
    for (int i = j + 1; i < m; ++i) {
      double v = A[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
      L[(size_t)i * m + j] = v / ljj;
    }
  }
  // X = L^-1 (lower), row by row: X[i][j] = -(sum_{k=j}^{i-1} L[i][k] X[k][j]) / L[i][i]
  for (int i = 0; i < m; ++i) {
    X[(size_t)i * m + i] = 1.0 / L[(size_t)i * m + i];
    for (int j = 0; j < i; ++j) {
      double v = 0.0;
      for (int k = j; k < i; ++k) v += L[(size_t)i * m + k] * X[(size_t)k * m + j];
      X[(size_t)i * m + j] = -v / L[(size_t)i * m + i];
    }
  }
  for (int i = 0; i < m; ++i)
    for (int j = 0; j <= i; ++j) {
      double v = 0.0;
      for (int k = i; k < m; ++k) v += X[(size_t)k * m + i] * X[(size_t)k * m + j];
      A[(size_t)i * m + j] = A[(size_t)j * m + i] = v;
    }
  return true;
}

template <typename T>
__global__ __launch_bounds__(256) void k_ml_coarse(int nL, int mL, const int32_t* __restrict__ cidx,
                                                   const int32_t* __restrict__ cpos,
                                                   const double* __restrict__ Ainv,
                                                   const double* __restrict__ cdinv,
                                                   const T* __restrict__ b, T* __restrict__ out,
                                                   const DevState* st, int check_done) {
  if (check_done && st->done) return;
  // one wave per row; row and its dense position are uniform within the wave
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= nL) return;
  const int p = cpos[row];
  if (p < 0) {
    if (lane == 0) out[row] = (T)(cdinv[row] * (double)b[row]);
    return;
  }
  const double* __restrict__ a = Ainv + (size_t)p * mL;
  double s = 0.0;
  for (int l = lane; l < mL; l += 64) s += a[l] * (double)b[cidx[l]];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) out[row] = (T)s;
}

// The two transfer products of one level on the host (see Level).
struct HostMats {
  int ld = 0;
  std::vector<int32_t> drp, dcol, urp, ucol;
  std::vector<double> dval, uval, udiag;
};

HostMats build_level_mats(const HostLevel& A, const std::vector<int32_t>& agg, int nc,
                          double omega) {
  const int n = A.n;
  HostMats M;
  M.ld = (n + 63) / 64 * 64;
  // smoother weights s_i = w_i / A_ii
  std::vector<double> s(n, 0.0);
  for (int i = 0; i < n; ++i)
    if (A.active[i]) s[i] = (A.rowlen(i) > 0 ? omega : 1.0) / A.diag[i];
  // Q = (I - S A) P: row i, column b: [agg_i == b] (1 - s_i A_ii) + s_i sum_{j in b} w_ij
  std::vector<int32_t> qrp, qcol;
  std::vector<double> qval;
  build_rows<double>(n, qrp, qcol, qval, [&] {
    return [&, ra = RowAccumulator<double>(nc)](int i, std::vector<int32_t>& col,
                                                std::vector<double>& val) mutable {
      if (agg[i] < 0) return;
      ra.add(agg[i], 1.0 - s[i] * A.diag[i]);
      for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) ra.add(agg[A.col[e]], s[i] * A.w[e]);
      ra.flush(col, val);
    };
  });
  // up = [M | Q], M = 2S - S A S: off-diagonal s_i w_ij s_j, diagonal 2 s_i - s_i^2 A_ii;
  // row i holds A's row, then Q's row, so its offset is known and the rows fill in parallel
  M.urp.assign((size_t)n + 1, 0);
  M.udiag.assign(n, 0.0);
  for (int i = 0; i < n; ++i) M.urp[i + 1] = A.rp[i + 1] + qrp[i + 1];
  M.ucol.resize(M.urp[n]);
  M.uval.resize(M.urp[n]);
  for_chunks(n, setup_threads(n), [&](int b, int e) {
    for (int i = b; i < e; ++i) {
      int o = M.urp[i];
      for (int k = A.rp[i]; k < A.rp[i + 1]; ++k, ++o) {
        M.ucol[o] = A.col[k];
        M.uval[o] = s[i] * A.w[k] * s[A.col[k]];
      }
      for (int k = qrp[i]; k < qrp[i + 1]; ++k, ++o) {
        M.ucol[o] = M.ld + qcol[k];
        M.uval[o] = qval[k];
      }
      if (A.active[i]) M.udiag[i] = 2.0 * s[i] - s[i] * s[i] * A.diag[i];
    }
  });
  // down = Q^T (rows = aggregates, columns increasing): each thread counts the entries of
  // its range of Q's rows per aggregate, so that it writes its part of every row of Q^T
  // after the earlier ranges' parts, in increasing order of Q's rows
  const int nt = setup_threads(n);
  std::vector<std::vector<int32_t>> cnt(nt, std::vector<int32_t>(nc, 0));
  run_ranges(n, nt, [&](int t, int b, int e) {
    for (int k = qrp[b]; k < qrp[e]; ++k) cnt[t][qcol[k]]++;
  });
  M.drp.assign((size_t)nc + 1, 0);
  for (int a = 0; a < nc; ++a) {
    int off = M.drp[a];
    for (int t = 0; t < nt; ++t) {
      const int c = cnt[t][a];
      cnt[t][a] = off;  // thread t's first slot in row a
      off += c;
    }
    M.drp[a + 1] = off;
  }
  M.dcol.assign(qcol.size(), 0);
  M.dval.assign(qcol.size(), 0.0);
  run_ranges(n, nt, [&](int t, int b, int e) {
    std::vector<int32_t>& fill = cnt[t];
    for (int i = b; i < e; ++i)
      for (int k = qrp[i]; k < qrp[i + 1]; ++k) {
        const int slot = fill[qcol[k]]++;
        M.dcol[slot] = i;
        M.dval[slot] = qval[k];
      }
  });
  return M;
}

// The coarsest level's exact solve on the host: dense inverse over its vertices with
// neighbours, 1/A_vv for the others (0 for an inactive vertex).
struct HostCoarsest {
  int n = 0, m = 0;
  std::vector<int32_t> cidx, cpos;
  std::vector<double> Ainv, cdinv;
};

int build_coarsest(const HostLevel& A, HostCoarsest& C) {
  const int n = A.n;
  C.n = n;
  C.cidx.clear();
  C.cpos.assign(n, -1);
  for (int i = 0; i < n; ++i)
    if (A.rowlen(i) > 0) {
      C.cpos[i] = (int32_t)C.cidx.size();
      C.cidx.push_back(i);
    }
  const int m = C.m = (int)C.cidx.size();
  C.Ainv.assign((size_t)m * m, 0.0);
  C.cdinv.assign(n, 0.0);
  for (int k = 0; k < m; ++k) {
    const int i = C.cidx[k];
    C.Ainv[(size_t)k * m + k] = A.diag[i];
    for (int e = A.rp[i]; e < A.rp[i + 1]; ++e) C.Ainv[(size_t)k * m + C.cpos[A.col[e]]] -= A.w[e];
  }
  for (int i = 0; i < n; ++i)
    if (A.active[i] && C.cpos[i] < 0) C.cdinv[i] = 1.0 / A.diag[i];
  if (m > 0 && !spd_inverse_rowmajor(m, C.Ainv))
    return err(ISIRA_E_PRECOND, "coarsest level of the multilevel hierarchy is not positive definite");
  return ISIRA_OK;
}

// All levels on the host: lev[0] = L-hat in internal indices (trimmed row empty and
// inactive), aggs[l] the aggregation of level l in device numbering of level l+1, mats[l]
// its transfer products.
int build_host(int n, const int32_t* rp, const int32_t* col, const double* w,
               const int32_t* perm, int trim, const Params& prm, std::vector<HostLevel>& lev,
               std::vector<std::vector<int32_t>>& aggs, std::vector<HostMats>& mats,
               HostCoarsest& co) {
  lev.assign(1, HostLevel{});
  aggs.clear();
  mats.clear();
  {
    HostLevel& A = lev[0];
    A.n = n;
    A.rp.assign((size_t)n + 1, 0);
    A.diag.assign(n, 0.0);
    A.active.assign(n, 1);
    A.active[trim] = 0;
    // row lengths without the trimmed vertex, then the rows in parallel
    const int nt = setup_threads(n);
    for_chunks(n, nt, [&](int b, int e) {
      for (int i = b; i < e; ++i) {
        int len = 0;
        if (i != trim)
          for (int k = rp[i]; k < rp[i + 1]; ++k) len += col[k] != trim;
        A.rp[i + 1] = len;
      }
    });
    for (int i = 0; i < n; ++i) A.rp[i + 1] += A.rp[i];
    A.col.resize(A.rp[n]);
    A.w.resize(A.rp[n]);
    for_chunks(n, nt, [&](int b, int e) {
      for (int i = b; i < e; ++i) {
        double d = 0.0;
        int o = A.rp[i];
        for (int k = rp[i]; k < rp[i + 1]; ++k) {
          const double we = w ? w[k] : 1.0;
          d += we;
          if (i != trim && col[k] != trim) {
            A.col[o] = col[k];
            A.w[o] = we;
            ++o;
          }
        }
        A.diag[i] = i == trim ? 0.0 : d;
      }
    });
  }
  std::vector<int32_t> by_key(n);
  for (int i = 0; i < n; ++i) by_key[perm[i]] = i;  // increasing caller label
  for (;;) {
    const HostLevel& A = lev.back();
    int conn = 0;
    for (int i = 0; i < A.n; ++i) conn += A.rowlen(i) > 0;
    if (conn <= prm.coarse_max) break;
    if ((int)lev.size() >= prm.max_levels)
      return err(ISIRA_E_PRECOND, "multilevel hierarchy: coarsest level still above coarse_max at max_levels");
    std::vector<int32_t> agg;
    const int nc = aggregate(A, by_key, agg);  // ids in creation order (the rule's ids)
    // device numbering of the coarse level: aggregates in the order of their first member
    // on this level, so that neighbouring rows of this level's products touch neighbouring
    // coarse entries; the rule's ids stay the tie-break keys of the next aggregation
    std::vector<int32_t> first(nc, A.n), dev(nc);
    for (int i = 0; i < A.n; ++i)
      if (agg[i] >= 0) first[agg[i]] = std::min(first[agg[i]], i);
    std::vector<int32_t> byfirst(nc);
    for (int a = 0; a < nc; ++a) byfirst[a] = a;
    std::sort(byfirst.begin(), byfirst.end(), [&](int x, int y) { return first[x] < first[y]; });
    for (int r = 0; r < nc; ++r) dev[byfirst[r]] = r;
    for (int i = 0; i < A.n; ++i)
      if (agg[i] >= 0) agg[i] = dev[agg[i]];
    HostLevel C = coarsen(A, agg, nc);
    mats.push_back(build_level_mats(A, agg, nc, prm.omega));
    aggs.push_back(std::move(agg));
    lev.push_back(std::move(C));
    by_key = dev;  // device index of the aggregate with rule id 0, 1, ...
  }
  return build_coarsest(lev.back(), co);
}

std::vector<float> to32(const std::vector<double>& v) {
  std::vector<float> f(v.size());
  for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
  return f;
}

int upload_level(Level& L, int n, int nc, const HostMats& M, Hierarchy& H) {
  L.n = n;
  L.nc = nc;
  L.ld = M.ld;
  int64_t& by = H.device_bytes;
  int rc;
  if ((rc = dal(*H.mem, &L.down_rp, M.drp.size(), by)) || (rc = dal(*H.mem, &L.down_col, M.dcol.size(), by)) ||
      (rc = dal(*H.mem, &L.down_v64, M.dval.size(), by)) || (rc = dal(*H.mem, &L.down_v32, M.dval.size(), by)) ||
      (rc = dal(*H.mem, &L.up_rp, M.urp.size(), by)) || (rc = dal(*H.mem, &L.up_col, M.ucol.size(), by)) ||
      (rc = dal(*H.mem, &L.up_v64, M.uval.size(), by)) || (rc = dal(*H.mem, &L.up_v32, M.uval.size(), by)) ||
      (rc = dal(*H.mem, &L.up_diag64, M.udiag.size(), by)) || (rc = dal(*H.mem, &L.up_diag32, M.udiag.size(), by)) ||
      (rc = dal(*H.mem, &L.buf64, (size_t)L.ld + nc, by)) || (rc = dal(*H.mem, &L.buf32, (size_t)L.ld + nc, by)))
    return rc;
  if ((rc = put(L.down_rp, M.drp)) || (rc = put(L.down_col, M.dcol)) || (rc = put(L.down_v64, M.dval)) ||
      (rc = put(L.down_v32, to32(M.dval))) || (rc = put(L.up_rp, M.urp)) || (rc = put(L.up_col, M.ucol)) ||
      (rc = put(L.up_v64, M.uval)) || (rc = put(L.up_v32, to32(M.uval))) ||
      (rc = put(L.up_diag64, M.udiag)) || (rc = put(L.up_diag32, to32(M.udiag))))
    return rc;
  // the level buffers are read in full by the products' own-row loads: keep them finite
  MLCK(hipMemset(L.buf64, 0, ((size_t)L.ld + nc) * sizeof(double)));
  MLCK(hipMemset(L.buf32, 0, ((size_t)L.ld + nc) * sizeof(float)));
  if ((rc = build_spmv_plan(*H.mem, nc, M.drp.data(), M.dcol.data(), L.down))) return rc;
  if ((rc = build_spmv_plan(*H.mem, n, M.urp.data(), M.ucol.data(), L.up))) return rc;
  H.stored_nnz += (int64_t)M.dcol.size() + (int64_t)M.ucol.size();
  return ISIRA_OK;
}

int upload_coarsest(const HostCoarsest& C, Hierarchy& H) {
  H.nL = C.n;
  H.mL = C.m;
  int64_t& by = H.device_bytes;
  int rc;
  if ((rc = dal(*H.mem, &H.cidx, C.cidx.size(), by)) || (rc = dal(*H.mem, &H.cpos, C.cpos.size(), by)) ||
      (rc = dal(*H.mem, &H.Ainv, C.Ainv.size(), by)) || (rc = dal(*H.mem, &H.cdinv, C.cdinv.size(), by)) ||
      (rc = dal(*H.mem, &H.bufL64, (size_t)C.n, by)) || (rc = dal(*H.mem, &H.bufL32, (size_t)C.n, by)))
    return rc;
  if ((rc = put(H.cidx, C.cidx)) || (rc = put(H.cpos, C.cpos)) || (rc = put(H.Ainv, C.Ainv)) ||
      (rc = put(H.cdinv, C.cdinv)))
    return rc;
  MLCK(hipMemset(H.bufL64, 0, (size_t)C.n * sizeof(double)));
  MLCK(hipMemset(H.bufL32, 0, (size_t)C.n * sizeof(float)));
  return ISIRA_OK;
}

}  // namespace

void release(Hierarchy& H) {
  if (!H.mem) return;  // nothing was ever allocated
  for (Level& L : H.lv) {
    free_spmv_plan(*H.mem, L.down);
    free_spmv_plan(*H.mem, L.up);
    dfr(*H.mem, L.down_rp); dfr(*H.mem, L.down_col); dfr(*H.mem, L.down_v64); dfr(*H.mem, L.down_v32);
    dfr(*H.mem, L.up_rp); dfr(*H.mem, L.up_col); dfr(*H.mem, L.up_v64); dfr(*H.mem, L.up_v32); dfr(*H.mem, L.up_diag64);
    dfr(*H.mem, L.up_diag32); dfr(*H.mem, L.buf64); dfr(*H.mem, L.buf32);
  }
  dfr(*H.mem, H.cidx); dfr(*H.mem, H.cpos); dfr(*H.mem, H.Ainv); dfr(*H.mem, H.cdinv); dfr(*H.mem, H.bufL64); dfr(*H.mem, H.bufL32);
  dfr(*H.mem, H.zero64); dfr(*H.mem, H.zero32);
  DevMem* mem = H.mem;
  H = Hierarchy{};
  H.mem = mem;
}

int setup(Hierarchy& H, int n, const int32_t* rp, const int32_t* col, const double* w,
          const int32_t* perm, int trim, const Params& prm) {
  release(H);
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<HostLevel> lev;
  std::vector<std::vector<int32_t>> aggs;
  std::vector<HostMats> mats;
  HostCoarsest co;
  int rc = build_host(n, rp, col, w, perm, trim, prm, lev, aggs, mats, co);
  if (rc) return rc;
  const int L = (int)lev.size() - 1;
  H.lv.resize(L);
  H.trim = trim;
  H.omega = prm.omega;
  H.coarse_max = prm.coarse_max;
  for (int l = 0; l < L; ++l)
    if ((rc = upload_level(H.lv[l], lev[l].n, lev[l + 1].n, mats[l], H))) {
      release(H);
      return rc;
    }
  if ((rc = upload_coarsest(co, H))) {
    release(H);
    return rc;
  }
  int maxc = 1;
  for (int l = 0; l < L; ++l) maxc = std::max(maxc, H.lv[l].nc);
  if ((rc = dal(*H.mem, &H.zero64, (size_t)maxc, H.device_bytes)) ||
      (rc = dal(*H.mem, &H.zero32, (size_t)maxc, H.device_bytes))) {
    release(H);
    return rc;
  }
  if (hipMemset(H.zero64, 0, (size_t)maxc * 8) != hipSuccess ||
      hipMemset(H.zero32, 0, (size_t)maxc * 4) != hipSuccess) {
    release(H);
    return err(ISIRA_E_HIP, "hipMemset failed");
  }
  for (int l = 0; l <= L; ++l) {
    const HostLevel& A = lev[l];
    int conn = 0;
    for (int i = 0; i < A.n; ++i) conn += A.rowlen(i) > 0;
    H.rows.push_back(l == 0 ? A.n - 1 : A.n);
    H.offnnz.push_back((int64_t)A.col.size());
    H.connected.push_back(conn);
  }
  H.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  H.ready = true;
  return ISIRA_OK;
}

template <typename T>
void apply(const Hierarchy& H, const T* in, T* out, int check_done, DevState* st, RedBuf rb,
           hipStream_t s, bool in_place) {
  constexpr bool f64 = sizeof(T) == 8;
  const int L = (int)H.lv.size();
  T* bL;
  if constexpr (f64) bL = H.bufL64; else bL = H.bufL32;
  // b0: the finest level's buffer (b_0, then x_1 at ld)
  T* b0;
  if (L == 0) {
    b0 = bL;
  } else if (in_place) {
    b0 = const_cast<T*>(in);
  } else {
    if constexpr (f64) b0 = H.lv[0].buf64; else b0 = H.lv[0].buf32;
  }
  if (b0 != in)
    (void)hipMemcpyAsync(b0, in, (size_t)(L ? H.lv[0].n : H.nL) * sizeof(T),
                         hipMemcpyDeviceToDevice, s);
  auto buf = [&](int l) -> T* {
    if (l == 0) return b0;
    if constexpr (f64) return H.lv[l].buf64; else return H.lv[l].buf32;
  };
  const int vm = f64 ? kF64Pos : kF32Pos;
  for (int l = 0; l < L; ++l) {
    const Level& lv = H.lv[l];
    SpmvArgs<T> a{};
    a.rp = lv.down_rp;
    a.col = lv.down_col;
    if constexpr (f64) {
      a.vals = lv.down_v64;
      a.diag = H.zero64;
    } else {
      a.vals = lv.down_v32;
      a.diag = H.zero32;
    }
    a.x = buf(l);
    a.y = l + 1 < L ? buf(l + 1) : bL;
    a.n = lv.n;  // length of x read by the products (bounds the hub copy)
    a.trim = -1;
    a.st = st;
    a.check_done = check_done;
    launch_spmv<T>(lv.down, vm, a, rb, s);
  }
  T* xL = L ? buf(L - 1) + H.lv[L - 1].ld : out;
  k_ml_coarse<T><<<(H.nL + 3) / 4, 256, 0, s>>>(H.nL, H.mL, H.cidx, H.cpos, H.Ainv, H.cdinv,
                                                 bL, xL, st, check_done);
  for (int l = L - 1; l >= 0; --l) {
    const Level& lv = H.lv[l];
    SpmvArgs<T> a{};
    a.rp = lv.up_rp;
    a.col = lv.up_col;
    if constexpr (f64) {
      a.vals = lv.up_v64;
      a.diag = lv.up_diag64;
    } else {
      a.vals = lv.up_v32;
      a.diag = lv.up_diag32;
    }
    a.x = buf(l);
    a.y = l > 0 ? buf(l - 1) + H.lv[l - 1].ld : out;
    a.n = lv.ld + lv.nc;
    a.trim = l == 0 ? H.trim : -1;
    a.st = st;
    a.check_done = check_done;
    launch_spmv<T>(lv.up, vm, a, rb, s);
  }
}

}  // namespace ml
}  // namespace isira

// Host-only: the hierarchy's shape for a caller CSR (caller labels, no relabelling), as
// isira_ml_setup would build it; no GPU is touched.
extern "C" int isira_ml_shape(int64_t n, const int32_t* row_ptr, const int32_t* col,
                              const double* w, int64_t trim, const isira_ml_options* opt,
                              isira_ml_info* info) {
  return isira::guarded([&]() -> int {
    using namespace isira::ml;
    if (n < 3 || !row_ptr || !col || !opt || !info) return isira::set_error(ISIRA_E_ARG, "bad argument");
    if (trim < 0 || trim >= n) return isira::set_error(ISIRA_E_ARG, "trim out of range");
    if (!(opt->omega > 0.0 && opt->omega < 1.0) || opt->coarse_max < 0 || opt->coarse_max > 2048 ||
        opt->max_levels < 1 || opt->max_levels > ISIRA_ML_MAX_LEVELS)
      return isira::set_error(ISIRA_E_ARG, "options out of range");
    std::vector<int32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    std::vector<HostLevel> lev;
    std::vector<std::vector<int32_t>> aggs;
    std::vector<HostMats> mats;
    HostCoarsest co;
    Params prm{opt->omega, opt->coarse_max, opt->max_levels};
    const int rc = build_host((int)n, row_ptr, col, w, perm.data(), (int)trim, prm, lev, aggs, mats, co);
    if (rc) return rc;
    std::memset(info, 0, sizeof(*info));
    info->levels = (int32_t)lev.size();
    for (size_t l = 0; l < lev.size() && l < ISIRA_ML_MAX_LEVELS; ++l) {
      int64_t conn = 0;
      for (int i = 0; i < lev[l].n; ++i) conn += lev[l].rowlen(i) > 0;
      info->rows[l] = l == 0 ? lev[l].n - 1 : lev[l].n;
      info->offdiag_nnz[l] = (int64_t)lev[l].col.size();
      info->connected[l] = conn;
    }
    info->coarsest_dense = co.m;
    for (const HostMats& M : mats) info->stored_nnz += (int64_t)M.dcol.size() + (int64_t)M.ucol.size();
    return ISIRA_OK;
  });
}

// Host-only: level `level` of the same hierarchy as CSR of its off-diagonal weights (the
// matrix entries are their negatives), its diagonal and its aggregation map into the next
// level (all -1 on the coarsest).  Level 0 is in the caller's labels with the trimmed
// vertex's row empty; a coarse level numbers its vertices in the order of their aggregates'
// first members on the finer level.  With rp_out NULL only *rows and *nnz are set.
extern "C" int isira_ml_level_matrix(int64_t n, const int32_t* row_ptr, const int32_t* col,
                                     const double* w, int64_t trim, const isira_ml_options* opt,
                                     int32_t level, int64_t* rows, int64_t* nnz, int32_t* rp_out,
                                     int32_t* col_out, double* w_out, double* diag_out,
                                     int32_t* agg_out) {
  return isira::guarded([&]() -> int {
    using namespace isira::ml;
    if (n < 3 || !row_ptr || !col || !opt || !rows || !nnz) return isira::set_error(ISIRA_E_ARG, "bad argument");
    if (trim < 0 || trim >= n) return isira::set_error(ISIRA_E_ARG, "trim out of range");
    if (!(opt->omega > 0.0 && opt->omega < 1.0) || opt->coarse_max < 0 || opt->coarse_max > 2048 ||
        opt->max_levels < 1 || opt->max_levels > ISIRA_ML_MAX_LEVELS)
      return isira::set_error(ISIRA_E_ARG, "options out of range");
    std::vector<int32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    std::vector<HostLevel> lev;
    std::vector<std::vector<int32_t>> aggs;
    std::vector<HostMats> mats;
    HostCoarsest co;
    Params prm{opt->omega, opt->coarse_max, opt->max_levels};
    const int rc = build_host((int)n, row_ptr, col, w, perm.data(), (int)trim, prm, lev, aggs, mats, co);
    if (rc) return rc;
    if (level < 0 || level >= (int)lev.size()) return isira::set_error(ISIRA_E_ARG, "level out of range");
    const HostLevel& A = lev[level];
    *rows = A.n;
    *nnz = (int64_t)A.col.size();
    if (!rp_out) return ISIRA_OK;
    if (!col_out || !w_out || !diag_out || !agg_out) return isira::set_error(ISIRA_E_ARG, "NULL output");
    std::copy(A.rp.begin(), A.rp.end(), rp_out);
    std::copy(A.col.begin(), A.col.end(), col_out);
    std::copy(A.w.begin(), A.w.end(), w_out);
    std::copy(A.diag.begin(), A.diag.end(), diag_out);
    if (level < (int)aggs.size())
      std::copy(aggs[level].begin(), aggs[level].end(), agg_out);
    else
      std::fill(agg_out, agg_out + A.n, -1);
    return ISIRA_OK;
  });
}

namespace isira {
namespace ml {

template void apply<double>(const Hierarchy&, const double*, double*, int, DevState*, RedBuf,
                            hipStream_t, bool);
template void apply<float>(const Hierarchy&, const float*, float*, int, DevState*, RedBuf,
                           hipStream_t, bool);

}  // namespace ml
}  // namespace isira
