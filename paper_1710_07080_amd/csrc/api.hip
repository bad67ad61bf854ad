// Host side of the gfx950 iSIRA library: context creation (validation, connectivity,
// relabelling, SpMV plan, degrees / trim index / delta on the GPU), the outer loop of
// Algorithm 3.2, the inner PCG driver and the operator-level entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "guard.h"
#include "internal.h"
#include "multilevel.h"
#include "spai.h"

using namespace isira;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define CKH(expr)                                                                     \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ISIRA_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

int hw_threads() {
  unsigned h = std::thread::hardware_concurrency();
  return h == 0 ? 1 : (h > 16 ? 16 : (int)h);
}

// f(begin, end) over contiguous ranges of [0, n), one host thread each (a range whose
// thread cannot be started runs on the calling thread); an exception in any range is
// rethrown after every thread has joined.
template <typename F>
void parallel_for(int64_t n, F f) {
  const int nt = hw_threads();
  if (n < 100000 || nt == 1) {
    f(0, n);
    return;
  }
  std::vector<std::exception_ptr> ex(nt);
  std::vector<std::thread> th;
  th.reserve(nt);
  const int64_t chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int64_t b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) continue;
    auto job = [&, t, b, e] {
      try {
        f(b, e);
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
  for (auto& x : ex)
    if (x) std::rethrow_exception(x);
}

}  // namespace

// ------------------------------------------------------------------------ device memory

void isira::DevMem::attach(void* base, size_t bytes) {
  // the range is used from its first 256-byte boundary on
  const uintptr_t b = (uintptr_t)base;
  const uintptr_t a = (b + kAlign - 1) / kAlign * kAlign;
  base_ = (char*)a;
  cap_ = bytes > (a - b) ? (bytes - (a - b)) / kAlign * kAlign : 0;
  free_.clear();
  if (cap_ > 0) free_[0] = cap_;
}

int isira::DevMem::alloc(void** p, size_t bytes) {
  *p = nullptr;
  const size_t need = dev_round(bytes);
  if (!base_) {
    const hipError_t e = hipMalloc(p, need);
    if (e != hipSuccess) {
      *p = nullptr;
      return ISIRA_E_HIP;
    }
  } else {
    auto it = free_.begin();
    while (it != free_.end() && it->second < need) ++it;
    if (it == free_.end()) return ISIRA_E_WORKSPACE;
    const size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > need) free_[off + need] = len - need;
    *p = base_ + off;
  }
  live_[*p] = need;
  in_use_ += need;
  if (in_use_ > peak_) peak_ = in_use_;
  return ISIRA_OK;
}

void isira::DevMem::release(void* p) {
  auto it = live_.find(p);
  if (it == live_.end()) return;
  const size_t len = it->second;
  live_.erase(it);
  in_use_ -= len;
  if (!base_) {
    (void)hipFree(p);
    return;
  }
  size_t off = (size_t)((char*)p - base_), end = off + len;
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && nx->first == end) {  // merge with the next free range
    end += nx->second;
    nx = free_.erase(nx);
  }
  if (nx != free_.begin()) {  // merge with the previous one
    auto pv = std::prev(nx);
    if (pv->first + pv->second == off) {
      off = pv->first;
      free_.erase(pv);
    }
  }
  free_[off] = end - off;
}

int isira::dev_alloc_bytes(DevMem& m, void** p, size_t bytes) {
  const int rc = m.alloc(p, bytes);
  if (rc == ISIRA_E_WORKSPACE)
    return fail(rc, "workspace too small: no free range of " + std::to_string(dev_round(bytes)) +
                        " bytes (" + std::to_string(m.in_use()) + " of " +
                        std::to_string(m.capacity()) + " bytes in use)");
  if (rc != ISIRA_OK)
    return fail(rc, "hipMalloc(" + std::to_string(dev_round(bytes)) + " bytes) failed");
  return ISIRA_OK;
}

// ----------------------------------------------------- scratch of the allocation-free CGS2
// Device memory of isira_orthonormalize_noalloc: the reduction partials of its column dots,
// the column values, a saved norm and the small state.  One copy per GPU, held until the
// process ends; every call on a GPU uses the same copy.
constexpr int kNoAllocMaxCols = ISIRA_MAX_BASIS;
constexpr size_t kNoAllocPartials = (size_t)(kNoAllocMaxCols + 2) * kStreamGrid;  // doubles
constexpr size_t kNoAllocH = kNoAllocPartials;             // kMaxCols column values
constexpr size_t kNoAllocNorm0 = kNoAllocH + kMaxCols;      // ||z||^2 before the first pass
constexpr size_t kNoAllocState = (kNoAllocNorm0 + 1 + 31) / 32 * 32;  // DevState, 256-B aligned
constexpr size_t kNoAllocBytes =
    (kNoAllocState * sizeof(double) + sizeof(DevState) + 255) / 256 * 256;
static_assert(kNoAllocBytes <= ((size_t)2 << 20), "scratch of the allocation-free CGS2 exceeds 2 MiB");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_addr;  // per device: device address of `scratch`

// Address of this GPU's copy of `scratch` (the device current on entry), looked up once per
// device.  Host code uses only this address, never the array's name.
int scratch_address(void** out) {
  *out = nullptr;
  int dev = 0;
  CKH(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_addr.size() <= dev) g_scratch_addr.resize(dev + 1, nullptr);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ISIRA_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return ISIRA_OK;
}
}  // namespace

// ------------------------------------------------------------------------------ context

struct isira_ctx {
  DevMem mem;  // every device buffer of the context (own hipMallocs or the caller's workspace)
  int64_t n = 0, nnz = 0;
  int ld = 0;  // leading dimension of dense n-by-m blocks
  int wdt = ISIRA_W_NONE;
  hipStream_t stream = nullptr;
  std::vector<int32_t> perm, iperm;  // perm[new] = caller label, iperm[label] = new
  // device graph (relabelled)
  int32_t* rp = nullptr;
  int32_t* col = nullptr;
  double* w64 = nullptr;
  float* w32 = nullptr;
  double* deg = nullptr;
  float* deg32 = nullptr;
  int32_t* d_perm = nullptr;   // new -> label
  int32_t* d_iperm = nullptr;  // label -> new
  int32_t* d_emap = nullptr;   // internal stored entry -> caller entry index
  SpmvPlan plan;
  RedBuf rb{nullptr, nullptr};
  DevState* st = nullptr;
  DevState* st_host = nullptr;  // pinned
  double* hbuf = nullptr;       // device kMaxCols
  double* hbuf_host = nullptr;  // pinned 2 * kMaxCols (second half: CGS2 first-pass values)
  unsigned char* up_host = nullptr;  // pinned upload ring for small host-to-device copies
  size_t up_off = 0;                 // next free byte; reset whenever the stream is idle
  double* scal4 = nullptr;      // device 4
  int trim_default = 0;         // internal index
  int64_t trim_label = 0;
  double max_deg = 0, min_deg = 0;
  // solve workspace
  int ws_m = 0, ws_k = 0;
  // entries past ld of the inner residual buffers ri64/ri32: the multilevel cycle runs in
  // place there (x of its second level after the residual); ws_tail is what is allocated
  int ri_tail = 0, ws_tail = 0;
  double *U = nullptr, *W = nullptr, *Vout = nullptr;
  double *Vin64 = nullptr, *Y64 = nullptr;
  float *Vin32 = nullptr, *Y32 = nullptr;
  double *r64 = nullptr, *z64 = nullptr, *tmp64 = nullptr;
  double *x64 = nullptr, *ri64 = nullptr, *p64 = nullptr, *q64 = nullptr, *dinv64 = nullptr,
         *y64 = nullptr;
  float *x32 = nullptr, *ri32 = nullptr, *p32 = nullptr, *q32 = nullptr, *dinv32 = nullptr,
        *y32 = nullptr;
  double *wa64 = nullptr, *wb64 = nullptr;  // MINRES directions
  float *wa32 = nullptr, *wb32 = nullptr;
  int minres_next = 1;  // number of the next MINRES iteration to queue
  double* svec = nullptr;  // device ISIRA_MAX_BASIS
  double* Sdev = nullptr;  // device ISIRA_MAX_BASIS^2
  double* Ginv = nullptr;  // device kMaxC^2
  // learned preconditioner: values of M in internal order (spw.diag32/diag64/offd)
  double spai_sigma = 0.0;
  int spai_trim = -1;
  bool has_learned = false;
  // multilevel preconditioner (hierarchy of L-hat for the trim index ml.trim)
  ml::Hierarchy ml;
  spai::SpaiWork spw;
  // this GPU's copy of the allocation-free CGS2 scratch (looked up at creation)
  unsigned char* scratch_dev = nullptr;
};

// Power-law test on the degree-sorted labels: at least a quarter of the gathers hit the
// kHubTestCols highest-degree vertices (the hub-cached product shape is then used).
static bool power_law(int64_t n, const int32_t* rp, const int32_t* col,
                      const std::vector<int32_t>& rank) {
  if (n <= 4 * (int64_t)kHubTestCols) return false;
  int64_t hits = 0;
  const int64_t nnz = rp[n];
  for (int64_t j = 0; j < nnz; ++j) hits += rank[col[j]] < kHubTestCols;
  return (double)hits >= 0.25 * (double)nnz;
}

// Reverse Cuthill-McKee order of a connected graph: breadth-first search from a
// pseudo-peripheral vertex (two sweeps starting at a minimum-degree vertex), neighbours
// taken in increasing degree, and the visiting order reversed.  perm[new] = old label.
static void rcm_order(int64_t n, const int32_t* rp, const int32_t* col,
                      const std::vector<int32_t>& deg, std::vector<int32_t>& perm,
                      std::vector<int32_t>& iperm) {
  std::vector<int32_t> order(n), level(n);
  auto bfs = [&](int32_t start, bool sorted) {
    std::fill(level.begin(), level.end(), -1);
    int64_t head = 0, tail = 0;
    order[tail++] = start;
    level[start] = 0;
    std::vector<int32_t> nb;
    while (head < tail) {
      const int32_t v = order[head++];
      nb.clear();
      for (int32_t j = rp[v]; j < rp[v + 1]; ++j)
        if (level[col[j]] < 0) {
          level[col[j]] = level[v] + 1;
          nb.push_back(col[j]);
        }
      if (sorted)
        std::stable_sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
      for (int32_t u : nb) order[tail++] = u;
    }
    return order[tail - 1];  // a vertex of the last level
  };
  int32_t start = 0;
  for (int64_t i = 1; i < n; ++i)
    if (deg[i] < deg[start]) start = (int32_t)i;
  for (int sweep = 0; sweep < 2; ++sweep) start = bfs(start, false);
  bfs(start, true);
  for (int64_t i = 0; i < n; ++i) {
    perm[i] = order[n - 1 - i];
    iperm[perm[i]] = (int32_t)i;
  }
}

// SpMV work units of a CSR matrix with n rows (the relabelled Laplacian: rows by
// decreasing length, or in reverse Cuthill-McKee order; a multilevel transfer matrix: any
// order): a row longer than the unit size is cut into chunks; runs of the other rows are
// packed greedily, in order, into stream units of at most unit-size nonzeros and a row
// limit.  A stream unit sums each row with G lanes, G the smallest power of two >=
// (longest row) / 8, capped at 64.  Matrices whose gathers concentrate on the first kHubTestCols
// columns (the highest-degree vertices after relabelling) use the hub-cached shape.
int isira::build_spmv_plan(DevMem& mem, int n, const int32_t* rp, const int32_t* col, SpmvPlan& P) {
  const int64_t nnz = rp[n];
  int64_t hits = 0;
  for (int64_t j = 0; j < nnz; ++j) hits += col[j] < kHubTestCols;
  P.hub = (n > 4 * kHubTestCols && (double)hits >= 0.25 * (double)nnz) ? 1 : 0;
  const int unnz = P.hub ? kHubUnitNnz : kUnitNnz;
  const int urows = P.hub ? kHubUnitRows : kUnitRows;
  const int chunk = unnz;  // nonzeros per piece of a long row
  std::vector<int4> units;
  std::vector<int32_t> rowof, base, nch;
  int nchunks = 0;
  int row = 0;
  while (row < n) {
    const int len = rp[row + 1] - rp[row];
    if (len > unnz) {
      const int nc = (len + chunk - 1) / chunk;
      rowof.push_back(row);
      base.push_back(nchunks);
      nch.push_back(nc);
      for (int c = 0; c < nc; ++c) {
        const int j0 = rp[row] + c * chunk;
        const int j1 = std::min(rp[row + 1], j0 + chunk);
        units.push_back(make_int4(row, j0, j1, -(nchunks + c + 1)));
      }
      nchunks += nc;
      ++row;
      continue;
    }
    const int r0 = row;
    int lmax = 0, cnt = 0;
    while (row < n && row - r0 < urows) {
      const int l = rp[row + 1] - rp[row];
      if (l > unnz || cnt + l > unnz) break;
      cnt += l;
      lmax = std::max(lmax, l);
      ++row;
    }
    int G = 1;
    while (G < 64 && G * 8 < lmax) G <<= 1;
    units.push_back(make_int4(r0, rp[r0], rp[row], ((row - r0) << 8) | G));
  }
  P.n_units = (int)units.size();
  P.grid = std::max(1, std::min(P.n_units, P.hub ? kHubGrid : kSpmvGrid));
  P.n_split_units = nchunks;
  P.n_split_rows = (int)rowof.size();
  int rc;
  if ((rc = dalloc(mem, &P.units, units.size()))) return rc;
  if ((rc = dalloc(mem, &P.split_rowof, rowof.size()))) return rc;
  if ((rc = dalloc(mem, &P.split_base, rowof.size()))) return rc;
  if ((rc = dalloc(mem, &P.split_nchunk, rowof.size()))) return rc;
  if ((rc = dalloc(mem, &P.split_part, (size_t)nchunks))) return rc;
  if ((rc = dalloc(mem, &P.split_red, rowof.size()))) return rc;
  if (!units.empty())
    CKH(hipMemcpy(P.units, units.data(), units.size() * sizeof(int4), hipMemcpyHostToDevice));
  if (!rowof.empty()) {
    CKH(hipMemcpy(P.split_rowof, rowof.data(), rowof.size() * 4, hipMemcpyHostToDevice));
    CKH(hipMemcpy(P.split_base, base.data(), base.size() * 4, hipMemcpyHostToDevice));
    CKH(hipMemcpy(P.split_nchunk, nch.data(), nch.size() * 4, hipMemcpyHostToDevice));
  }
  return ISIRA_OK;
}

void isira::free_spmv_plan(DevMem& mem, SpmvPlan& P) {
  dfree(mem, P.units); dfree(mem, P.split_base); dfree(mem, P.split_nchunk);
  dfree(mem, P.split_rowof); dfree(mem, P.split_part); dfree(mem, P.split_red);
  P = SpmvPlan{};
}

// Stream units: of two consecutive ones, the first plus the next row exceeds the unit size or
// the first holds the row limit, so there are at most 2 (nnz / unit + n / rows) + 1; chunk
// units and split rows are at most nnz / unit + n_split each (smallest shape's constants).
size_t isira::spmv_plan_bytes_bound(int64_t n, int64_t nnz) {
  const size_t unnz = (size_t)std::min(kUnitNnz, kHubUnitNnz);
  const size_t urows = (size_t)std::min(kUnitRows, kHubUnitRows);
  const size_t split = (size_t)nnz / unnz + 1;
  const size_t units = 2 * ((size_t)nnz / unnz + (size_t)n / urows) + 1 + (size_t)nnz / unnz + split;
  return dev_round(units * sizeof(int4)) + 3 * dev_round(split * 4) + dev_round((size_t)nnz / unnz * 8 + split * 8) +
         dev_round(split * 8);
}

static void free_workspace(isira_ctx* c) {
  dfree(c->mem, c->U); dfree(c->mem, c->W); dfree(c->mem, c->Vout); dfree(c->mem, c->Vin64); dfree(c->mem, c->Y64); dfree(c->mem, c->Vin32);
  dfree(c->mem, c->Y32); dfree(c->mem, c->r64); dfree(c->mem, c->z64); dfree(c->mem, c->tmp64); dfree(c->mem, c->x64); dfree(c->mem, c->ri64);
  dfree(c->mem, c->p64); dfree(c->mem, c->q64); dfree(c->mem, c->dinv64); dfree(c->mem, c->y64); dfree(c->mem, c->x32); dfree(c->mem, c->ri32);
  dfree(c->mem, c->p32); dfree(c->mem, c->q32); dfree(c->mem, c->dinv32); dfree(c->mem, c->y32);
  dfree(c->mem, c->wa64); dfree(c->mem, c->wb64); dfree(c->mem, c->wa32); dfree(c->mem, c->wb32);
  c->ws_m = c->ws_k = 0;
}

static int ensure_workspace(isira_ctx* c, int m, int kmax) {
  if (c->ws_m >= m && c->ws_k >= kmax && c->ws_tail >= c->ri_tail && c->r64) return ISIRA_OK;
  free_workspace(c);
  const size_t ld = (size_t)c->ld;
  int rc;
  if ((rc = dalloc(c->mem, &c->U, ld * m))) return rc;
  if ((rc = dalloc(c->mem, &c->W, ld * m))) return rc;
  if ((rc = dalloc(c->mem, &c->Vout, ld * kmax))) return rc;
  // deflation blocks of the inner solve: whole column groups, zeroed once (the kernels read
  // the padding columns and weight them by 0, which needs finite values)
  const size_t kpad = (size_t)std::max(pick_cm(kmax), 4);
  if ((rc = dalloc(c->mem, &c->Vin64, ld * kpad))) return rc;
  if ((rc = dalloc(c->mem, &c->Y64, ld * kpad))) return rc;
  if ((rc = dalloc(c->mem, &c->Vin32, ld * kpad))) return rc;
  if ((rc = dalloc(c->mem, &c->Y32, ld * kpad))) return rc;
  CKH(hipMemset(c->Vin64, 0, ld * kpad * sizeof(double)));
  CKH(hipMemset(c->Y64, 0, ld * kpad * sizeof(double)));
  CKH(hipMemset(c->Vin32, 0, ld * kpad * sizeof(float)));
  CKH(hipMemset(c->Y32, 0, ld * kpad * sizeof(float)));
  for (double** p : {&c->r64, &c->z64, &c->tmp64, &c->x64, &c->p64, &c->q64,
                     &c->dinv64, &c->y64, &c->wa64, &c->wb64})
    if ((rc = dalloc(c->mem, p, ld))) return rc;
  for (float** p : {&c->x32, &c->p32, &c->q32, &c->dinv32, &c->y32, &c->wa32, &c->wb32})
    if ((rc = dalloc(c->mem, p, ld))) return rc;
  if ((rc = dalloc(c->mem, &c->ri64, ld + c->ri_tail))) return rc;
  if ((rc = dalloc(c->mem, &c->ri32, ld + c->ri_tail))) return rc;
  c->ws_tail = c->ri_tail;
  c->ws_m = m;
  c->ws_k = kmax;
  return ISIRA_OK;
}

extern "C" int isira_default_options(isira_options* o) {
  if (!o) return ISIRA_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->m = 0;
  o->q = 0;
  o->k0 = 4;
  o->inner_rtol = 1e-1;
  o->max_inner = 1000;
  o->max_outer = 20000;
  o->inner_prec = ISIRA_FP64;
  o->precond = ISIRA_PC_JACOBI;
  o->trim_index = -1;
  o->delta = 0.0;
  o->seed = 12345;
  o->u0 = nullptr;
  o->check_every = 8;
  return ISIRA_OK;
}

static int validate_graph(int64_t n, int64_t nnz, const int32_t* rp, const int32_t* col,
                          const void* w, int wdt, int check_sym) {
  if (rp[0] != 0 || rp[n] != nnz) return fail(ISIRA_E_GRAPH, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  std::atomic<int> bad{0};
  std::atomic<int64_t> where{-1};
  parallel_for(n, [&](int64_t b, int64_t e) {
    for (int64_t i = b; i < e && !bad.load(std::memory_order_relaxed); ++i) {
      const int s = rp[i], t = rp[i + 1];
      if (t < s) { bad = 1; where = i; return; }
      for (int j = s; j < t; ++j) {
        const int c = col[j];
        if (c < 0 || c >= n) { bad = 2; where = i; return; }
        if (c == i) { bad = 3; where = i; return; }
        if (j > s && col[j - 1] >= c) { bad = 4; where = i; return; }
        if (wdt == ISIRA_W_F32) {
          const float v = ((const float*)w)[j];
          if (!(v > 0.0f) || !std::isfinite(v)) { bad = 5; where = i; return; }
        } else if (wdt == ISIRA_W_F64) {
          const double v = ((const double*)w)[j];
          if (!(v > 0.0) || !std::isfinite(v)) { bad = 5; where = i; return; }
        }
        if (check_sym) {
          const int32_t* lo = col + rp[c];
          const int32_t* hi = col + rp[c + 1];
          const int32_t* f = std::lower_bound(lo, hi, (int32_t)i);
          if (f == hi || *f != i) { bad = 6; where = i; return; }
          const int64_t jt = f - col;
          if (wdt == ISIRA_W_F32 && ((const float*)w)[jt] != ((const float*)w)[j]) { bad = 7; where = i; return; }
          if (wdt == ISIRA_W_F64 && ((const double*)w)[jt] != ((const double*)w)[j]) { bad = 7; where = i; return; }
        }
      }
    }
  });
  static const char* msg[] = {"", "row_ptr decreasing", "column index out of range",
                              "self loop", "columns not sorted/unique", "weight not positive",
                              "pattern not symmetric", "weights not symmetric"};
  if (bad) return fail(ISIRA_E_GRAPH, std::string(msg[bad.load()]) + " at row " + std::to_string(where.load()));
  return ISIRA_OK;
}

static bool connected(int64_t n, const int32_t* rp, const int32_t* col) {
  std::vector<uint8_t> seen(n, 0);
  std::vector<int32_t> stack;
  stack.reserve(1024);
  stack.push_back(0);
  seen[0] = 1;
  int64_t count = 1;
  while (!stack.empty()) {
    const int v = stack.back();
    stack.pop_back();
    for (int j = rp[v]; j < rp[v + 1]; ++j) {
      const int u = col[j];
      if (!seen[u]) {
        seen[u] = 1;
        ++count;
        stack.push_back(u);
      }
    }
  }
  return count == n;
}

static int create_impl(isira_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                       const int32_t* col, const void* w, int32_t w_dtype, void* stream,
                       int32_t validate, void* workspace, size_t ws_bytes);

extern "C" int isira_create(isira_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                            const int32_t* col, const void* w, int32_t w_dtype, void* stream,
                            int32_t validate) {
  return guarded([&]() -> int {
    return create_impl(out, n, nnz, row_ptr, col, w, w_dtype, stream, validate, nullptr, 0);
  });
}

static int create_impl(isira_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                       const int32_t* col, const void* w, int32_t w_dtype, void* stream,
                       int32_t validate, void* workspace, size_t ws_bytes) {
  if (!out) return fail(ISIRA_E_ARG, "out is NULL");
  *out = nullptr;
  if (n < 3 || n >= (1ll << 31) - 64 || nnz < 2 || nnz >= (1ll << 31) || !row_ptr || !col)
    return fail(ISIRA_E_ARG, "need 3 <= n < 2^31, 2 <= nnz < 2^31 and non-NULL CSR arrays");
  if (w_dtype != ISIRA_W_NONE && w_dtype != ISIRA_W_F32 && w_dtype != ISIRA_W_F64)
    return fail(ISIRA_E_ARG, "bad w_dtype");
  if (w_dtype != ISIRA_W_NONE && !w) return fail(ISIRA_E_ARG, "weights are NULL");
  int rc = validate_graph(n, nnz, row_ptr, col, w, w_dtype, validate);
  if (rc) return rc;
  if (!connected(n, row_ptr, col)) return fail(ISIRA_E_DISCONNECTED, "graph is not connected");

  void* scratch_dev = nullptr;
  if ((rc = scratch_address(&scratch_dev))) return rc;
  isira_ctx* ctx = new isira_ctx();
  if (workspace) ctx->mem.attach(workspace, ws_bytes);
  ctx->scratch_dev = (unsigned char*)scratch_dev;
  ctx->spw.mem = &ctx->mem;
  ctx->ml.mem = &ctx->mem;
  ctx->n = n;
  ctx->nnz = nnz;
  ctx->ld = (int)((n + 63) / 64 * 64);
  ctx->wdt = w_dtype;
  ctx->stream = (hipStream_t)stream;
  // relabel: stable sort by decreasing row length
  std::vector<int32_t> cnt(n);
  int32_t maxc = 0;
  for (int64_t i = 0; i < n; ++i) {
    cnt[i] = row_ptr[i + 1] - row_ptr[i];
    maxc = std::max(maxc, cnt[i]);
  }
  {
    std::vector<int64_t> bucket((size_t)maxc + 2, 0);
    for (int64_t i = 0; i < n; ++i) bucket[maxc - cnt[i] + 1]++;
    for (size_t b = 1; b < bucket.size(); ++b) bucket[b] += bucket[b - 1];
    ctx->perm.resize(n);
    ctx->iperm.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t pos = bucket[maxc - cnt[i]]++;
      ctx->perm[pos] = (int32_t)i;
      ctx->iperm[i] = (int32_t)pos;
    }
  }
  // Graphs whose gathers do not concentrate on a few hub labels (and whose rows all fit one
  // stream unit) are relabelled in reverse Cuthill-McKee order instead, so that the x
  // entries a unit gathers sit close together in memory.
  if (maxc <= kUnitNnz && !power_law(n, row_ptr, col, ctx->iperm)) rcm_order(n, row_ptr, col, cnt, ctx->perm, ctx->iperm);
  std::vector<int32_t> rp2(n + 1), col2(nnz);
  rp2[0] = 0;
  for (int64_t r = 0; r < n; ++r) rp2[r + 1] = rp2[r] + cnt[ctx->perm[r]];
  std::vector<double> w2d;
  std::vector<float> w2f;
  if (w_dtype != ISIRA_W_NONE) {
    w2d.resize(nnz);
    w2f.resize(nnz);
  }
  std::vector<int32_t> emap(nnz);
  parallel_for(n, [&](int64_t b, int64_t e) {
    std::vector<std::pair<int32_t, int32_t>> tmp;
    for (int64_t r = b; r < e; ++r) {
      const int old = ctx->perm[r];
      const int s = row_ptr[old], t = row_ptr[old + 1];
      tmp.resize(t - s);
      for (int j = s; j < t; ++j) tmp[j - s] = {ctx->iperm[col[j]], j};
      std::sort(tmp.begin(), tmp.end());
      const int o = rp2[r];
      for (size_t j = 0; j < tmp.size(); ++j) {
        col2[o + j] = tmp[j].first;
        emap[o + j] = tmp[j].second;
        double wv = 1.0;
        if (w_dtype == ISIRA_W_F32) wv = ((const float*)w)[tmp[j].second];
        if (w_dtype == ISIRA_W_F64) wv = ((const double*)w)[tmp[j].second];
        if (w_dtype != ISIRA_W_NONE) {
          w2d[o + j] = wv;
          w2f[o + j] = (float)wv;
        }
      }
    }
  });
  auto cleanup = [&](int code) {
    isira_destroy(ctx);
    return code;
  };
  if ((rc = dalloc(ctx->mem, &ctx->rp, n + 1))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->col, nnz))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->deg, ctx->ld))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->deg32, ctx->ld))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->d_perm, n))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->d_iperm, n))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->d_emap, nnz))) return cleanup(rc);
  if (w_dtype != ISIRA_W_NONE) {
    if ((rc = dalloc(ctx->mem, &ctx->w64, nnz))) return cleanup(rc);
    if ((rc = dalloc(ctx->mem, &ctx->w32, nnz))) return cleanup(rc);
  }
  if ((rc = dalloc(ctx->mem, &ctx->rb.partials, kPartialsElems))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->rb.counters, 64))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->st, 1))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->hbuf, kMaxCols))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->scal4, 4))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->svec, ISIRA_MAX_BASIS))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->Sdev, (size_t)ISIRA_MAX_BASIS * ISIRA_MAX_BASIS))) return cleanup(rc);
  if ((rc = dalloc(ctx->mem, &ctx->Ginv, (size_t)kMaxC * kMaxC))) return cleanup(rc);
  if (hipHostMalloc((void**)&ctx->st_host, sizeof(DevState)) != hipSuccess ||
      hipHostMalloc((void**)&ctx->hbuf_host, 2 * kMaxCols * sizeof(double)) != hipSuccess ||
      hipHostMalloc((void**)&ctx->up_host, kUploadRing) != hipSuccess)
    return cleanup(fail(ISIRA_E_HIP, "hipHostMalloc failed"));
  hipStream_t s = ctx->stream;
  auto up = [&](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
  };
  if (up(ctx->rp, rp2.data(), (n + 1) * 4) || up(ctx->col, col2.data(), nnz * 4) ||
      up(ctx->d_perm, ctx->perm.data(), n * 4) || up(ctx->d_iperm, ctx->iperm.data(), n * 4) ||
      up(ctx->d_emap, emap.data(), nnz * 4))
    return cleanup(fail(ISIRA_E_HIP, "upload failed"));
  if (w_dtype != ISIRA_W_NONE &&
      (up(ctx->w64, w2d.data(), nnz * 8) || up(ctx->w32, w2f.data(), nnz * 4)))
    return cleanup(fail(ISIRA_E_HIP, "weight upload failed"));
  if (hipMemsetAsync(ctx->rb.counters, 0, 64 * sizeof(unsigned), s) ||
      hipMemsetAsync(ctx->st, 0, sizeof(DevState), s) ||
      hipMemsetAsync(ctx->deg, 0, ctx->ld * 8, s) || hipMemsetAsync(ctx->deg32, 0, ctx->ld * 4, s))
    return cleanup(fail(ISIRA_E_HIP, "memset failed"));
  if ((rc = build_spmv_plan(ctx->mem, (int)n, rp2.data(), col2.data(), ctx->plan))) return cleanup(rc);
  // degrees, trim index (Remark 4.1(i)) and delta (Remark 4.1(ii)) on the GPU
  launch_degree(ctx->rp, w_dtype == ISIRA_W_NONE ? nullptr : (w_dtype == ISIRA_W_F32 ? (const void*)ctx->w32 : (const void*)ctx->w64),
                w_dtype == ISIRA_W_NONE ? ISIRA_W_NONE : (w_dtype == ISIRA_W_F32 ? ISIRA_W_F32 : ISIRA_W_F64),
                (int)n, ctx->deg, ctx->deg32, s);
  launch_argmax_degree(ctx->deg, ctx->d_perm, (int)n, ctx->st, ctx->rb, ctx->scal4, s);
  double out4[4];
  if (hipMemcpyAsync(out4, ctx->scal4, sizeof(out4), hipMemcpyDeviceToHost, s) ||
      hipStreamSynchronize(s))
    return cleanup(fail(ISIRA_E_HIP, std::string("setup kernels failed: ") + hipGetErrorString(hipGetLastError())));
  ctx->max_deg = out4[0];
  ctx->trim_default = (int)out4[1];
  ctx->min_deg = out4[2];
  ctx->trim_label = (int64_t)out4[3];
  *out = ctx;
  return ISIRA_OK;
}

// ------------------------------------------------------------- caller-owned workspace

// Device bytes of ensure_workspace(m, kmax) for leading dimension ld and tail entries.
static size_t solve_ws_bytes(size_t ld, int m, int kmax, int tail) {
  const size_t kpad = (size_t)std::max(pick_cm(kmax), 4);
  return 2 * dev_round(ld * m * 8) + dev_round(ld * kmax * 8) + 2 * dev_round(ld * kpad * 8) +
         2 * dev_round(ld * kpad * 4) + 10 * dev_round(ld * 8) + 7 * dev_round(ld * 4) +
         dev_round((ld + tail) * 8) + dev_round((ld + tail) * 4);
}

// Device bytes create_impl allocates (the SpMV plan by its bound).
static size_t create_bytes(int64_t n, int64_t nnz, int wdt) {
  const size_t ld = (size_t)((n + 63) / 64 * 64);
  size_t b = dev_round((n + 1) * 4) + dev_round(nnz * 4) + dev_round(ld * 8) + dev_round(ld * 4) +
             2 * dev_round(n * 4) + dev_round(nnz * 4);
  if (wdt != ISIRA_W_NONE) b += dev_round(nnz * 8) + dev_round(nnz * 4);
  b += dev_round(kPartialsElems * 8) + dev_round(64 * 4) + dev_round(sizeof(DevState)) +
       dev_round(kMaxCols * 8) + dev_round(4 * 8) + dev_round(ISIRA_MAX_BASIS * 8) +
       dev_round((size_t)ISIRA_MAX_BASIS * ISIRA_MAX_BASIS * 8) + dev_round((size_t)kMaxC * kMaxC * 8);
  return b + spmv_plan_bytes_bound(n, nnz);
}

static void solve_sizes(int k, const isira_options* opt, int* m_out) {
  const int q = (opt && opt->q > 0) ? opt->q : k + 10;
  *m_out = (opt && opt->m > 0) ? opt->m : 2 * q;
}

extern "C" size_t isira_workspace_bytes(int64_t n, int64_t nnz, int32_t w_dtype, int32_t k,
                                        const isira_options* opt, int32_t flags) {
  if (n < 3 || nnz < 2 || k < 1 || k > ISIRA_MAX_K) return 0;
  int m = 0;
  solve_sizes(k, opt, &m);
  if (m < 2 || m > ISIRA_MAX_BASIS) return 0;
  const size_t ld = (size_t)((n + 63) / 64 * 64);
  size_t b = create_bytes(n, nnz, w_dtype) + solve_ws_bytes(ld, m, k, 0);
  if (flags & ISIRA_WS_LEARNED)  // the network's buffers and a pruned copy of every entry
    b += spai::work_bytes(n, nnz) + dev_round((n + 1) * 4) + 2 * dev_round(nnz * 4) + dev_round(n * 4);
  return b + ((size_t)1 << 20);  // slack for alignment of the caller's pointer
}

extern "C" int isira_create_ws(isira_ctx** out, int64_t n, int64_t nnz, const int32_t* row_ptr,
                               const int32_t* col, const void* w, int32_t w_dtype,
                               int32_t csr_on_device, void* workspace, size_t ws_bytes,
                               int32_t k, const isira_options* opt, void* stream,
                               int32_t validate) {
  return guarded([&]() -> int {
    if (!out) return fail(ISIRA_E_ARG, "out is NULL");
    *out = nullptr;
    if (!workspace || ws_bytes == 0) return fail(ISIRA_E_ARG, "workspace is NULL or empty");
    if (k < 1 || k > ISIRA_MAX_K) return fail(ISIRA_E_ARG, "need 1 <= k <= 64");
    int m = 0;
    solve_sizes(k, opt, &m);
    if (m < 2 || m > ISIRA_MAX_BASIS) return fail(ISIRA_E_ARG, "need 2 <= m <= 192");
    if (n < 3 || n >= (1ll << 31) - 64 || nnz < 2 || nnz >= (1ll << 31) || !row_ptr || !col)
      return fail(ISIRA_E_ARG, "need 3 <= n < 2^31, 2 <= nnz < 2^31 and non-NULL CSR arrays");
    // device CSR: the host-side validation, connectivity check and relabelling read a host copy
    std::vector<int32_t> hrp, hcol;
    std::vector<unsigned char> hw;
    if (csr_on_device) {
      hrp.resize(n + 1);
      hcol.resize(nnz);
      CKH(hipMemcpy(hrp.data(), row_ptr, (n + 1) * 4, hipMemcpyDeviceToHost));
      CKH(hipMemcpy(hcol.data(), col, nnz * 4, hipMemcpyDeviceToHost));
      if (w_dtype != ISIRA_W_NONE && w) {
        hw.resize(nnz * (w_dtype == ISIRA_W_F32 ? 4 : 8));
        CKH(hipMemcpy(hw.data(), w, hw.size(), hipMemcpyDeviceToHost));
      }
      row_ptr = hrp.data();
      col = hcol.data();
      if (!hw.empty()) w = hw.data();
    }
    isira_ctx* ctx = nullptr;
    int rc = create_impl(&ctx, n, nnz, row_ptr, col, w, w_dtype, stream, validate, workspace, ws_bytes);
    if (rc) return rc;
    // the solve workspace for (k, m) now, so that later calls carve nothing more
    if ((rc = ensure_workspace(ctx, m, k))) {
      isira_destroy(ctx);
      return rc;
    }
    *out = ctx;
    return ISIRA_OK;
  });
}

extern "C" int isira_memory_info(const isira_ctx* c, size_t* in_use, size_t* peak,
                                 size_t* capacity) {
  return guarded([&]() -> int {
    if (!c) return fail(ISIRA_E_ARG, "NULL context");
    if (in_use) *in_use = c->mem.in_use();
    if (peak) *peak = c->mem.peak();
    if (capacity) *capacity = c->mem.capacity();
    return ISIRA_OK;
  });
}

extern "C" void isira_destroy(isira_ctx* c) {
  if (!c) return;
  free_workspace(c);
  dfree(c->mem, c->rp); dfree(c->mem, c->col); dfree(c->mem, c->w64); dfree(c->mem, c->w32); dfree(c->mem, c->deg); dfree(c->mem, c->deg32);
  dfree(c->mem, c->d_perm); dfree(c->mem, c->d_iperm); dfree(c->mem, c->d_emap);
  free_spmv_plan(c->mem, c->plan);
  dfree(c->mem, c->rb.partials); dfree(c->mem, c->rb.counters); dfree(c->mem, c->st); dfree(c->mem, c->hbuf); dfree(c->mem, c->scal4);
  dfree(c->mem, c->svec); dfree(c->mem, c->Sdev); dfree(c->mem, c->Ginv);
  spai::free_work(c->spw);
  ml::release(c->ml);
  if (c->st_host) (void)hipHostFree(c->st_host);
  if (c->hbuf_host) (void)hipHostFree(c->hbuf_host);
  if (c->up_host) (void)hipHostFree(c->up_host);
  delete c;
}

extern "C" int isira_get_info(const isira_ctx* c, isira_info* info) {
  return guarded([&]() -> int {
    if (!c || !info) return fail(ISIRA_E_ARG, "NULL argument");
    info->n = c->n;
    info->nnz = c->nnz;
    info->trim_index = c->trim_label;
    info->max_degree = c->max_deg;
    info->min_degree = c->min_deg;
    info->delta_default = 2.0 * c->max_deg;
    info->norm1 = 2.0 * c->max_deg;
    info->n_spmv_units = c->plan.n_units;
    info->n_spmv_blocks = c->plan.grid;
    info->n_split_rows = c->plan.n_split_rows;
    info->has_learned = c->has_learned ? 1 : 0;
    return ISIRA_OK;
  });
}

// ------------------------------------------------------------------------------ helpers

namespace {

int valmode64(const isira_ctx* c) { return c->wdt == ISIRA_W_NONE ? kUnitNeg : kF64Neg; }
int valmode32(const isira_ctx* c) { return c->wdt == ISIRA_W_NONE ? kUnitNeg : kF32Neg; }

// y = L x (+ delta V t) in FP64 on internal vectors; red: see SpmvArgs.
void spmv64(isira_ctx* c, const double* x, double* y, const double* V, int nv,
            const double* tvec, double delta, int red, double theta) {
  SpmvArgs<double> a{};
  a.rp = c->rp;
  a.col = c->col;
  a.vals = c->w64;
  a.x = x;
  a.y = y;
  a.diag = c->deg;
  a.n = (int)c->n;
  a.trim = -1;
  a.V = V;
  a.ldv = c->ld;
  a.c = nv;
  a.tvec = tvec;
  a.delta = delta;
  a.red = red;
  a.theta = theta;
  a.st = c->st;
  launch_spmv<double>(c->plan, valmode64(c), a, c->rb, c->stream);
}

// Waits for the stream; afterwards the upload ring is free again.
int stream_sync(isira_ctx* c) {
  CKH(hipStreamSynchronize(c->stream));
  c->up_off = 0;
  return ISIRA_OK;
}

#define SYNC_OR_RETURN(c)           \
  do {                              \
    const int rc_ = stream_sync(c); \
    if (rc_) return rc_;            \
  } while (0)

int sync_state(isira_ctx* c) {
  CKH(hipMemcpyAsync(c->st_host, c->st, sizeof(DevState), hipMemcpyDeviceToHost, c->stream));
  return stream_sync(c);
}

// Queues a copy of hbuf[0:count) into hbuf_host[off:off+count) (read after a sync).
int read_h(isira_ctx* c, int count, int off = 0) {
  CKH(hipMemcpyAsync(c->hbuf_host + off, c->hbuf, count * sizeof(double), hipMemcpyDeviceToHost,
                     c->stream));
  return ISIRA_OK;
}

// Host-to-device copy of a small host array through the pinned ring, so that the copy is
// queued on the stream like a kernel instead of stalling the host; the ring is reused only
// after the stream has drained.
int upload(isira_ctx* c, void* dst, const void* src, size_t bytes) {
  if (bytes > kUploadRing) {
    CKH(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    return stream_sync(c);
  }
  if (c->up_off + bytes > kUploadRing) {
    int rc = stream_sync(c);
    if (rc) return rc;
  }
  unsigned char* h = c->up_host + c->up_off;
  std::memcpy(h, src, bytes);
  CKH(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, c->stream));
  c->up_off += (bytes + 255) & ~(size_t)255;
  return ISIRA_OK;
}

// G^{-1} for G = I + delta C (SPD, c x c) by Cholesky; column-major output.
bool spd_inverse(int c, const std::vector<double>& G, std::vector<double>& Ginv) {
  std::vector<double> L((size_t)c * c, 0.0);
  for (int j = 0; j < c; ++j) {
    double s = G[j + (size_t)j * c];
    for (int t = 0; t < j; ++t) s -= L[j + (size_t)t * c] * L[j + (size_t)t * c];
    if (!(s > 0.0)) return false;
    const double ljj = std::sqrt(s);
    L[j + (size_t)j * c] = ljj;
    for (int i = j + 1; i < c; ++i) {
      double v = G[i + (size_t)j * c];
      for (int t = 0; t < j; ++t) v -= L[i + (size_t)t * c] * L[j + (size_t)t * c];
      L[i + (size_t)j * c] = v / ljj;
    }
  }
  Ginv.assign((size_t)c * c, 0.0);
  for (int col = 0; col < c; ++col) {
    std::vector<double> y(c, 0.0);
    for (int i = 0; i < c; ++i) {  // L y = e_col
      double v = (i == col) ? 1.0 : 0.0;
      for (int t = 0; t < i; ++t) v -= L[i + (size_t)t * c] * y[t];
      y[i] = v / L[i + (size_t)i * c];
    }
    for (int i = c - 1; i >= 0; --i) {  // L^T x = y
      double v = y[i];
      for (int t = i + 1; t < c; ++t) v -= L[t + (size_t)i * c] * Ginv[t + (size_t)col * c];
      Ginv[i + (size_t)col * c] = v / L[i + (size_t)i * c];
    }
  }
  return true;
}

// Inner-solve configuration of one solve.
struct InnerCfg {
  int prec;     // ISIRA_FP64 / ISIRA_FP32
  int precond;  // ISIRA_PC_JACOBI / ISIRA_PC_LEARNED / ISIRA_PC_MULTILEVEL
  double sigma, delta, rtol;
  int trim;     // internal index
  int maxit, check_every;
  int first_batch = 0;  // iterations queued with the set-up (0: check_every)
  bool rank_one = true;  // the (sigma/n) 1-hat 1-hat^T term of eq. (2.15) in the operator
  int solver = ISIRA_SOLVER_PCG;
};

// Solve the trimmed shifted deflated system (2.15) for right-hand side r64 (internal order,
// FP64) with c deflation columns already in Vin/Y and Ginv.  The mean removed from r64 is
// `mean`, or (when mean_sum is given) the device value *mean_sum / n.  inner_pcg_start only
// queues the set-up and the first batch of iterations; inner_pcg_finish waits and queues
// further batches until the device-side test has stopped the iteration.  The solution
// (still trimmed, inner precision) is left in x32/x64.
template <typename T>
struct PcgBufs {
  T *x, *r, *p, *q, *dinv, *y, *wa, *wb;
  const T *V, *Y;
};
template <typename T>
PcgBufs<T> pcg_bufs(isira_ctx* c) {
  if constexpr (sizeof(T) == 8) {
    return PcgBufs<T>{c->x64, c->ri64, c->p64, c->q64, c->dinv64, c->y64, c->wa64, c->wb64,
                      c->Vin64, c->Y64};
  } else {
    return PcgBufs<T>{c->x32, c->ri32, c->p32, c->q32, c->dinv32, c->y32, c->wa32, c->wb32,
                      c->Vin32, c->Y32};
  }
}

// Preconditioned MINRES iterations (Jacobi + eq. (3.5) preconditioner, which stays SPD for
// any shift below the minimum degree).  Buffers: x; the Lanczos vectors v_j, v_{j-1} in r and
// y (they swap roles every iteration); z (normalized preconditioned vector) in p; the
// directions w_j, w_{j-1} in wa and wb (swapping); the product in q.  Iteration j (from 1)
// has parity (j - 1) & 1; the first call (init) sets up v_1 = rhs, gamma_1 and z_1.
template <typename T>
void minres_batch(isira_ctx* c, const InnerCfg& cfg, int nc, int iters, int init, int j0) {
  const int n = (int)c->n;
  const PcgBufs<T> b = pcg_bufs<T>(c);
  hipStream_t s = c->stream;
  const int vm = sizeof(T) == 8 ? valmode64(c) : valmode32(c);
  T* vb[2] = {b.r, b.y};
  T* wb[2] = {b.wa, b.wb};
  const double sig_over_n = cfg.rank_one ? cfg.sigma / (double)n : 0.0;
  SpmvArgs<T> a{};
  a.rp = c->rp;
  a.col = c->col;
  a.vals = sizeof(T) == 8 ? (const void*)c->w64 : (const void*)c->w32;
  a.x = b.p;
  a.y = b.q;
  a.diag = sizeof(T) == 8 ? (const T*)c->deg : (const T*)c->deg32;
  a.n = n;
  a.trim = cfg.trim;
  a.sigma = cfg.sigma;
  a.ldv = c->ld;
  a.delta = cfg.delta;
  a.red = 4;  // delta_j = z^T K-hat z, the deflation and rank-one terms folded in
  a.st = c->st;
  a.check_done = 1;
  a.fold_c = nc;
  a.fold_nblk = stream_grid(n);
  a.fold_partials = c->rb.partials;
  a.fold_sig_over_n = sig_over_n;
  int it = 0;
  if (init) {
    launch_minres_a<T>(n, b.q, vb[0], vb[1], b.dinv, b.V, c->ld, nc, c->Ginv, cfg.delta,
                       cfg.trim, sig_over_n, 1, c->st, c->rb, s);
    launch_minres_b<T>(n, b.p, wb[1], wb[0], b.x, vb[0], vb[1], b.dinv, b.V, c->ld, nc,
                       cfg.delta, 1, 0, c->st, c->rb, s);
  }
  for (; it < iters; ++it) {
    const int j = j0 + it;  // iteration number, from 1
    const int par = (j - 1) & 1;
    launch_spmv<T>(c->plan, vm, a, c->rb, s);
    launch_minres_a<T>(n, b.q, vb[par], vb[1 - par], b.dinv, b.V, c->ld, nc, c->Ginv,
                       cfg.delta, cfg.trim, sig_over_n, 0, c->st, c->rb, s);
    launch_minres_b<T>(n, b.p, wb[1 - par], wb[par], b.x, vb[1 - par], nullptr, b.dinv, b.V,
                       c->ld, nc, cfg.delta, 0, j, c->st, c->rb, s);
  }
}

template <typename T>
void pcg_batch(isira_ctx* c, const InnerCfg& cfg, int nc, int iters, int init) {
  const int n = (int)c->n;
  const PcgBufs<T> b = pcg_bufs<T>(c);
  hipStream_t s = c->stream;
  const bool learned = cfg.precond == ISIRA_PC_LEARNED;
  const bool multilevel = cfg.precond == ISIRA_PC_MULTILEVEL;
  const int vm = sizeof(T) == 8 ? valmode64(c) : valmode32(c);
  SpmvArgs<T> a{};
  a.rp = c->rp;
  a.col = c->col;
  a.vals = sizeof(T) == 8 ? (const void*)c->w64 : (const void*)c->w32;
  a.x = b.p;
  a.y = b.q;
  a.diag = sizeof(T) == 8 ? (const T*)c->deg : (const T*)c->deg32;
  a.n = n;
  a.trim = cfg.trim;
  a.sigma = cfg.sigma;
  // the deflation term delta V-hat (V-hat^T p) and the rank-one term (sigma/n) 1-hat 1-hat^T p
  // of the operator are applied by the residual update (which reads V-hat anyway) and folded
  // into p^T q by the product's finishing dispatch, which also reduces the p-update's sums
  a.sig_over_n = 0.0;
  a.V = nullptr;
  a.ldv = c->ld;
  a.c = 0;
  a.tvec = nullptr;
  a.delta = cfg.delta;
  a.red = 1;
  a.st = c->st;
  a.check_done = 1;
  a.fold_c = nc;
  a.fold_nblk = stream_grid(n);
  a.fold_partials = c->rb.partials;
  const double sig_over_n = cfg.rank_one ? cfg.sigma / (double)n : 0.0;
  a.fold_sig_over_n = sig_over_n;
  // one iteration: [product] then the residual update and the preconditioned direction;
  // the first call (init) has no product and starts from x = 0, r = rhs
  for (int it = 0; it < iters; ++it) {
    const int first = init && it == 0;
    if (!first) launch_spmv<T>(c->plan, vm, a, c->rb, s);
    if (learned && c->spw.pruned) {
      // pruned M: the residual update, then u = M r with the dots of the Jacobi form and its
      // finishing dispatch (eq. (3.5)), then z = u - delta Y g and the new direction
      launch_pcg_update1_plain<T>(n, b.x, b.r, b.p, b.q, b.V, c->ld, nc, cfg.delta, cfg.trim,
                                  sig_over_n, first, c->st, c->rb, s, /*with_fin=*/false);
      spai::sparse_step<T>(c->spw, n, b.r, b.y, b.V, c->ld, nc, c->Ginv, cfg.delta, first, c->st,
                           c->rb, s);
      launch_pcg_update2_learned<T>(n, b.y, b.p, b.Y, c->ld, nc, b.V, cfg.delta, first, c->st,
                                    c->rb, s);
    } else if (learned) {
      // y = M r with the dots V-hat^T y and r^T y, then eq. (3.5)
      launch_pcg_update1_plain<T>(n, b.x, b.r, b.p, b.q, b.V, c->ld, nc, cfg.delta, cfg.trim,
                                  sig_over_n, first, c->st, c->rb, s);
      spai::apply<T>(c->spw, c->plan, c->rp, c->col, b.r, b.y, n, cfg.trim, b.V, c->ld, nc,
                     c->st, c->rb, s);
      launch_spai_finish_rho(nc, c->Ginv, cfg.delta, first, c->st, s);
      launch_pcg_update2_learned<T>(n, b.y, b.p, b.Y, c->ld, nc, b.V, cfg.delta, first, c->st,
                                    c->rb, s);
    } else if (multilevel) {
      // y = cycle(r) with the dots V-hat^T y and r^T y, then eq. (3.5)
      launch_pcg_update1_plain<T>(n, b.x, b.r, b.p, b.q, b.V, c->ld, nc, cfg.delta, cfg.trim,
                                  sig_over_n, first, c->st, c->rb, s);
      ml::apply<T>(c->ml, b.r, b.y, 1, c->st, c->rb, s, /*in_place=*/true);
      launch_multidot<T>(n, b.V, c->ld, nc, b.r, c->ld, 1, b.y, nullptr, 0, 0, c->st->t2, c->rb, s,
                         &c->st->done);
      launch_spai_finish_rho(nc, c->Ginv, cfg.delta, first, c->st, s);
      launch_pcg_update2_learned<T>(n, b.y, b.p, b.Y, c->ld, nc, b.V, cfg.delta, first, c->st,
                                    c->rb, s);
    } else {
      launch_pcg_update1<T>(n, b.x, b.r, b.p, b.q, b.dinv, b.V, c->ld, nc, c->Ginv, cfg.delta,
                            cfg.trim, sig_over_n, first, c->st, c->rb, s);
      launch_pcg_update2<T>(n, b.r, b.p, b.dinv, b.V, c->ld, nc, cfg.delta, first, c->st,
                            c->rb, s);
    }
  }
}

template <typename T>
void inner_pcg_start(isira_ctx* c, const InnerCfg& cfg, const double* r64, double mean,
                     const double* mean_sum, int nc) {
  const int n = (int)c->n;
  const PcgBufs<T> b = pcg_bufs<T>(c);
  launch_pcg_reset(c->st, cfg.rtol * cfg.rtol, cfg.maxit, c->stream);
  launch_rhs_prep<T>(n, r64, mean, mean_sum, 1.0 / (double)n, cfg.trim, b.r, b.x, c->stream);
  const int first = cfg.first_batch > 0 ? cfg.first_batch : cfg.check_every;
  if (cfg.solver == ISIRA_SOLVER_MINRES) {
    minres_batch<T>(c, cfg, nc, first, 1, 1);
    c->minres_next = 1 + first;
  } else {
    pcg_batch<T>(c, cfg, nc, 1 + first, 1);
  }
}

// `synced`: st_host already holds the state after the queued batch (no wait needed first).
template <typename T>
int inner_pcg_finish(isira_ctx* c, const InnerCfg& cfg, int nc, bool synced, int* iters,
                     int* status, double* relres) {
  int rc;
  for (;;) {
    if (!synced && (rc = sync_state(c))) return rc;
    synced = false;
    if (c->st_host->done) break;
    if (cfg.solver == ISIRA_SOLVER_MINRES) {
      minres_batch<T>(c, cfg, nc, cfg.check_every, 0, c->minres_next);
      c->minres_next += cfg.check_every;
    } else {
      pcg_batch<T>(c, cfg, nc, cfg.check_every, 0);
    }
  }
  *iters = c->st_host->it;
  *status = c->st_host->status;
  *relres = c->st_host->rr0 > 0 ? std::sqrt(c->st_host->rr / c->st_host->rr0) : 0.0;
  return ISIRA_OK;
}

template <typename T>
int inner_pcg(isira_ctx* c, const InnerCfg& cfg, const double* r64, double mean, int nc,
              int* iters, int* status, double* relres) {
  inner_pcg_start<T>(c, cfg, r64, mean, nullptr, nc);
  return inner_pcg_finish<T>(c, cfg, nc, false, iters, status, relres);
}

// Classical Gram-Schmidt twice against [U(:,0:nu) Vout(:,0:nv) 1/sqrt(n)] in place on z.
// With `selective`, the second pass runs only when the first one kept less than 1/sqrt(2)
// of the norm (the test of Daniel, Gragg, Kaufman and Stewart, decided on the device, so
// nothing waits for it): otherwise the first pass is already orthogonal to working
// precision and the second pass's dispatches return at once.
// cgs2_queue only queues the work: ||z||^2 before the first pass goes to
// hbuf_host[kMaxCols + nc + 1] and at the end to st->red[2], both valid after the next sync.
int cgs2_queue(isira_ctx* c, const double* U, int nu, const double* V, int nv, double* z,
               bool selective = false) {
  const int n = (int)c->n;
  hipStream_t s = c->stream;
  const int nc = nu + nv;
  launch_multidot<double>(n, U, c->ld, nu, V, c->ld, nv, z, nullptr, 1, 1, c->hbuf, c->rb, s);
  int rc;
  if ((rc = read_h(c, nc + 2, kMaxCols))) return rc;
  launch_gemv_sub(n, U, c->ld, nu, V, c->ld, nv, c->hbuf, 1, z, selective ? 1 : 0, c->st, c->rb, s);
  const int32_t* skip = nullptr;
  if (selective) {
    launch_dgks_decide(c->hbuf + nc + 1, c->st, s);
    skip = &c->st->cgs_skip;
  }
  // the second pass overwrites hbuf only after the copy and the test above (stream order)
  launch_multidot<double>(n, U, c->ld, nu, V, c->ld, nv, z, nullptr, 1, 0, c->hbuf, c->rb, s, skip);
  launch_gemv_sub(n, U, c->ld, nu, V, c->ld, nv, c->hbuf, 1, z, 1, c->st, c->rb, s, skip);
  return ISIRA_OK;
}

// norms[0] = ||z|| before the second pass, norms[1] = after (after sync_state).
void cgs2_norms(const isira_ctx* c, int nc, double* norms) {
  norms[0] = std::sqrt(std::max(0.0, c->hbuf_host[kMaxCols + nc + 1]));
  norms[1] = std::sqrt(std::max(0.0, c->st_host->red[2]));
}

int cgs2(isira_ctx* c, const double* U, int nu, const double* V, int nv, double* z,
         double* norms) {
  int rc;
  if ((rc = cgs2_queue(c, U, nu, V, nv, z))) return rc;
  if ((rc = sync_state(c))) return rc;
  cgs2_norms(c, nu + nv, norms);
  return ISIRA_OK;
}

}  // namespace

// ------------------------------------------------------------------------------ solve

extern "C" int isira_solve(isira_ctx* c, int32_t k, double sigma, double tol,
                           const isira_options* optp, double* evals, double* evecs,
                           double* resid, isira_stats* stats) {
  return guarded([&]() -> int {
    if (!c) return fail(ISIRA_E_ARG, "NULL context");
    isira_options opt;
    if (optp) opt = *optp; else isira_default_options(&opt);
    const int n = (int)c->n;
    const int q = opt.q > 0 ? opt.q : k + 10;
    const int m = opt.m > 0 ? opt.m : 2 * q;
    const int k0 = opt.k0 > 0 ? opt.k0 : 4;
    if (k < 1 || k > ISIRA_MAX_K || k > n - 2) return fail(ISIRA_E_ARG, "need 1 <= k <= min(64, n-2)");
    if (!(tol > 0.0)) return fail(ISIRA_E_ARG, "tol must be > 0");
    if (!(sigma >= 0.0) || !(sigma < c->min_deg)) return fail(ISIRA_E_ARG, "need 0 <= sigma < min degree");
    if (q < k || m <= q || m > ISIRA_MAX_BASIS || m + k > n - 1 || k0 >= m || k0 > n - 2)
      return fail(ISIRA_E_ARG, "need k <= q < m <= 192, m + k <= n - 1 and k0 < m");
    if (!evals || !evecs || !resid) return fail(ISIRA_E_ARG, "NULL output");
    if (opt.inner_prec != ISIRA_FP64 && opt.inner_prec != ISIRA_FP32) return fail(ISIRA_E_ARG, "bad inner_prec");
    if (opt.precond == ISIRA_PC_LEARNED && (!c->has_learned)) return fail(ISIRA_E_PRECOND, "no learned preconditioner installed");
    if (opt.precond != ISIRA_PC_JACOBI && opt.precond != ISIRA_PC_LEARNED && opt.precond != ISIRA_PC_MULTILEVEL)
      return fail(ISIRA_E_ARG, "bad precond");
    int trim = c->trim_default;
    if (opt.trim_index >= 0) {
      if (opt.trim_index >= n) return fail(ISIRA_E_ARG, "trim_index out of range");
      trim = c->iperm[opt.trim_index];
    }
    if (opt.precond == ISIRA_PC_LEARNED && (c->spai_trim != trim || c->spai_sigma != sigma))
      return fail(ISIRA_E_PRECOND, "learned preconditioner was installed for another sigma or trim index");
    if (opt.shift_mode != ISIRA_SHIFT_FIXED && opt.shift_mode != ISIRA_SHIFT_MOVING)
      return fail(ISIRA_E_ARG, "bad shift_mode");
    const bool moving = opt.shift_mode == ISIRA_SHIFT_MOVING;
    if (moving && opt.precond == ISIRA_PC_LEARNED)
      return fail(ISIRA_E_PRECOND, "the learned preconditioner is built for one shift; it cannot follow a moving shift");
    if (opt.precond == ISIRA_PC_MULTILEVEL && (!c->ml.ready || c->ml.trim != trim))
      return fail(ISIRA_E_PRECOND, "no multilevel hierarchy set up for this trim index");
    if (moving && opt.precond == ISIRA_PC_MULTILEVEL)
      return fail(ISIRA_E_PRECOND, "the moving shift runs MINRES with the Jacobi preconditioner only");
    const double delta = opt.delta > 0 ? opt.delta : 2.0 * c->max_deg;
    int rc = ensure_workspace(c, m, k);
    if (rc) return rc;
    hipStream_t s = c->stream;
    const int ld = c->ld;
    isira_stats S{};
    const double t_start = now_ms();
    // events around the Ritz residual kernel: its own time goes to ms_residual, the rest of the
    // wait that follows it (the first inner batch queued behind it) to ms_inner
    struct EventPair {
      hipEvent_t a = nullptr, b = nullptr;
      ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
      }
    } ev;
    CKH(hipEventCreate(&ev.a));
    CKH(hipEventCreate(&ev.b));
    InnerCfg cfg;
    cfg.prec = opt.inner_prec;
    cfg.precond = opt.precond;
    cfg.sigma = sigma;
    cfg.delta = delta;
    cfg.rtol = opt.inner_rtol > 0 ? opt.inner_rtol : 1e-1;
    cfg.trim = trim;
    cfg.maxit = opt.max_inner > 0 ? opt.max_inner : 1000;
    cfg.check_every = opt.check_every > 0 ? opt.check_every : 8;
    cfg.rank_one = opt.drop_rank_one == 0;
    // a moving shift can make the trimmed system indefinite (Thm 2.8), so it is solved by MINRES
    cfg.solver = moving ? ISIRA_SOLVER_MINRES : ISIRA_SOLVER_PCG;
    const double sigma_cap = 0.5 * c->min_deg;  // keeps diag(d - sigma) positive
    const int max_outer = opt.max_outer > 0 ? opt.max_outer : 20000;
    // Jacobi inverse diagonal (Remark 3.2) in both precisions
    launch_dinv<double>(n, c->deg, sigma, trim, c->dinv64, s);
    launch_dinv<float>(n, c->deg, sigma, trim, c->dinv32, s);
    uint64_t draws = 0;
    int capture_count = 0;

    // ---- start block: column means removed, orthonormalized (CGS2 against 1 and previous)
    if (opt.u0) {
      std::vector<double> col(n);
      for (int j = 0; j < k0; ++j) {
        CKH(hipMemcpyAsync(c->tmp64, opt.u0 + (size_t)j * n, (size_t)n * 8, hipMemcpyHostToDevice, s));
        launch_gather<double, double>(n, c->tmp64, c->d_perm, c->z64, s);
        // z64[new] = u0[perm[new]]
        double nrm[2];
        if ((rc = cgs2(c, c->U, j, c->Vout, 0, c->z64, nrm))) return rc;
        while (!(nrm[1] > 1e-10 * nrm[0] && nrm[1] > 0.0)) {
          S.breakdowns++;
          launch_fill_replacement(n, opt.seed, draws++, c->d_perm, c->z64, s);
          if ((rc = cgs2(c, c->U, j, c->Vout, 0, c->z64, nrm))) return rc;
        }
        launch_scale(n, c->z64, 1.0 / nrm[1], c->U + (size_t)j * ld, s);
      }
    } else {
      for (int j = 0; j < k0; ++j) {
        double nrm[2];
        do {
          launch_fill_replacement(n, opt.seed, draws++, c->d_perm, c->z64, s);
          if ((rc = cgs2(c, c->U, j, c->Vout, 0, c->z64, nrm))) return rc;
        } while (!(nrm[1] > 1e-10 * nrm[0] && nrm[1] > 0.0));
        launch_scale(n, c->z64, 1.0 / nrm[1], c->U + (size_t)j * ld, s);
      }
    }
    int kk = k0;  // current basis size
    std::vector<double> H((size_t)m * m, 0.0);  // column-major, leading dimension m
    for (int j = 0; j < kk; ++j) {
      spmv64(c, c->U + (size_t)j * ld, c->W + (size_t)j * ld, nullptr, 0, nullptr, 0.0, 0, 0.0);
      S.spmv_total++;
    }
    for (int j = 0; j < kk; ++j) {
      launch_multidot<double>(n, c->U, ld, kk, nullptr, ld, 0, c->W + (size_t)j * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
      if ((rc = read_h(c, kk))) return rc;
      SYNC_OR_RETURN(c);
      for (int i = 0; i < kk; ++i) H[i + (size_t)j * m] = c->hbuf_host[i];
    }
    for (int i = 0; i < kk; ++i)
      for (int j = 0; j < i; ++j) {
        const double v = 0.5 * (H[i + (size_t)j * m] + H[j + (size_t)i * m]);
        H[i + (size_t)j * m] = H[j + (size_t)i * m] = v;
      }

    int nconv = 0;
    std::vector<double> Hk, theta, Sm, Spack;
    std::vector<double> Cmat;  // c x c Gram V-hat^T M^-1 V-hat (column-major, ld kMaxC)
    Cmat.assign((size_t)kMaxC * kMaxC, 0.0);
    int outer = 0;
    int its_pair = 0;
    int64_t inner_pair = 0;
    bool not_conv = false;

    auto refresh_smw = [&](int cnew) -> int {
      // new column cnew of C = V-hat^T P0 V-hat (P0 = M^-1 Jacobi or learned M); then G^-1
      const int cc = cnew + 1;
      if (cfg.precond == ISIRA_PC_MULTILEVEL) {
        if (cfg.prec == ISIRA_FP64) {
          ml::apply<double>(c->ml, c->Vin64 + (size_t)cnew * ld, c->Y64 + (size_t)cnew * ld, 0, c->st, c->rb, s);
          launch_multidot<double>(n, c->Vin64, ld, cc, nullptr, ld, 0, c->Y64 + (size_t)cnew * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
        } else {
          ml::apply<float>(c->ml, c->Vin32 + (size_t)cnew * ld, c->Y32 + (size_t)cnew * ld, 0, c->st, c->rb, s);
          launch_multidot<float>(n, c->Vin32, ld, cc, nullptr, ld, 0, c->Y32 + (size_t)cnew * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
        }
      } else if (cfg.precond == ISIRA_PC_LEARNED) {
        if (cfg.prec == ISIRA_FP64) {
          spai::apply_plain<double>(c->spw, c->plan, c->rp, c->col,
                                    c->Vin64 + (size_t)cnew * ld, c->Y64 + (size_t)cnew * ld, n, trim, s);
          launch_multidot<double>(n, c->Vin64, ld, cc, nullptr, ld, 0, c->Y64 + (size_t)cnew * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
        } else {
          spai::apply_plain<float>(c->spw, c->plan, c->rp, c->col,
                                   c->Vin32 + (size_t)cnew * ld, c->Y32 + (size_t)cnew * ld, n, trim, s);
          launch_multidot<float>(n, c->Vin32, ld, cc, nullptr, ld, 0, c->Y32 + (size_t)cnew * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
        }
      } else if (cfg.prec == ISIRA_FP64) {
        launch_multidot<double>(n, c->Vin64, ld, cc, nullptr, ld, 0, c->Vin64 + (size_t)cnew * ld, c->dinv64, 0, 0, c->hbuf, c->rb, s);
      } else {
        launch_multidot<float>(n, c->Vin32, ld, cc, nullptr, ld, 0, c->Vin32 + (size_t)cnew * ld, c->dinv32, 0, 0, c->hbuf, c->rb, s);
      }
      int r2 = read_h(c, cc);
      if (r2) return r2;
      SYNC_OR_RETURN(c);
      for (int i = 0; i < cc; ++i) {
        Cmat[i + (size_t)cnew * kMaxC] = c->hbuf_host[i];
        Cmat[cnew + (size_t)i * kMaxC] = c->hbuf_host[i];
      }
      std::vector<double> G((size_t)cc * cc), Gi;
      for (int j = 0; j < cc; ++j)
        for (int i = 0; i < cc; ++i)
          G[i + (size_t)j * cc] = (i == j ? 1.0 : 0.0) + delta * Cmat[i + (size_t)j * kMaxC];
      if (!spd_inverse(cc, G, Gi)) return fail(ISIRA_E_PRECOND, "SMW capacitance matrix not positive definite");
      return upload(c, c->Ginv, Gi.data(), Gi.size() * 8);
    };

    auto expand_with = [&](double* z) -> int {
      // orthonormalize z against [U V 1] and append u, w = (L + delta V V^T) u and the new
      // column of H.  Everything is queued behind one wait; on a CGS2 breakdown (rare) the
      // queued results are discarded and a replacement vector is expanded instead.
      double nrm[2];
      int r2;
      double t0 = now_ms();
      double* u = c->U + (size_t)kk * ld;
      double* w = c->W + (size_t)kk * ld;
      for (;;) {
        if ((r2 = cgs2_queue(c, c->U, kk, c->Vout, nconv, z, /*selective=*/true))) return r2;
        launch_scale_dev(n, z, c->st->red + 2, u, s);
        if (nconv > 0)
          launch_multidot<double>(n, c->Vout, ld, nconv, nullptr, ld, 0, u, nullptr, 0, 0, c->hbuf, c->rb, s);
        spmv64(c, u, w, c->Vout, nconv, c->hbuf, delta, 0, 0.0);
        launch_multidot<double>(n, c->U, ld, kk + 1, nullptr, ld, 0, w, nullptr, 0, 0, c->hbuf, c->rb, s);
        if ((r2 = read_h(c, kk + 1))) return r2;
        if ((r2 = sync_state(c))) return r2;
        S.spmv_total++;
        cgs2_norms(c, kk + nconv, nrm);
        if (nrm[1] > 1e-10 * nrm[0] && nrm[1] > 0.0) break;
        S.breakdowns++;
        launch_fill_replacement(n, opt.seed, draws++, c->d_perm, z, s);
      }
      for (int i = 0; i <= kk; ++i) {
        H[i + (size_t)kk * m] = c->hbuf_host[i];
        H[kk + (size_t)i * m] = c->hbuf_host[i];
      }
      kk += 1;
      S.ms_ortho += now_ms() - t0;
      return ISIRA_OK;
    };

    int recent_its[4];
    std::fill(recent_its, recent_its + 4, cfg.check_every);
    int n_inner = 0;
    auto start_inner = [&]() {
      // the right-hand side is the Ritz residual in r64; its sum is st->red[1]
      if (cfg.prec == ISIRA_FP64) {
        inner_pcg_start<double>(c, cfg, c->r64, 0.0, c->st->red + 1, nconv);
      } else {
        inner_pcg_start<float>(c, cfg, c->r64, 0.0, c->st->red + 1, nconv);
      }
    };

    while (nconv < k) {
      if (outer >= max_outer) {
        not_conv = true;
        break;
      }
      outer++;
      its_pair++;
      S.basis_cols_total += kk + nconv;
      // ---- Rayleigh-Ritz: the eigenvalues of H (ascending) and the eigenvector of the
      // smallest; all eigenvectors only when a pair is locked or the basis restarts
      double t0 = now_ms();
      Hk.assign((size_t)kk * kk, 0.0);
      for (int j = 0; j < kk; ++j)
        for (int i = 0; i < kk; ++i) Hk[i + (size_t)j * kk] = H[i + (size_t)j * m];
      theta.assign(kk, 0.0);
      Sm.assign((size_t)kk * kk, 0.0);
      if ((rc = isira_symeig_lowest(kk, Hk.data(), theta.data(), Sm.data())))
        return fail(rc, "Rayleigh-Ritz eigensolver did not converge");
      bool all_vectors = false;
      auto rayleigh_ritz_all = [&]() -> int {
        if (all_vectors) return ISIRA_OK;
        const double t1 = now_ms();
        const int r2 = isira_symeig(kk, Hk.data(), theta.data(), Sm.data());
        S.ms_rr_host += now_ms() - t1;
        if (r2) return fail(r2, "Rayleigh-Ritz eigensolver did not converge");
        all_vectors = true;
        return ISIRA_OK;
      };
      S.ms_rr_host += now_ms() - t0;
      // ---- Ritz residual r = W s1 - theta1 U s1.  The inner solve for it is queued at once,
      // behind the same wait: when the pair turns out converged that work is simply dropped.
      t0 = now_ms();
      if ((rc = upload(c, c->svec, Sm.data(), kk * 8))) return rc;
      CKH(hipEventRecord(ev.a, s));
      launch_ritz_residual(n, c->U, c->W, ld, kk, c->svec, theta[0], c->r64, c->st, c->rb, s);
      CKH(hipEventRecord(ev.b, s));
      start_inner();
      if ((rc = sync_state(c))) return rc;
      const double rn = std::sqrt(std::max(0.0, c->st_host->red[0]));
      {
        float ms_res = 0.0f;
        CKH(hipEventElapsedTime(&ms_res, ev.a, ev.b));
        const double window = now_ms() - t0;
        S.ms_residual += std::min((double)ms_res, window);
        S.ms_inner += std::max(0.0, window - (double)ms_res);
      }
      if (rn < tol) {
        // the lock purges with S(:, 2:kk), so the locked vector is taken from the same full
        // decomposition; its fresh FP64 residual decides
        if ((rc = rayleigh_ritz_all())) return rc;
        if ((rc = upload(c, c->svec, Sm.data(), kk * 8))) return rc;
        double* v = c->Vout + (size_t)nconv * ld;
        launch_ritz_vector(n, c->U, ld, kk, c->svec, v, s);
        spmv64(c, v, c->tmp64, nullptr, 0, nullptr, 0.0, 2, theta[0]);
        S.spmv_total++;
        if ((rc = sync_state(c))) return rc;
        const double true_r = std::sqrt(std::max(0.0, c->st_host->red[0]));
        if (true_r < tol) {
          evals[nconv] = theta[0];
          resid[nconv] = true_r;
          if (nconv < ISIRA_STATS_MAX) {
            S.outer_per_pair[nconv] = its_pair;
            S.inner_per_pair[nconv] = (int32_t)inner_pair;
          }
          if (opt.verbose)
            fprintf(stderr, "isira: pair %d lambda=%.15g resid=%.3e outer=%d inner=%lld\n", nconv,
                    theta[0], true_r, its_pair, (long long)inner_pair);
          its_pair = 0;
          inner_pair = 0;
          launch_masked_copy<double>(n, v, trim, c->Vin64 + (size_t)nconv * ld, s);
          launch_masked_copy<float>(n, v, trim, c->Vin32 + (size_t)nconv * ld, s);
          // eigenvector purging: U <- U S(:, 2:k), W <- W S(:, 2:k), H <- diag(theta_2..)
          t0 = now_ms();
          if (kk > 1) {
            // S(:, 2:kk) row by row for the tall-skinny product
            Spack.assign((size_t)kk * (kk - 1), 0.0);
            for (int j = 1; j < kk; ++j)
              for (int i = 0; i < kk; ++i) Spack[(size_t)i * (kk - 1) + (j - 1)] = Sm[i + (size_t)j * kk];
            if ((rc = upload(c, c->Sdev, Spack.data(), Spack.size() * 8))) return rc;
            launch_tsgemm_inplace(n, c->U, ld, kk, c->Sdev, kk - 1, s);
            launch_tsgemm_inplace(n, c->W, ld, kk, c->Sdev, kk - 1, s);
          }
          std::fill(H.begin(), H.end(), 0.0);
          for (int j = 1; j < kk; ++j) H[(j - 1) + (size_t)(j - 1) * m] = theta[j];
          kk -= 1;
          S.ms_restart += now_ms() - t0;
          nconv += 1;
          if (nconv < k) {
            // the purge step's moving shift: sigma <- theta_2 (capped); the Jacobi diagonal
            // and the whole SMW capacitance matrix then change with it
            const double sigma_new = (moving && kk >= 1) ? std::min(theta[1], sigma_cap) : cfg.sigma;
            if (sigma_new != cfg.sigma) {
              cfg.sigma = sigma_new;
              launch_dinv<double>(n, c->deg, cfg.sigma, trim, c->dinv64, s);
              launch_dinv<float>(n, c->deg, cfg.sigma, trim, c->dinv32, s);
              for (int j = 0; j < nconv; ++j)
                if ((rc = refresh_smw(j))) return rc;
            } else if ((rc = refresh_smw(nconv - 1))) {
              return rc;
            }
            if (kk == 0) {  // empty basis: start again from a replacement vector
              launch_fill_replacement(n, opt.seed, draws++, c->d_perm, c->z64, s);
              if ((rc = expand_with(c->z64))) return rc;
            }
          }
          continue;
        }
        // the carried W has drifted: recompute W = (L + delta V V^T) U and H = U^T W
        S.refreshes++;
        for (int j = 0; j < kk; ++j) {
          if (nconv > 0)
            launch_multidot<double>(n, c->Vout, ld, nconv, nullptr, ld, 0, c->U + (size_t)j * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
          spmv64(c, c->U + (size_t)j * ld, c->W + (size_t)j * ld, c->Vout, nconv, c->hbuf, delta, 0, 0.0);
          S.spmv_total++;
        }
        for (int j = 0; j < kk; ++j) {
          launch_multidot<double>(n, c->U, ld, kk, nullptr, ld, 0, c->W + (size_t)j * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
          if ((rc = read_h(c, kk))) return rc;
          if ((rc = stream_sync(c))) return rc;
          for (int i = 0; i < kk; ++i) H[i + (size_t)j * m] = c->hbuf_host[i];
        }
        for (int i = 0; i < kk; ++i)
          for (int j = 0; j < i; ++j) {
            const double v2 = 0.5 * (H[i + (size_t)j * m] + H[j + (size_t)i * m]);
            H[i + (size_t)j * m] = H[j + (size_t)i * m] = v2;
          }
        continue;
      }
      if (kk == m) {
        // subspace restart: U <- U S(:, 1:q), W <- W S(:, 1:q), H <- diag(theta_1..theta_q)
        // (the queued inner solve reads neither U nor W)
        if ((rc = rayleigh_ritz_all())) return rc;
        t0 = now_ms();
        S.restarts++;
        Spack.assign((size_t)kk * q, 0.0);
        for (int j = 0; j < q; ++j)
          for (int i = 0; i < kk; ++i) Spack[(size_t)i * q + j] = Sm[i + (size_t)j * kk];
        if ((rc = upload(c, c->Sdev, Spack.data(), Spack.size() * 8))) return rc;
        launch_tsgemm_inplace(n, c->U, ld, kk, c->Sdev, q, s);
        launch_tsgemm_inplace(n, c->W, ld, kk, c->Sdev, q, s);
        std::fill(H.begin(), H.end(), 0.0);
        for (int j = 0; j < q; ++j) H[j + (size_t)j * m] = theta[j];
        kk = q;
        S.ms_restart += now_ms() - t0;
      }
      // ---- subspace expansion: trimmed deflated inner solve, enlargement (2.5)
      t0 = now_ms();
      int its = 0, status = 0;
      double rel = 0.0;
      if (cfg.prec == ISIRA_FP64) {
        rc = inner_pcg_finish<double>(c, cfg, nconv, true, &its, &status, &rel);
      } else {
        rc = inner_pcg_finish<float>(c, cfg, nconv, true, &its, &status, &rel);
      }
      if (rc) return rc;
      // the next inner solve queues as many iterations with its set-up as the most any of
      // the last four took: launches past convergence return at once, each round trip
      // to the host for another batch costs a wait
      recent_its[n_inner++ & 3] = its;
      cfg.first_batch = std::max(1, std::min(cfg.check_every,
                                             *std::max_element(recent_its, recent_its + 4)));
      if (status == kPcgBreakdown) S.inner_fallbacks++;
      if (status == kPcgCapped) S.inner_capped++;
      S.inner_total += its;
      S.spmv_total += its;
      inner_pair += its;
      if (cfg.prec == ISIRA_FP64) {
        launch_enlarge<double>(n, c->x64, c->z64, c->st, c->rb, s);
      } else {
        launch_enlarge<float>(n, c->x32, c->z64, c->st, c->rb, s);
      }
      if (opt.capture_r && opt.capture_z && opt.capture_count && capture_count < opt.capture_cap) {
        double* cr = opt.capture_r + (size_t)capture_count * n;
        double* cz = opt.capture_z + (size_t)capture_count * n;
        // z_hat (trimmed entry 0) and r' = (L-hat - sigma I) z_hat: the pair that an
        // approximate inverse of L-hat - sigma I should map onto each other
        const double* zin = c->x64;
        if (cfg.prec != ISIRA_FP64) {
          launch_gather<float, double>(n, c->x32, c->d_iperm, cz, s);
          launch_gather<double, double>(n, cz, c->d_perm, c->y64, s);
          zin = c->y64;
        } else {
          launch_gather<double, double>(n, c->x64, c->d_iperm, cz, s);
        }
        SpmvArgs<double> ca{};
        ca.rp = c->rp; ca.col = c->col; ca.vals = c->w64; ca.x = zin; ca.y = c->tmp64;
        ca.diag = c->deg; ca.n = n; ca.trim = trim; ca.sigma = cfg.sigma;
        launch_spmv<double>(c->plan, valmode64(c), ca, c->rb, s);
        launch_gather<double, double>(n, c->tmp64, c->d_iperm, cr, s);
        capture_count++;
        *opt.capture_count = capture_count;
      }
      S.ms_inner += now_ms() - t0;
      if ((rc = expand_with(c->z64))) return rc;
    }
    // ---- outputs: sign-normalized eigenvectors in caller labels
    for (int j = 0; j < nconv; ++j) {
      double* v = c->Vout + (size_t)j * ld;
      launch_signed_gather(n, v, c->d_perm, c->d_iperm, evecs + (size_t)j * n, c->scal4, c->rb, s);
    }
    SYNC_OR_RETURN(c);
    S.n_converged = nconv;
    S.outer_total = outer;
    S.ms_total = now_ms() - t_start;
    S.trim_index = c->perm[trim];
    S.delta = delta;
    S.sigma_last = cfg.sigma;
    if (stats) *stats = S;
    return not_conv ? ISIRA_NOT_CONVERGED : ISIRA_OK;
  });
}

// ------------------------------------------------------------------------------ operators

extern "C" int isira_laplacian_apply(isira_ctx* c, const double* x, double* y) {
  return guarded([&]() -> int {
    if (!c || !x || !y) return fail(ISIRA_E_ARG, "NULL argument");
    int rc = ensure_workspace(c, std::max(c->ws_m, 2), std::max(c->ws_k, 1));
    if (rc) return rc;
    const int n = (int)c->n;
    launch_gather<double, double>(n, x, c->d_perm, c->x64, c->stream);
    spmv64(c, c->x64, c->y64, nullptr, 0, nullptr, 0.0, 0, 0.0);
    launch_gather<double, double>(n, c->y64, c->d_iperm, y, c->stream);
    SYNC_OR_RETURN(c);
    return ISIRA_OK;
  });
}

extern "C" int isira_laplacian_apply_f32(isira_ctx* c, const float* x, float* y) {
  return guarded([&]() -> int {
    if (!c || !x || !y) return fail(ISIRA_E_ARG, "NULL argument");
    int rc = ensure_workspace(c, std::max(c->ws_m, 2), std::max(c->ws_k, 1));
    if (rc) return rc;
    const int n = (int)c->n;
    launch_gather<float, float>(n, x, c->d_perm, c->x32, c->stream);
    SpmvArgs<float> a{};
    a.rp = c->rp;
    a.col = c->col;
    a.vals = c->w32;
    a.x = c->x32;
    a.y = c->y32;
    a.diag = c->deg32;
    a.n = n;
    a.trim = -1;
    launch_spmv<float>(c->plan, valmode32(c), a, c->rb, c->stream);
    launch_gather<float, float>(n, c->y32, c->d_iperm, y, c->stream);
    SYNC_OR_RETURN(c);
    return ISIRA_OK;
  });
}

extern "C" int isira_time_spmv(isira_ctx* c, int32_t prec, int32_t reps, int32_t cold,
                               double* ms_per) {
  return guarded([&]() -> int {
    if (!c || reps < 1 || !ms_per) return fail(ISIRA_E_ARG, "bad argument");
    int rc = ensure_workspace(c, std::max(c->ws_m, 2), std::max(c->ws_k, 1));
    if (rc) return rc;
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    launch_fill_replacement(n, 7, 0, c->d_perm, c->x64, s);
    launch_gather<double, float>(n, c->x64, c->d_iperm, c->x32, s);  // any FP32 data will do
    // cold: before every timed launch, read and write a buffer of twice the 256 MB memory-side
    // cache, so that no launch finds the graph or x in a cache left warm by the one before
    constexpr size_t kFlush = (size_t)512 << 20;
    double* flush = nullptr;
    if (cold && (rc = dalloc(c->mem, &flush, kFlush / 8))) return rc;
    if (flush) CKH(hipMemsetAsync(flush, 0, kFlush, s));
    hipEvent_t e0, e1;
    CKH(hipEventCreate(&e0));
    CKH(hipEventCreate(&e1));
    SpmvArgs<float> a32{};
    a32.rp = c->rp; a32.col = c->col; a32.vals = c->w32; a32.x = c->x32; a32.y = c->y32;
    a32.diag = c->deg32; a32.n = n; a32.trim = -1;
    SpmvArgs<double> a64{};
    a64.rp = c->rp; a64.col = c->col; a64.vals = c->w64; a64.x = c->x64; a64.y = c->y64;
    a64.diag = c->deg; a64.n = n; a64.trim = -1;
    auto launch = [&]() {
      if (prec == ISIRA_FP64) launch_spmv_probe<double>(c->plan, valmode64(c), a64, c->rb.partials, s);
      else launch_spmv_probe<float>(c->plan, valmode32(c), a32, c->rb.partials, s);
    };
    for (int w = 0; w < 3; ++w) launch();
    double total = 0.0;
    float ms = 0;
    if (!cold) {
      CKH(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) launch();
      CKH(hipEventRecord(e1, s));
      CKH(hipEventSynchronize(e1));
      CKH(hipEventElapsedTime(&ms, e0, e1));
      total = ms;
    } else {
      for (int r = 0; r < reps; ++r) {
        launch_scale((int)(kFlush / 8), flush, 1.0, flush, s);
        CKH(hipEventRecord(e0, s));
        launch();
        CKH(hipEventRecord(e1, s));
        CKH(hipEventSynchronize(e1));
        CKH(hipEventElapsedTime(&ms, e0, e1));
        total += ms;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    dfree(c->mem, flush);
    *ms_per = total / reps;
    return ISIRA_OK;
  });
}

extern "C" int isira_inner_solve(isira_ctx* c, const double* r, const double* V, int32_t nc,
                                 double sigma, double delta, int64_t trim, double rtol,
                                 int32_t max_it, int32_t prec, int32_t precond, int32_t solver,
                                 double* z, int32_t* iters, double* relres) {
  return guarded([&]() -> int {
    if (!c || !r || !z || (nc > 0 && !V)) return fail(ISIRA_E_ARG, "NULL argument");
    if (nc < 0 || nc > kMaxC || nc > c->n - 3) return fail(ISIRA_E_ARG, "bad c");
    if (!(sigma >= 0.0) || !(sigma < c->min_deg)) return fail(ISIRA_E_ARG, "need 0 <= sigma < min degree");
    if (prec != ISIRA_FP64 && prec != ISIRA_FP32) return fail(ISIRA_E_ARG, "bad prec");
    if (precond == ISIRA_PC_LEARNED && !c->has_learned) return fail(ISIRA_E_PRECOND, "no learned preconditioner installed");
    if (solver != ISIRA_SOLVER_PCG && solver != ISIRA_SOLVER_MINRES) return fail(ISIRA_E_ARG, "bad solver");
    if (solver == ISIRA_SOLVER_MINRES && precond != ISIRA_PC_JACOBI)
      return fail(ISIRA_E_ARG, "MINRES runs with the Jacobi preconditioner only");
    if (precond != ISIRA_PC_JACOBI && precond != ISIRA_PC_LEARNED && precond != ISIRA_PC_MULTILEVEL)
      return fail(ISIRA_E_ARG, "bad precond");
    int rc = ensure_workspace(c, std::max(c->ws_m, 2), std::max(c->ws_k, std::max(1, (int)nc)));
    if (rc) return rc;
    const int n = (int)c->n;
    const int ld = c->ld;
    hipStream_t s = c->stream;
    InnerCfg cfg;
    cfg.prec = prec;
    cfg.precond = precond;
    cfg.sigma = sigma;
    cfg.delta = delta > 0 ? delta : 2.0 * c->max_deg;
    cfg.rtol = rtol;
    cfg.trim = trim >= 0 ? c->iperm[trim] : c->trim_default;
    if (precond == ISIRA_PC_LEARNED && (c->spai_trim != cfg.trim || c->spai_sigma != sigma))
      return fail(ISIRA_E_PRECOND, "learned preconditioner was installed for another sigma or trim index");
    if (precond == ISIRA_PC_MULTILEVEL && (!c->ml.ready || c->ml.trim != cfg.trim))
      return fail(ISIRA_E_PRECOND, "no multilevel hierarchy set up for this trim index");
    cfg.maxit = max_it > 0 ? max_it : 1000;
    cfg.check_every = 8;
    cfg.solver = solver;
    launch_dinv<double>(n, c->deg, sigma, cfg.trim, c->dinv64, s);
    launch_dinv<float>(n, c->deg, sigma, cfg.trim, c->dinv32, s);
    // deflation columns (internal order, trimmed row zeroed) and the SMW capacitance
    std::vector<double> Cm((size_t)nc * nc);
    for (int j = 0; j < nc; ++j) {
      launch_gather<double, double>(n, V + (size_t)j * n, c->d_perm, c->tmp64, s);
      launch_masked_copy<double>(n, c->tmp64, cfg.trim, c->Vin64 + (size_t)j * ld, s);
      launch_masked_copy<float>(n, c->tmp64, cfg.trim, c->Vin32 + (size_t)j * ld, s);
    }
    for (int j = 0; j < nc; ++j) {
      if (precond == ISIRA_PC_MULTILEVEL) {
        if (prec == ISIRA_FP64) {
          ml::apply<double>(c->ml, c->Vin64 + (size_t)j * ld, c->Y64 + (size_t)j * ld, 0, c->st, c->rb, s);
          launch_multidot<double>(n, c->Vin64, ld, nc, nullptr, ld, 0, c->Y64 + (size_t)j * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
        } else {
          ml::apply<float>(c->ml, c->Vin32 + (size_t)j * ld, c->Y32 + (size_t)j * ld, 0, c->st, c->rb, s);
          launch_multidot<float>(n, c->Vin32, ld, nc, nullptr, ld, 0, c->Y32 + (size_t)j * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
        }
      } else if (precond == ISIRA_PC_LEARNED) {
        if (prec == ISIRA_FP64) {
          spai::apply_plain<double>(c->spw, c->plan, c->rp, c->col,
                                    c->Vin64 + (size_t)j * ld, c->Y64 + (size_t)j * ld, n, cfg.trim, s);
          launch_multidot<double>(n, c->Vin64, ld, nc, nullptr, ld, 0, c->Y64 + (size_t)j * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
        } else {
          spai::apply_plain<float>(c->spw, c->plan, c->rp, c->col,
                                   c->Vin32 + (size_t)j * ld, c->Y32 + (size_t)j * ld, n, cfg.trim, s);
          launch_multidot<float>(n, c->Vin32, ld, nc, nullptr, ld, 0, c->Y32 + (size_t)j * ld, nullptr, 0, 0, c->hbuf, c->rb, s);
        }
      } else if (prec == ISIRA_FP64) {
        launch_multidot<double>(n, c->Vin64, ld, nc, nullptr, ld, 0, c->Vin64 + (size_t)j * ld, c->dinv64, 0, 0, c->hbuf, c->rb, s);
      } else {
        launch_multidot<float>(n, c->Vin32, ld, nc, nullptr, ld, 0, c->Vin32 + (size_t)j * ld, c->dinv32, 0, 0, c->hbuf, c->rb, s);
      }
      if ((rc = read_h(c, nc))) return rc;
      SYNC_OR_RETURN(c);
      for (int i = 0; i < nc; ++i) Cm[i + (size_t)j * nc] = c->hbuf_host[i];
    }
    if (nc > 0) {
      std::vector<double> G((size_t)nc * nc), Gi;
      for (int j = 0; j < nc; ++j)
        for (int i = 0; i < nc; ++i)
          G[i + (size_t)j * nc] = (i == j ? 1.0 : 0.0) + cfg.delta * 0.5 * (Cm[i + (size_t)j * nc] + Cm[j + (size_t)i * nc]);
      if (!spd_inverse(nc, G, Gi)) return fail(ISIRA_E_PRECOND, "SMW capacitance matrix not positive definite");
      if ((rc = upload(c, c->Ginv, Gi.data(), Gi.size() * 8))) return rc;
    }
    CKH(hipMemcpyAsync(c->tmp64, r, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    launch_gather<double, double>(n, c->tmp64, c->d_perm, c->r64, s);
    int its = 0, status = 0;
    double rel = 0.0;
    if (prec == ISIRA_FP64) rc = inner_pcg<double>(c, cfg, c->r64, 0.0, nc, &its, &status, &rel);
    else rc = inner_pcg<float>(c, cfg, c->r64, 0.0, nc, &its, &status, &rel);
    if (rc) return rc;
    if (prec == ISIRA_FP64) launch_enlarge<double>(n, c->x64, c->z64, c->st, c->rb, s);
    else launch_enlarge<float>(n, c->x32, c->z64, c->st, c->rb, s);
    launch_gather<double, double>(n, c->z64, c->d_iperm, z, s);
    SYNC_OR_RETURN(c);
    if (iters) *iters = its;
    if (relres) *relres = rel;
    return ISIRA_OK;
  });
}

extern "C" int isira_orthonormalize(isira_ctx* c, const double* Q, int32_t ncols,
                                    const double* z, double* u, double* norms) {
  return guarded([&]() -> int {
    if (!c || !z || !u || !norms || (ncols > 0 && !Q)) return fail(ISIRA_E_ARG, "NULL argument");
    if (ncols < 0 || ncols > ISIRA_MAX_BASIS) return fail(ISIRA_E_ARG, "bad ncols");
    int rc = ensure_workspace(c, std::max(c->ws_m, ncols + 1), std::max(c->ws_k, 1));
    if (rc) return rc;
    const int n = (int)c->n;
    const int ld = c->ld;
    hipStream_t s = c->stream;
    for (int j = 0; j < ncols; ++j) launch_gather<double, double>(n, Q + (size_t)j * n, c->d_perm, c->U + (size_t)j * ld, s);
    launch_gather<double, double>(n, z, c->d_perm, c->z64, s);
    if ((rc = cgs2(c, c->U, ncols, c->Vout, 0, c->z64, norms))) return rc;
    launch_scale(n, c->z64, norms[1] > 0 ? 1.0 / norms[1] : 0.0, c->tmp64, s);
    launch_gather<double, double>(n, c->tmp64, c->d_iperm, u, s);
    SYNC_OR_RETURN(c);
    return ISIRA_OK;
  });
}

// Allocation-free variant of isira_orthonormalize for callers that cannot allocate: the
// vectors stay in the caller's labels (Gram-Schmidt does not depend on the order of the
// rows), z is copied into u and orthogonalized there, and every intermediate lives in this
// GPU's `scratch`.  Each value in scratch is written before it is read, so nothing is
// cleared; calls that overlap on one GPU share scratch and race.
extern "C" int isira_orthonormalize_noalloc(isira_ctx* c, const double* Q, int32_t ncols,
                                            const double* z, double* u, double* norms) {
  return guarded([&]() -> int {
    if (!c || !z || !u || !norms || (ncols > 0 && !Q)) return fail(ISIRA_E_ARG, "NULL argument");
    if (ncols < 0 || ncols > kNoAllocMaxCols)
      return fail(ISIRA_E_ARG, "ncols must be 0.." + std::to_string(kNoAllocMaxCols) +
                                   " (the allocation-free scratch holds the partials of at most " +
                                   std::to_string(kNoAllocMaxCols) + " columns)");
    if (!c->scratch_dev) return fail(ISIRA_E_STATE, "no scratch address for this context");
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    double* base = (double*)c->scratch_dev;
    RedBuf rb{base, nullptr};
    double* h = base + kNoAllocH;
    double* norm0 = base + kNoAllocNorm0;
    DevState* st = (DevState*)(base + kNoAllocState);
    CKH(hipMemcpyAsync(u, z, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    // first pass: h = [Q 1]^T u and u^T u, then u -= Q h_Q + 1 (1^T u) / n
    launch_multidot<double>(n, Q, n, ncols, nullptr, n, 0, u, nullptr, 1, 1, h, rb, s);
    CKH(hipMemcpyAsync(norm0, h + ncols + 1, sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_gemv_sub(n, Q, n, ncols, nullptr, n, 0, h, 1, u, 0, st, rb, s);
    // second pass, with ||u||^2 into st->red[2]
    launch_multidot<double>(n, Q, n, ncols, nullptr, n, 0, u, nullptr, 1, 0, h, rb, s);
    launch_gemv_sub(n, Q, n, ncols, nullptr, n, 0, h, 1, u, 1, st, rb, s);
    launch_scale_dev(n, u, st->red + 2, u, s);
    double sq[2];
    CKH(hipMemcpyAsync(&sq[0], norm0, sizeof(double), hipMemcpyDeviceToHost, s));
    CKH(hipMemcpyAsync(&sq[1], st->red + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    CKH(hipStreamSynchronize(s));
    norms[0] = std::sqrt(std::max(0.0, sq[0]));
    norms[1] = std::sqrt(std::max(0.0, sq[1]));
    return ISIRA_OK;
  });
}

// ------------------------------------------------------------------------------ multilevel

extern "C" int isira_ml_default_options(isira_ml_options* o) {
  if (!o) return fail(ISIRA_E_ARG, "NULL argument");
  std::memset(o, 0, sizeof(*o));
  o->omega = 0.9;
  o->coarse_max = 512;
  o->max_levels = 24;
  o->trim_index = -1;
  return ISIRA_OK;
}

static void fill_ml_info(const ml::Hierarchy& H, isira_ml_info* info) {
  std::memset(info, 0, sizeof(*info));
  info->levels = (int32_t)H.rows.size();
  for (size_t l = 0; l < H.rows.size() && l < ISIRA_ML_MAX_LEVELS; ++l) {
    info->rows[l] = H.rows[l];
    info->offdiag_nnz[l] = H.offnnz[l];
    info->connected[l] = H.connected[l];
  }
  info->coarsest_dense = H.mL;
  info->stored_nnz = H.stored_nnz;
  info->device_bytes = H.device_bytes;
  info->setup_ms = H.setup_ms;
}

extern "C" int isira_ml_setup(isira_ctx* c, const isira_ml_options* opt, isira_ml_info* info) {
  return guarded([&]() -> int {
    if (!c) return fail(ISIRA_E_ARG, "NULL context");
    isira_ml_options o;
    isira_ml_default_options(&o);
    if (opt) o = *opt;
    if (!(o.omega > 0.0 && o.omega < 1.0)) return fail(ISIRA_E_ARG, "need 0 < omega < 1");
    if (o.coarse_max < 0 || o.coarse_max > 2048) return fail(ISIRA_E_ARG, "need 0 <= coarse_max <= 2048");
    if (o.max_levels < 1 || o.max_levels > ISIRA_ML_MAX_LEVELS) return fail(ISIRA_E_ARG, "need 1 <= max_levels <= ISIRA_ML_MAX_LEVELS");
    if (o.trim_index >= c->n) return fail(ISIRA_E_ARG, "trim_index out of range");
    const int n = (int)c->n;
    const int trim = o.trim_index >= 0 ? c->iperm[o.trim_index] : c->trim_default;
    std::vector<int32_t> rp((size_t)n + 1), col((size_t)c->nnz);
    std::vector<double> w;
    CKH(hipStreamSynchronize(c->stream));
    CKH(hipMemcpy(rp.data(), c->rp, rp.size() * 4, hipMemcpyDeviceToHost));
    CKH(hipMemcpy(col.data(), c->col, col.size() * 4, hipMemcpyDeviceToHost));
    if (c->wdt != ISIRA_W_NONE) {
      w.resize((size_t)c->nnz);
      CKH(hipMemcpy(w.data(), c->w64, w.size() * 8, hipMemcpyDeviceToHost));
    }
    ml::Params prm{o.omega, o.coarse_max, o.max_levels};
    const int rc = ml::setup(c->ml, n, rp.data(), col.data(), w.empty() ? nullptr : w.data(),
                             c->perm.data(), trim, prm);
    if (rc) return rc;
    // the in-place cycle needs room for the second level after the inner residual
    c->ri_tail = c->ml.lv.empty() ? 0 : c->ml.lv[0].nc;
    if (c->ws_tail < c->ri_tail) free_workspace(c);
    if (info) fill_ml_info(c->ml, info);
    return ISIRA_OK;
  });
}

extern "C" int isira_ml_apply(isira_ctx* c, int32_t prec, const double* x, double* y) {
  return guarded([&]() -> int {
    if (!c || !x || !y) return fail(ISIRA_E_ARG, "NULL argument");
    if (prec != ISIRA_FP64 && prec != ISIRA_FP32) return fail(ISIRA_E_ARG, "bad prec");
    if (!c->ml.ready) return fail(ISIRA_E_STATE, "no multilevel hierarchy set up");
    int rc = ensure_workspace(c, std::max(c->ws_m, 2), std::max(c->ws_k, 1));
    if (rc) return rc;
    const int n = (int)c->n;
    hipStream_t s = c->stream;
    launch_gather<double, double>(n, x, c->d_perm, c->tmp64, s);
    if (prec == ISIRA_FP64) {
      launch_masked_copy<double>(n, c->tmp64, c->ml.trim, c->ri64, s);
      ml::apply<double>(c->ml, c->ri64, c->y64, 0, c->st, c->rb, s);
      launch_gather<double, double>(n, c->y64, c->d_iperm, y, s);
    } else {
      launch_masked_copy<float>(n, c->tmp64, c->ml.trim, c->ri32, s);
      ml::apply<float>(c->ml, c->ri32, c->y32, 0, c->st, c->rb, s);
      launch_gather<float, double>(n, c->y32, c->d_iperm, y, s);
    }
    CKH(hipGetLastError());
    SYNC_OR_RETURN(c);
    return ISIRA_OK;
  });
}

extern "C" int isira_ml_get_info(const isira_ctx* c, isira_ml_info* info) {
  return guarded([&]() -> int {
    if (!c || !info) return fail(ISIRA_E_ARG, "NULL argument");
    if (!c->ml.ready) return fail(ISIRA_E_STATE, "no multilevel hierarchy set up");
    fill_ml_info(c->ml, info);
    return ISIRA_OK;
  });
}

// ------------------------------------------------------------------------------ learned SPAI

extern "C" int32_t isira_spai_nparam(void) { return spai::nparam(); }

static int spai_trim_internal(const isira_ctx* c, int64_t trim, int* out) {
  if (trim >= c->n) return fail(ISIRA_E_ARG, "trim index out of range");
  *out = trim >= 0 ? c->iperm[trim] : c->trim_default;
  return ISIRA_OK;
}

extern "C" int isira_spai_install(isira_ctx* c, const float* params, double sigma, int64_t trim) {
  return guarded([&]() -> int {
    if (!c || !params) return fail(ISIRA_E_ARG, "NULL argument");
    if (!(sigma >= 0.0) || !(sigma < c->min_deg)) return fail(ISIRA_E_ARG, "need 0 <= sigma < min degree");
    int t, rc;
    if ((rc = spai_trim_internal(c, trim, &t))) return rc;
    const void* wts = c->wdt == ISIRA_W_NONE ? nullptr : (const void*)c->w32;
    const int wdt = c->wdt == ISIRA_W_NONE ? ISIRA_W_NONE : ISIRA_W_F32;
    const int frc = spai::forward(c->spw, c->rp, c->col, wts, wdt, c->deg, (int)c->n, c->nnz, sigma, t,
                                  params, c->stream);
    if (frc == ISIRA_E_WORKSPACE) return frc;  // message set by the allocator
    if (frc) return fail(ISIRA_E_HIP, "SPAI forward failed");
    SYNC_OR_RETURN(c);
    spai::free_pruned(c->spw);  // new values: any earlier pruning is void
    c->has_learned = true;
    c->spai_sigma = sigma;
    c->spai_trim = t;
    return ISIRA_OK;
  });
}

extern "C" int isira_spai_prune(isira_ctx* c, double tau, int64_t* kept) {
  return guarded([&]() -> int {
    if (!c) return fail(ISIRA_E_ARG, "NULL context");
    if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(ISIRA_E_ARG, "need a finite tau >= 0");
    if (!c->has_learned) return fail(ISIRA_E_PRECOND, "no learned preconditioner installed");
    const int64_t n = c->n, nnz = c->nnz;
    std::vector<int32_t> rp((size_t)n + 1), col((size_t)nnz);
    std::vector<float> off((size_t)nnz), dg((size_t)n);
    CKH(hipStreamSynchronize(c->stream));
    CKH(hipMemcpy(rp.data(), c->rp, rp.size() * 4, hipMemcpyDeviceToHost));
    CKH(hipMemcpy(col.data(), c->col, col.size() * 4, hipMemcpyDeviceToHost));
    CKH(hipMemcpy(off.data(), c->spw.offd, off.size() * 4, hipMemcpyDeviceToHost));
    CKH(hipMemcpy(dg.data(), c->spw.diag32, dg.size() * 4, hipMemcpyDeviceToHost));
    // keep m_ij when nonzero and |m_ij| >= tau sqrt(M_ii M_jj), decided in FP64 from the
    // stored FP32 values; symmetric in (i, j) because m_ij and m_ji are equal
    std::vector<uint8_t> keep((size_t)nnz);
    std::vector<int32_t> cnt((size_t)n);
    std::atomic<int> asym{0};
    parallel_for(n, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e; ++i) {
        int k = 0;
        for (int32_t j = rp[i]; j < rp[i + 1]; ++j) {
          const double m = (double)off[j];
          const bool kp = m != 0.0 && std::fabs(m) >= tau * std::sqrt((double)dg[i] * (double)dg[col[j]]);
          keep[j] = kp;
          k += kp;
          if (kp) {  // the transposed entry must carry the same value
            const int32_t o = col[j];
            const int32_t* f = std::lower_bound(col.data() + rp[o], col.data() + rp[o + 1], (int32_t)i);
            if (f == col.data() + rp[o + 1] || *f != (int32_t)i || off[f - col.data()] != off[j]) asym = 1;
          }
        }
        cnt[i] = k;
      }
    });
    if (asym) return fail(ISIRA_E_PRECOND, "learned values are not symmetric");
    std::vector<int32_t> prp((size_t)n + 1, 0);
    for (int64_t i = 0; i < n; ++i) prp[i + 1] = prp[i] + cnt[i];
    const int64_t pnnz = prp[n];
    std::vector<int32_t> pcol((size_t)pnnz);
    std::vector<float> pval((size_t)pnnz);
    parallel_for(n, [&](int64_t b, int64_t e) {
      for (int64_t i = b; i < e; ++i) {
        int32_t o = prp[i];
        for (int32_t j = rp[i]; j < rp[i + 1]; ++j) {
          if (keep[j]) {
            pcol[o] = col[j];
            pval[o] = off[j];
            ++o;
          } else {
            off[j] = 0.0f;
          }
        }
      }
    });
    spai::free_pruned(c->spw);
    int rc;
    auto undo = [&](int code) {
      spai::free_pruned(c->spw);
      return code;
    };
    if ((rc = dalloc(c->mem, &c->spw.prp, (size_t)n + 1))) return undo(rc);
    if ((rc = dalloc(c->mem, &c->spw.pcol, (size_t)pnnz))) return undo(rc);
    if ((rc = dalloc(c->mem, &c->spw.pval, (size_t)pnnz))) return undo(rc);
    std::vector<int32_t> plong;
    for (int64_t i = 0; i < n; ++i)
      if (cnt[i] > kSpLongRow) plong.push_back((int32_t)i);
    if ((rc = dalloc(c->mem, &c->spw.plong, plong.size()))) return undo(rc);
    hipError_t e = hipMemcpy(c->spw.prp, prp.data(), prp.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && !plong.empty())
      e = hipMemcpy(c->spw.plong, plong.data(), plong.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && pnnz > 0) e = hipMemcpy(c->spw.pcol, pcol.data(), pcol.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess && pnnz > 0) e = hipMemcpy(c->spw.pval, pval.data(), pval.size() * 4, hipMemcpyHostToDevice);
    // the full-pattern values follow the pruning too (export, and any product on the pattern)
    if (e == hipSuccess) e = hipMemcpy(c->spw.offd, off.data(), off.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      c->has_learned = false;  // the device values may be half updated: install again
      return undo(fail(ISIRA_E_HIP, std::string("isira_spai_prune upload: ") + hipGetErrorString(e)));
    }
    c->spw.pruned = true;
    c->spw.pnnz = pnnz;
    c->spw.n_long = (int64_t)plong.size();
    if (kept) *kept = pnnz;
    return ISIRA_OK;
  });
}

extern "C" int isira_spai_export(isira_ctx* c, float* diag, float* offd) {
  return guarded([&]() -> int {
    if (!c || !diag || !offd) return fail(ISIRA_E_ARG, "NULL argument");
    if (!c->has_learned) return fail(ISIRA_E_PRECOND, "no learned preconditioner installed");
    launch_gather<float, float>((int)c->n, c->spw.diag32, c->d_iperm, diag, c->stream);
    spai::scatter_offd(c->nnz, c->spw.offd, c->d_emap, offd, c->stream);
    SYNC_OR_RETURN(c);
    return ISIRA_OK;
  });
}

extern "C" int isira_spai_loss_grad(isira_ctx* c, const float* params, double sigma, int64_t trim,
                                    const float* r, const float* z, int32_t S, float* grad,
                                    double* loss) {
  return guarded([&]() -> int {
    if (!c || !params || !r || !z || !grad || !loss) return fail(ISIRA_E_ARG, "NULL argument");
    if (S < 1 || S > 64) return fail(ISIRA_E_ARG, "need 1 <= S <= 64 samples per call");
    if (!(sigma >= 0.0) || !(sigma < c->min_deg)) return fail(ISIRA_E_ARG, "need 0 <= sigma < min degree");
    int t, rc;
    if ((rc = spai_trim_internal(c, trim, &t))) return rc;
    const void* wts = c->wdt == ISIRA_W_NONE ? nullptr : (const void*)c->w32;
    const int wdt = c->wdt == ISIRA_W_NONE ? ISIRA_W_NONE : ISIRA_W_F32;
    c->has_learned = false;  // the forward pass below overwrites the installed values
    spai::free_pruned(c->spw);
    const int lrc = spai::loss_grad(c->spw, c->rp, c->col, wts, wdt, c->deg, (int)c->n, c->nnz, sigma, t,
                                    params, c->d_perm, r, z, S, grad, loss, c->rb, c->stream);
    if (lrc == ISIRA_E_WORKSPACE) return lrc;
    if (lrc) return fail(ISIRA_E_HIP, "SPAI loss/gradient failed");
    return ISIRA_OK;
  });
}

extern "C" int isira_adam_step(isira_ctx* c, float* param, const float* grad, float* m, float* v,
                               int32_t count, float lr, float beta1, float beta2, float eps,
                               int32_t step) {
  return guarded([&]() -> int {
    if (!c || !param || !grad || !m || !v || count < 1 || step < 1) return fail(ISIRA_E_ARG, "bad argument");
    spai::adam(param, grad, m, v, count, lr, beta1, beta2, eps, step, c->stream);
    SYNC_OR_RETURN(c);
    return ISIRA_OK;
  });
}

extern "C" const char* isira_strerror(int code) {
  switch (code) {
    case ISIRA_OK: return "ok";
    case ISIRA_NOT_CONVERGED: return "not converged (max_outer reached)";
    case ISIRA_E_ARG: return "invalid argument";
    case ISIRA_E_GRAPH: return "invalid graph";
    case ISIRA_E_DISCONNECTED: return "graph not connected";
    case ISIRA_E_HIP: return "HIP runtime error";
    case ISIRA_E_PRECOND: return "preconditioner error";
    case ISIRA_E_STATE: return "invalid state";
    case ISIRA_E_WORKSPACE: return "workspace too small";
    case ISIRA_E_HOST: return "host-side failure";
    default: return "unknown error";
  }
}

extern "C" const char* isira_last_error(void) { return g_err.c_str(); }

// shared with spai.hip
namespace isira {
int set_error(int code, const char* msg) { return fail(code, msg); }
}
