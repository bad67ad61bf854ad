// gfx950 kernels of the iSIRA hot path: Laplacian SpMV (binned, persistent, split long
// rows), fused PCG updates for the trimmed shifted deflated system (2.15) with the
// Jacobi + Sherman-Morrison-Woodbury preconditioner (3.5), enlargement (2.5), column dots
// and updates of classical Gram-Schmidt, Ritz residuals and tall-skinny basis rotations.
//
// Reductions are deterministic: every workgroup writes one partial per value, and the last
// workgroup to arrive (integer arrival counter) sums the partials in a fixed order.
#include "internal.h"

namespace isira {

// ------------------------------------------------------------------ reduction helpers

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename T>
__device__ __forceinline__ T group_sum(T v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum one double over the workgroup; the result is valid in thread 0.
__device__ __forceinline__ double block_sum1(double v, double* sh4) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh4[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  return s;
}

// Publish this workgroup's partials and report whether it is the last to arrive.
__device__ __forceinline__ bool arrive_last(unsigned* counter) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    s_last = (prev == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) __threadfence();
  return last;
}

// Finishing dispatch: out[v] = sum over workgroups of partials[v * nblk + b], one wave per
// value (round-robin over the waves of the workgroup); each lane sums b = lane, lane + 64,
// ... in increasing order, then the wave sums its lanes: a fixed order.
constexpr int kFin = 1024;  // threads of the finishing dispatches
__device__ void final_reduce(const double* partials, int nv, int nblk, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int v = wid; v < nv; v += nw) {
    const double* pv = partials + (size_t)v * nblk;
    double s = 0.0;
    int b = lane;
    for (; b + 7 * 64 < nblk; b += 8 * 64) {
      double t[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) t[i] = pv[b + i * 64];
#pragma unroll
      for (int i = 0; i < 8; ++i) s += t[i];
    }
    for (; b < nblk; b += 64) s += pv[b];
    s = wave_sum(s);
    if (lane == 0) out[v] = s;
  }
  __syncthreads();
}

// Sum one double over a workgroup of up to 1024 threads; valid in thread 0.
__device__ __forceinline__ double block_sum_any(double v) {
  __shared__ double sh[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) s += sh[w];
  return s;
}

template <int NV>
__device__ void write_partials(const double (&acc)[NV], int nv, double* partials) {
  __shared__ double sh[4][NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if (v < nv) {
      double s = wave_sum(acc[v]);
      if (lane == 0) sh[wid][v] = s;
    }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += blockDim.x)
    partials[(size_t)v * gridDim.x + blockIdx.x] = (sh[0][v] + sh[1][v]) + (sh[2][v] + sh[3][v]);
}

static_assert((size_t)(2 + kMaxC) * kStreamGrid <= kPartialsElems, "PCG partials");
static_assert((size_t)kMaxCols * kStreamGrid <= kPartialsElems, "multi-dot partials");
static_assert((size_t)kSpmvGrid <= kPartialsElems, "SpMV partials");



#define HIP_LAUNCH_CHECK() (void)hipGetLastError()

// ------------------------------------------------------------------ setup kernels

__global__ __launch_bounds__(kBlock) void k_degree(const int32_t* rp, const void* w, int wdt,
                                                   int n, double* d, float* d32) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int nwaves = (gridDim.x * kBlock) >> 6;
  for (int row = wave; row < n; row += nwaves) {
    const int b = rp[row], e = rp[row + 1];
    double s = 0.0;
    if (wdt == ISIRA_W_NONE) {
      s = (lane == 0) ? (double)(e - b) : 0.0;
    } else if (wdt == ISIRA_W_F32) {
      for (int j = b + lane; j < e; j += 64) s += (double)((const float*)w)[j];
    } else {
      for (int j = b + lane; j < e; j += 64) s += ((const double*)w)[j];
    }
    s = wave_sum(s);
    if (lane == 0) {
      d[row] = s;
      d32[row] = (float)s;
    }
  }
}

void launch_degree(const int32_t* rp, const void* w, int wdt, int n, double* d, float* d32,
                   hipStream_t s) {
  int grid = (n + 3) / 4;
  if (grid > 4096) grid = 4096;
  k_degree<<<grid, kBlock, 0, s>>>(rp, w, wdt, n, d, d32);
  HIP_LAUNCH_CHECK();
}

// max degree (lowest caller label among ties), its internal index, min degree.
__global__ __launch_bounds__(kBlock) void k_argmax_degree(const double* d, const int32_t* perm,
                                                          int n, int use_abs, double* partials,
                                                          unsigned* counter, double* out3) {
  double best = -1.0, best_lab = 1e300, best_int = -1.0, mn = 1e300;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    const double v = use_abs ? fabs(d[l]) : d[l];
    const double lab = (double)perm[l];
    if (v > best || (v == best && lab < best_lab)) {
      best = v;
      best_lab = lab;
      best_int = (double)l;
    }
    mn = v < mn ? v : mn;
  }
  // workgroup reduction by shared arrays (4 values per thread)
  __shared__ double sb[kBlock], sl[kBlock], si[kBlock], sm[kBlock];
  sb[threadIdx.x] = best;
  sl[threadIdx.x] = best_lab;
  si[threadIdx.x] = best_int;
  sm[threadIdx.x] = mn;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const int t = threadIdx.x + o;
      if (sb[t] > sb[threadIdx.x] || (sb[t] == sb[threadIdx.x] && sl[t] < sl[threadIdx.x])) {
        sb[threadIdx.x] = sb[t];
        sl[threadIdx.x] = sl[t];
        si[threadIdx.x] = si[t];
      }
      sm[threadIdx.x] = sm[t] < sm[threadIdx.x] ? sm[t] : sm[threadIdx.x];
    }
    __syncthreads();
  }
  const int G = gridDim.x;
  if (threadIdx.x == 0) {
    partials[0 * G + blockIdx.x] = sb[0];
    partials[1 * G + blockIdx.x] = sl[0];
    partials[2 * G + blockIdx.x] = si[0];
    partials[3 * G + blockIdx.x] = sm[0];
  }
  if (!arrive_last(counter)) return;
  if (threadIdx.x == 0) {
    double b = -1.0, bl = 1e300, bi = -1.0, m = 1e300;
    for (int k = 0; k < G; ++k) {
      const double v = partials[k], lab = partials[G + k];
      if (v > b || (v == b && lab < bl)) {
        b = v;
        bl = lab;
        bi = partials[2 * G + k];
      }
      m = partials[3 * G + k] < m ? partials[3 * G + k] : m;
    }
    out3[0] = b;
    out3[1] = bi;
    out3[2] = m;
    out3[3] = bl;
    *counter = 0u;
  }
}

void launch_argmax_degree(const double* d, const int32_t* perm, int n, DevState*, RedBuf rb,
                          double* out4, hipStream_t s) {
  int grid = stream_grid(n);
  if (grid > 256) grid = 256;
  k_argmax_degree<<<grid, kBlock, 0, s>>>(d, perm, n, 0, rb.partials, rb.counters + 0, out4);
  HIP_LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_signed_gather(int n, const double* __restrict__ v,
                                                          const int32_t* __restrict__ iperm,
                                                          const double* scal4,
                                                          double* __restrict__ out) {
  const double sgn = v[(int)scal4[1]] < 0.0 ? -1.0 : 1.0;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    out[l] = sgn * v[iperm[l]];
}

void launch_signed_gather(int n, const double* v, const int32_t* perm, const int32_t* iperm,
                          double* out, double* scal4, RedBuf rb, hipStream_t s) {
  int grid = stream_grid(n);
  if (grid > 256) grid = 256;
  k_argmax_degree<<<grid, kBlock, 0, s>>>(v, perm, n, 1, rb.partials, rb.counters + 0, scal4);
  k_signed_gather<<<stream_grid(n), kBlock, 0, s>>>(n, v, iperm, scal4, out);
  HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ sparse product

struct SplitInfo {
  const int32_t* rowof;  // per slot: the split row
  const int32_t* base;   // per slot: first chunk partial
  const int32_t* nchunk; // per slot: number of chunks
  double* part;          // per chunk partial sums
  double* red;           // per slot: reduction contribution (scratch)
  int32_t nslots;
};

// a load of data read once per launch: non-temporal when NT
template <bool NT, typename P>
__device__ __forceinline__ P stream_ld(const P* p) {
  if constexpr (NT) {
    return __builtin_nontemporal_load(p);
  } else {
    return *p;
  }
}

template <int VM, typename T, bool NT>
__device__ __forceinline__ T edge_val(const void* vals, int j) {
  if constexpr (VM == kUnitNeg) {
    return T(1);
  } else if constexpr (VM == kF64Neg || VM == kF64Pos) {
    return (T)stream_ld<NT>((const double*)vals + j);
  } else {
    return (T)stream_ld<NT>((const float*)vals + j);
  }
}

// Finish row `row` given the neighbour sum and the row's own x and diagonal entries;
// returns this row's reduction contribution.
template <int VM, typename T>
__device__ __forceinline__ double finish_row_xd(const SpmvArgs<T>& a, int row, T nsum, T xl,
                                                T dl, const double* sh_t, T shift_add) {
  T y = dl * xl;
  if constexpr (VM == kF32Pos || VM == kF64Pos) {
    y += nsum;
  } else {
    y -= nsum;
  }
  if (a.sigma != 0.0) y -= (T)a.sigma * xl;
  y += shift_add;
  if (a.c > 0) {
    // four columns in flight (the last group re-reads column c-1 with weight 0)
    T s = T(0);
    const T* __restrict__ V = a.V + row;
    for (int j0 = 0; j0 < a.c; j0 += 4) {
      T v4[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = j0 + i < a.c ? j0 + i : a.c - 1;
        v4[i] = V[(int64_t)j * a.ldv];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (j0 + i < a.c) s += v4[i] * (T)sh_t[j0 + i];
    }
    y += (T)a.delta * s;
  }
  if (row == a.trim) y = T(0);
  a.y[row] = y;
  if (a.red == 2) {
    const double dd = (double)y - a.theta * (double)xl;
    return dd * dd;
  }
  if (a.red == 1 || a.red == 3 || a.red == 4) return (double)xl * (double)y;
  return 0.0;
}

template <int VM, typename T>
__device__ __forceinline__ double finish_row(const SpmvArgs<T>& a, int row, T nsum,
                                             const double* sh_t, T shift_add) {
  return finish_row_xd<VM, T>(a, row, nsum, a.x[row], a.diag[row], sh_t, shift_add);
}

// x[c] for all PT slots of a thread (c = -1 marks an empty slot, whose value is 0).  Every
// load is unconditional, so that all of them are in flight before the first is used: an
// empty slot reads x[0], and with a hub cache a column below HUB reads xs[c] while its
// global load is redirected to x[0] as well (one shared cache line per wave).  Selecting
// between the LDS and the global pointer instead would make generic-address loads that
// the compiler waits for one at a time.
template <typename T, int PT, int HUB>
__device__ __forceinline__ void gather_slots(const int (&ci)[PT], const T* __restrict__ x,
                                             const T* xs, T (&g)[PT]) {
  T gg[PT];
#pragma unroll
  for (int k = 0; k < PT; ++k) {
    const int c = ci[k];
    const bool glob = HUB > 0 ? c >= HUB : c >= 0;
    gg[k] = x[glob ? c : 0];
  }
  if constexpr (HUB > 0) {
    T gl[PT];
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int c = ci[k];
      gl[k] = xs[(c >= 0 && c < HUB) ? c : 0];
    }
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int c = ci[k];
      g[k] = c < 0 ? T(0) : (c < HUB ? gl[k] : gg[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < PT; ++k) g[k] = ci[k] < 0 ? T(0) : gg[k];
  }
}

// Sparse product over work units (persistent grid, units taken round-robin).  A stream unit
// loads its column indices and its rows' pointers, own x entries and diagonal entries in one
// coalesced batch, gathers x for all its nonzeros and stages the products in LDS; each row
// is then summed from LDS by G lanes into a row sum in LDS, and every thread finishes the
// rows it loaded (coalesced stores).  A chunk unit of a long row sums its nonzeros into one
// partial.  Two shapes: 256 threads / 2048-nonzero units (8 workgroups per CU), and, for
// power-law graphs, 512 threads / 4096-nonzero units (2 workgroups per CU) with x of the
// HUB highest-degree columns (the first HUB labels after relabelling) staged once per
// workgroup in LDS, so that those gathers never reach L2.  In the hub shape, column
// indices and edge weights, read once per launch, are loaded non-temporally so that they
// do not displace lines of x from the L2 (the stream shape keeps ordinary loads: its
// matrix can stay in the memory-side cache between launches, which non-temporal loads
// bypass).  A thread's slots of the next unit are loaded as soon
// as the current unit is finished.  TAG only separates the symbol of the bandwidth probe
// (isira_time_spmv) from the solver's launches in profiler summaries.
template <typename T, int VM, int TAG, int NT, int UNNZ, int UROWS, int HUB>
__global__ __launch_bounds__(NT) void k_spmv(SpmvArgs<T> a, const int4* __restrict__ units,
                                             int n_units, double* partials,
                                             double* __restrict__ chunk_part) {
  if (a.check_done && a.st->done) return;
  constexpr bool kNT = HUB > 0;  // non-temporal column and weight loads (see above)
  constexpr int PT = UNNZ / NT;           // nonzeros per thread and unit
  constexpr int RPT = (UROWS + NT) / NT;  // row pointers per thread (UROWS + 1 entries)
  constexpr int RRT = UROWS / NT;         // rows finished per thread
  static_assert(UROWS % NT == 0, "unit rows");
  __shared__ T prod[UNNZ];
  __shared__ int srp[UROWS + 1];
  __shared__ T srow[UROWS];
  __shared__ T xs[HUB > 0 ? HUB : 1];
  __shared__ double sh_t[kMaxC];
  __shared__ T shT[NT / 64];
  const int tid = threadIdx.x;
  const double* tv = a.tvec ? a.tvec : (a.st ? a.st->t1 : nullptr);
  for (int j = tid; j < a.c; j += NT) sh_t[j] = tv[j];
  const T shift_add = (a.sig_over_n != 0.0) ? (T)(a.sig_over_n * a.st->sump) : T(0);
  const T* __restrict__ x = a.x;
  const T* __restrict__ dg = a.diag;
  const int32_t* __restrict__ col = a.col;
  const int32_t* __restrict__ rp = a.rp;
  if constexpr (HUB > 0) {
    const int hn = a.n < HUB ? a.n : HUB;
    for (int i = tid; i < hn; i += NT) xs[i] = x[i];
  }
  __syncthreads();
  // x gathers for all slots at once (see gather_slots)
  auto gather = [&](const int (&ci)[PT], T (&g)[PT]) { gather_slots<T, PT, HUB>(ci, x, xs, g); };
  // descriptors kept as plain scalars: int4 copies of HIP's vector type go through scratch
  struct Desc {
    int x, y, z, w;  // {r0 | row, j0, j1, (rows << 8 | G) | -(chunk + 1)}
  };
  auto ld_desc = [&](int i) -> Desc {
    if (i < n_units) {
      const int4 t = units[i];
      return Desc{t.x, t.y, t.z, t.w};
    }
    return Desc{0, 0, 0, 0};  // j0 = j1 and no rows: every load below is skipped
  };
  // everything a unit needs before its gathers, for the thread's slots
  struct Slots {
    int ci[PT];
    T v[PT];
    int rpv[RPT];
    T xv[RRT], dv[RRT];
  };
  auto load_slots = [&](const Desc& d, Slots& sl) {
#pragma unroll
    for (int k = 0; k < PT; ++k) {
      const int e = d.y + tid + k * NT;
      const bool in = e < d.z;
      sl.ci[k] = in ? stream_ld<kNT>(col + e) : -1;
      sl.v[k] = in ? edge_val<VM, T, kNT>(a.vals, e) : T(0);
    }
    const int nr = d.w >= 0 ? (d.w >> 8) : -1;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int t = tid + k * NT;
      sl.rpv[k] = (t <= nr) ? rp[d.x + t] : 0;
    }
#pragma unroll
    for (int k = 0; k < RRT; ++k) {
      const int t = tid + k * NT;
      const bool in = t < nr;
      sl.xv[k] = in ? x[d.x + t] : T(0);
      sl.dv[k] = in ? dg[d.x + t] : T(0);
    }
  };
  double acc = 0.0;
  const int G0 = gridDim.x;
  int u = blockIdx.x;
  Desc dcur = ld_desc(u);
  Desc dnxt = ld_desc(u + G0);
  Slots cur;
  load_slots(dcur, cur);
  for (; u < n_units; u += G0) {
    const Desc un = dcur;
    const int j0 = un.y;
    if (un.w >= 0) {
      const int r0 = un.x, nr = un.w >> 8, G = un.w & 255;
      const int R = NT / G, grp = tid / G, gl = tid - grp * G;
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        const int t = tid + k * NT;
        if (t <= nr) srp[t] = cur.rpv[k] - j0;
      }
      T gv[PT];
      gather(cur.ci, gv);
#pragma unroll
      for (int k = 0; k < PT; ++k) prod[tid + k * NT] = cur.v[k] * gv[k];
      __syncthreads();
      if (G == 1) {
        // one lane per row: the rows a thread sums are the rows it loaded
#pragma unroll
        for (int k = 0; k < RRT; ++k) {
          const int t = tid + k * NT;
          if (t < nr) {
            T s = T(0);
            const int e = srp[t + 1];
            for (int j = srp[t]; j < e; ++j) s += prod[j];
            acc += finish_row_xd<VM, T>(a, r0 + t, s, cur.xv[k], cur.dv[k], sh_t, shift_add);
          }
        }
        // prod and srp are rewritten by the next unit only after this barrier (G is uniform)
        __syncthreads();
      } else {
        for (int rr = grp; rr < nr; rr += R) {
          T s = T(0);
          const int e = srp[rr + 1];
          for (int j = srp[rr] + gl; j < e; j += G) s += prod[j];
          s = group_sum(s, G);
          if (gl == 0) srow[rr] = s;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < RRT; ++k) {
          const int t = tid + k * NT;
          if (t < nr)
            acc += finish_row_xd<VM, T>(a, r0 + t, srow[t], cur.xv[k], cur.dv[k], sh_t, shift_add);
        }
        // prod and srp were last read before the barrier above; srow is rewritten by the
        // next unit only after its first barrier
      }
    } else {
      T gv[PT];
      gather(cur.ci, gv);
      T s = T(0);
#pragma unroll
      for (int k = 0; k < PT; ++k) s += cur.v[k] * gv[k];
      s = wave_sum(s);
      if ((tid & 63) == 0) shT[tid >> 6] = s;
      __syncthreads();
      if (tid == 0) {
        T t = T(0);
        for (int w = 0; w < NT / 64; ++w) t += shT[w];
        chunk_part[-un.w - 1] = (double)t;
      }
      __syncthreads();
    }
    dcur = dnxt;
    dnxt = ld_desc(u + 2 * G0);
    load_slots(dcur, cur);
  }
  if (a.red == 0) return;
  const double bs = block_sum_any(acc);
  if (tid == 0) partials[blockIdx.x] = bs;
}

// Second dispatch of the sparse product (one workgroup): finishes the split rows from
// their chunk sums (fixed chunk order) and reduces the per-workgroup partials plus the
// split rows' contributions in a fixed order.
template <typename T, int VM>
__global__ __launch_bounds__(kFin) void k_spmv_fin(SpmvArgs<T> a, SplitInfo sp, int nblk,
                                                   const double* partials) {
  if (a.check_done && a.st->done) return;
  __shared__ double sh_t[kMaxC];
  __shared__ double fold[1];
  const int tid = threadIdx.x;
  if (a.fold_partials) {
    // sum(p) of the p-update, in a fixed order (V-hat^T p is already in st->t1)
    final_reduce(a.fold_partials, 1, a.fold_nblk, fold);
    if (tid == 0) a.st->sump = fold[0];
  }
  const double* tv = a.tvec ? a.tvec : (a.st ? a.st->t1 : nullptr);
  for (int j = tid; j < a.c; j += blockDim.x) sh_t[j] = tv[j];
  const T shift_add = (a.sig_over_n != 0.0) ? (T)(a.sig_over_n * a.st->sump) : T(0);
  __syncthreads();
  double acc = 0.0;
  for (int slot = tid; slot < sp.nslots; slot += blockDim.x) {
    double tot = 0.0;
    const int nb = sp.nchunk[slot], pb = sp.base[slot];
    for (int k = 0; k < nb; ++k) tot += sp.part[pb + k];
    acc += finish_row<VM, T>(a, sp.rowof[slot], (T)tot, sh_t, shift_add);
  }
  if (a.red == 0) return;
  for (int b = tid; b < nblk; b += blockDim.x) acc += partials[b];
  const double tot = block_sum_any(acc);
  if (tid == 0) {
    DevState* st = a.st;
    if (a.red == 1 || a.red == 4) {
      double pq = tot;
      if (a.fold_partials) {
        double tt = 0.0;
        for (int j = 0; j < a.fold_c; ++j) tt += st->t1[j] * st->t1[j];
        pq += a.delta * tt + a.fold_sig_over_n * fold[0] * fold[0];
      }
      st->pq = pq;
      if (a.red == 4) return;  // MINRES: delta_j = z^T K z, any sign
      const double alpha = st->rho / pq;
      if (!(pq > 0.0) || !isfinite(alpha)) {
        st->done = 1;
        st->status = kPcgBreakdown;
      }
      st->alpha = alpha;
    } else if (a.red == 2) {
      st->red[0] = tot;
    } else {
      st->red[1] = tot;
    }
  }
}

static SplitInfo split_info(const SpmvPlan& plan) {
  return SplitInfo{plan.split_rowof, plan.split_base, plan.split_nchunk, plan.split_part,
                   plan.split_red, plan.n_split_rows};
}

// The main dispatch and, when split rows or a reduction need it, the finishing dispatch
// (left out by the timing probe, whose output nobody reads).
template <typename T, int VM, int TAG>
static void spmv_dispatch(const SpmvPlan& plan, const SpmvArgs<T>& a, double* partials,
                          hipStream_t s, bool with_fin = true) {
  const SplitInfo sp = split_info(plan);
  constexpr int HUB = sizeof(T) == 8 ? kHubX64 : kHubX32;
  if (plan.hub) {
    k_spmv<T, VM, TAG, kHubThreads, kHubUnitNnz, kHubUnitRows, HUB>
        <<<plan.grid, kHubThreads, 0, s>>>(a, plan.units, plan.n_units, partials,
                                           plan.split_part);
  } else {
    k_spmv<T, VM, TAG, kBlock, kUnitNnz, kUnitRows, 0>
        <<<plan.grid, kBlock, 0, s>>>(a, plan.units, plan.n_units, partials, plan.split_part);
  }
  if (with_fin && (plan.n_split_rows > 0 || a.red != 0))
    k_spmv_fin<T, VM><<<1, kFin, 0, s>>>(a, sp, plan.grid, partials);
}

template <typename T>
void launch_spmv(const SpmvPlan& plan, int valmode, const SpmvArgs<T>& a, RedBuf rb,
                 hipStream_t s) {
  double* part = rb.partials ? rb.partials + kSpmvPartOff : nullptr;
  switch (valmode) {
    case kUnitNeg: spmv_dispatch<T, kUnitNeg, 0>(plan, a, part, s); break;
    case kF32Neg: spmv_dispatch<T, kF32Neg, 0>(plan, a, part, s); break;
    case kF64Neg: spmv_dispatch<T, kF64Neg, 0>(plan, a, part, s); break;
    case kF64Pos: spmv_dispatch<T, kF64Pos, 0>(plan, a, part, s); break;
    default: spmv_dispatch<T, kF32Pos, 0>(plan, a, part, s); break;
  }
  HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_spmv_probe(const SpmvPlan& plan, int valmode, const SpmvArgs<T>& a, double* partials,
                       hipStream_t s) {
  if (valmode == kUnitNeg) spmv_dispatch<T, kUnitNeg, 1>(plan, a, partials, s, false);
  else if (valmode == kF64Neg) spmv_dispatch<T, kF64Neg, 1>(plan, a, partials, s, false);
  else spmv_dispatch<T, kF32Neg, 1>(plan, a, partials, s, false);
  HIP_LAUNCH_CHECK();
}
template void launch_spmv_probe<double>(const SpmvPlan&, int, const SpmvArgs<double>&, double*,
                                        hipStream_t);
template void launch_spmv_probe<float>(const SpmvPlan&, int, const SpmvArgs<float>&, double*,
                                       hipStream_t);
template void launch_spmv<double>(const SpmvPlan&, int, const SpmvArgs<double>&, RedBuf,
                                  hipStream_t);
template void launch_spmv<float>(const SpmvPlan&, int, const SpmvArgs<float>&, RedBuf,
                                 hipStream_t);

// ------------------------------------------------------------------ PCG updates

// x += alpha p; r -= alpha (q + delta V-hat t1) with q the product without the deflation
// term and t1 = V-hat^T p, so that V-hat is read once per iteration; partials ||r||^2,
// r^T D^-1 r and V-hat^T (D^-1 r).  The finishing dispatch forms g = G^-1 t2 and rho = r^T z
// (eq. (3.5) makes r^T z = r^T D^-1 r - delta t2^T g), tests convergence and sets beta.
template <typename T, int CM>
__global__ __launch_bounds__(kBlock) void k_pcg_update1(int n, T* __restrict__ x,
                                                        T* __restrict__ r,
                                                        const T* __restrict__ p,
                                                        const T* __restrict__ q,
                                                        const T* __restrict__ dinv,
                                                        const T* __restrict__ V, int64_t ldv,
                                                        int c, const double* Ginv,
                                                        double delta, int trim,
                                                        double sig_over_n, int init,
                                                        DevState* st, double* partials) {
  if (st->done) return;
  constexpr int NV = 2 + (CM > 0 ? CM : 0);
  __shared__ T st1[CM > 0 ? CM : 1];
  if constexpr (CM > 0) {
    for (int j = threadIdx.x; j < CM; j += kBlock) st1[j] = (init || j >= c) ? T(0) : (T)st->t1[j];
    __syncthreads();
  }
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const T alpha = init ? T(0) : (T)st->alpha;
  const T dl = (T)delta;
  const T r1 = init ? T(0) : (T)(sig_over_n * st->sump);  // (sigma/n) 1-hat^T p
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    // all CM columns unconditionally (columns c..CM-1 are finite padding, weighted by 0),
    // so that every load is in flight before the first is used
    T vreg[CM > 0 ? CM : 1];
    T vt = T(0);
#pragma unroll
    for (int j = 0; j < CM; ++j) vreg[j] = V[l + (int64_t)j * ldv];
#pragma unroll
    for (int j = 0; j < CM; ++j) vt += vreg[j] * st1[j];
    T rl = r[l];
    if (!init) {
      x[l] += alpha * p[l];
      rl -= alpha * (q[l] + dl * vt + (l == trim ? T(0) : r1));
      r[l] = rl;
    }
    const T u = dinv[l] * rl;
    acc[0] += (double)rl * (double)rl;
    acc[1] += (double)rl * (double)u;
#pragma unroll
    for (int j = 0; j < CM; ++j) acc[2 + j] += (double)vreg[j] * (double)u;
  }
  write_partials<NV>(acc, 2 + c, partials);
}

// V-hat^T p of the next direction without a pass over V-hat: with z = (I - delta M V-hat
// G^-1 V-hat^T) M r (eq. (3.5)) and G = I + delta V-hat^T M V-hat, V-hat^T z = G^-1 V-hat^T M r
// = g, so V-hat^T (z + beta p) = g + beta V-hat^T p.  Called by the workgroup that has just
// set beta (thread 0) and holds g in LDS; nothing is left to do once the iteration stopped.
__device__ void next_t1(int c, const double* g, int init, DevState* st) {
  __syncthreads();
  if (st->done) return;
  const double beta = init ? 0.0 : st->beta;
  for (int j = threadIdx.x; j < c; j += blockDim.x) st->t1[j] = g[j] + beta * st->t1[j];
}

// Reduces the partials of k_pcg_update1 (one workgroup), forms g = G^-1 t2 and
// rho = r^T M^-1 r - delta t2^T g, tests convergence and sets beta.
__global__ __launch_bounds__(kFin) void k_pcg_fin1(int c, int nblk, const double* partials,
                                                     const double* Ginv, double delta, int init,
                                                     DevState* st) {
  if (st->done) return;
  __shared__ double red[2 + kMaxC];
  __shared__ double gsh[kMaxC];
  final_reduce(partials, 2 + c, nblk, red);
  // g = Ginv t2 (c x c, column-major)
  for (int j = threadIdx.x; j < c; j += blockDim.x) {
    double gj = 0.0;
    for (int i = 0; i < c; ++i) gj += Ginv[j + i * c] * red[2 + i];
    gsh[j] = gj;
    st->g[j] = gj;
    st->t2[j] = red[2 + j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tg = 0.0;
    for (int j = 0; j < c; ++j) tg += red[2 + j] * gsh[j];
    const double rr = red[0];
    const double rho_new = red[1] - delta * tg;
    st->rr = rr;
    st->rmr = red[1];
    if (init) {
      st->rr0 = rr;
      st->thresh2 = st->rtol2 * rr;
      st->rho = rho_new;
      st->beta = 0.0;
      st->it = 0;
      if (!(rr > 0.0)) st->done = 1;
      if (!(rho_new > 0.0) && rr > 0.0) {
        st->done = 1;
        st->status = kPcgBreakdown;
      }
    } else {
      st->it += 1;
      if (!(rr <= st->thresh2)) {
        if (st->it >= st->maxit) {
          st->done = 1;
          st->status = kPcgCapped;
        } else if (!(rho_new > 0.0) || !isfinite(rho_new)) {
          st->done = 1;
          st->status = kPcgBreakdown;
        } else {
          st->beta = rho_new / st->rho;
          st->rho = rho_new;
        }
      } else {
        st->done = 1;
      }
    }
  }
  next_t1(c, gsh, init, st);
}

// z = M^-1 (r - delta V-hat g); p = z + beta p; partial sum(p).
template <typename T, int CM>
__global__ __launch_bounds__(kBlock) void k_pcg_update2(int n, const T* __restrict__ r,
                                                        T* __restrict__ p,
                                                        const T* __restrict__ dinv,
                                                        const T* __restrict__ V, int64_t ldv,
                                                        int c, double delta, int init,
                                                        DevState* st, double* partials) {
  if (st->done) return;
  __shared__ T sg[CM > 0 ? CM : 1];
  for (int j = threadIdx.x; j < CM; j += kBlock) sg[j] = j < c ? (T)st->g[j] : T(0);
  __syncthreads();
  double acc[1] = {0.0};
  const T beta = init ? T(0) : (T)st->beta;
  const T dl = (T)delta;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    T vreg[CM > 0 ? CM : 1];
    T s = T(0);
#pragma unroll
    for (int j = 0; j < CM; ++j) vreg[j] = V[l + (int64_t)j * ldv];
#pragma unroll
    for (int j = 0; j < CM; ++j) s += vreg[j] * sg[j];
    const T z = dinv[l] * (r[l] - dl * s);
    const T pn = init ? z : z + beta * p[l];
    p[l] = pn;
    acc[0] += (double)pn;
  }
  write_partials<1>(acc, 1, partials);
}


#define ISIRA_CM_CASE(L, v) \
  case v:                   \
    L(v);                   \
    break;
#define ISIRA_CM_CASES(L)                                                                    \
  ISIRA_CM_CASE(L, 0) ISIRA_CM_CASE(L, 4) ISIRA_CM_CASE(L, 8) ISIRA_CM_CASE(L, 12)            \
  ISIRA_CM_CASE(L, 16) ISIRA_CM_CASE(L, 20) ISIRA_CM_CASE(L, 24) ISIRA_CM_CASE(L, 32)          \
  ISIRA_CM_CASE(L, 40) ISIRA_CM_CASE(L, 48)                                                    \
  default:                                                                                     \
    L(64);                                                                                     \
    break;

template <typename T>
void launch_pcg_update1(int n, T* x, T* r, const T* p, const T* q, const T* dinv, const T* V,
                        int64_t ldv, int c, const double* Ginv, double delta, int trim,
                        double sig_over_n, int init, DevState* st, RedBuf rb, hipStream_t s) {
  const int grid = stream_grid(n);
#define ISIRA_UPD1(CMV)                                                                   \
  k_pcg_update1<T, CMV><<<grid, kBlock, 0, s>>>(n, x, r, p, q, dinv, V, ldv, c, Ginv, delta, \
                                                trim, sig_over_n, init, st, rb.partials)
  switch (pick_cm(c)) {
    ISIRA_CM_CASES(ISIRA_UPD1)
  }
#undef ISIRA_UPD1
  k_pcg_fin1<<<1, kFin, 0, s>>>(c, grid, rb.partials, Ginv, delta, init, st);
  HIP_LAUNCH_CHECK();
}

// The partials (sum(p), V-hat^T p) are reduced by the next product's finishing dispatch.
template <typename T>
void launch_pcg_update2(int n, const T* r, T* p, const T* dinv, const T* V, int64_t ldv, int c,
                        double delta, int init, DevState* st, RedBuf rb, hipStream_t s) {
  const int grid = stream_grid(n);
#define ISIRA_UPD2(CMV)                                                                   \
  k_pcg_update2<T, CMV><<<grid, kBlock, 0, s>>>(n, r, p, dinv, V, ldv, c, delta, init, st, \
                                                rb.partials)
  switch (pick_cm(c)) {
    ISIRA_CM_CASES(ISIRA_UPD2)
  }
#undef ISIRA_UPD2
  HIP_LAUNCH_CHECK();
}
template void launch_pcg_update1<double>(int, double*, double*, const double*, const double*,
                                         const double*, const double*, int64_t, int,
                                         const double*, double, int, double, int, DevState*,
                                         RedBuf, hipStream_t);
template void launch_pcg_update1<float>(int, float*, float*, const float*, const float*,
                                        const float*, const float*, int64_t, int, const double*,
                                        double, int, double, int, DevState*, RedBuf,
                                        hipStream_t);
template void launch_pcg_update2<double>(int, const double*, double*, const double*,
                                         const double*, int64_t, int, double, int, DevState*,
                                         RedBuf, hipStream_t);
template void launch_pcg_update2<float>(int, const float*, float*, const float*, const float*,
                                        int64_t, int, double, int, DevState*, RedBuf,
                                        hipStream_t);

// ---- preconditioned MINRES (Paige-Saunders) for the indefinite inner systems of a moving
// shift.  One iteration: the product q = (L-hat - sigma I) z with its finishing dispatch
// (delta_j = z^T K-hat z with the deflation and rank-one terms folded in), k_minres_a + its
// finishing dispatch (the next Lanczos vector, gamma_{j+1} and the Givens rotation), and
// k_minres_b (the new direction, the solution update and the next preconditioned vector). ----

// v_new = K-hat z - (delta_j / gamma_j) v_j - (gamma_j / gamma_{j-1}) v_{j-1}, written over
// v_{j-1}; K-hat z = q + delta V-hat t1 + (sigma/n) 1-hat (1-hat^T z) with t1 = V-hat^T z.
// init: v_new = v_1 = vcur (the right-hand side), nothing written.
// Partials ||v||^2, v^T D^-1 v, V-hat^T (D^-1 v).
template <typename T, int CM>
__global__ __launch_bounds__(kBlock) void k_minres_a(int n, const T* __restrict__ q,
                                                     const T* __restrict__ vcur,
                                                     T* __restrict__ vprev,
                                                     const T* __restrict__ dinv,
                                                     const T* __restrict__ V, int64_t ldv,
                                                     int c, double delta, int trim,
                                                     double sig_over_n, int init,
                                                     DevState* st, double* partials) {
  if (st->done) return;
  constexpr int NV = 2 + (CM > 0 ? CM : 0);
  __shared__ T st1[CM > 0 ? CM : 1];
  if constexpr (CM > 0) {
    for (int j = threadIdx.x; j < CM; j += kBlock) st1[j] = j < c ? (T)st->t1[j] : T(0);
    __syncthreads();
  }
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  const double gam = st->rho;
  const T cd = init ? T(0) : (T)(st->pq / gam);
  const T cg = init ? T(0) : (T)(gam / st->mr[0]);
  const T dl = (T)delta;
  const T r1 = init ? T(0) : (T)(sig_over_n * st->sump);
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    T vreg[CM > 0 ? CM : 1];
#pragma unroll
    for (int j = 0; j < CM; ++j) vreg[j] = V[l + (int64_t)j * ldv];
    T vt = T(0);
#pragma unroll
    for (int j = 0; j < CM; ++j) vt += vreg[j] * st1[j];
    T vn = vcur[l];
    if (!init) {
      const T kz = q[l] + dl * vt + (l == trim ? T(0) : r1);
      vn = kz - cd * vn - cg * vprev[l];
      vprev[l] = vn;
    }
    const T u = dinv[l] * vn;
    acc[0] += (double)vn * (double)vn;
    acc[1] += (double)vn * (double)u;
#pragma unroll
    for (int j = 0; j < CM; ++j) acc[2 + j] += (double)vreg[j] * (double)u;
  }
  write_partials<NV>(acc, 2 + c, partials);
}

// Reduces the partials of the Lanczos step (one workgroup): g = G^-1 t2 (eq. (3.5)),
// gamma_{j+1} = sqrt(v^T M^-1 v) = sqrt(v^T D^-1 v - delta t2^T g), then one Givens rotation
// of the tridiagonal QR factorization and the recursively updated residual norm eta; stops
// when |eta| <= rtol eta_0.  V-hat^T z_{j+1} = g / gamma_{j+1} by the SMW identity.
__global__ __launch_bounds__(kFin) void k_minres_fin_a(int c, int nblk, const double* partials,
                                                         const double* Ginv, double delta,
                                                         int init, DevState* st) {
  if (st->done) return;
  __shared__ double red[2 + kMaxC];
  __shared__ double gsh[kMaxC];
  __shared__ double gnew_sh;
  final_reduce(partials, 2 + c, nblk, red);
  for (int j = threadIdx.x; j < c; j += blockDim.x) {
    double gj = 0.0;
    for (int i = 0; i < c; ++i) gj += Ginv[j + i * c] * red[2 + i];
    gsh[j] = gj;
    st->g[j] = gj;
    st->t2[j] = red[2 + j];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tg = 0.0;
    for (int j = 0; j < c; ++j) tg += red[2 + j] * gsh[j];
    const double vmv = red[1] - delta * tg;
    const double gnew = (vmv > 0.0 && isfinite(vmv)) ? sqrt(vmv) : 0.0;
    double* mr = st->mr;
    if (init) {
      mr[0] = 1.0;                  // gamma_0 (multiplies v_0 = 0)
      mr[1] = mr[2] = 1.0;          // c_1, c_0
      mr[3] = mr[4] = 0.0;          // s_1, s_0
      mr[5] = mr[6] = gnew;         // eta, eta_0
      st->rho = gnew;
      st->rr = st->rr0 = gnew * gnew;
      st->thresh2 = st->rtol2 * gnew * gnew;
      st->it = 0;
      st->last_it = -1;
      if (!(gnew > 0.0)) st->done = 1;
    } else {
      const double gam = st->rho, dlt = st->pq;
      const double cj = mr[1], cjm = mr[2], sj = mr[3], sjm = mr[4], eta = mr[5];
      const double a0 = cj * dlt - cjm * sj * gam;
      const double a1 = sqrt(a0 * a0 + gnew * gnew);
      const double a2 = sj * dlt + cjm * cj * gam;
      const double a3 = sjm * gam;
      st->it += 1;
      if (!(a1 > 0.0) || !isfinite(a1) || !isfinite(dlt)) {
        st->done = 1;
        st->status = kPcgBreakdown;
        st->last_it = -1;
      } else {
        const double cn = a0 / a1, sn = gnew / a1;
        mr[2] = cj;
        mr[4] = sj;
        mr[1] = cn;
        mr[3] = sn;
        mr[7] = a1;
        mr[8] = a2;
        mr[9] = a3;
        st->alpha = cn * eta;
        const double etan = -sn * eta;
        mr[5] = etan;
        mr[0] = gam;
        st->rho = gnew;
        st->rr = etan * etan;
        if (etan * etan <= st->thresh2 || !(gnew > 0.0)) {
          st->done = 1;
          st->last_it = st->it;
        } else if (st->it >= st->maxit) {
          st->done = 1;
          st->status = kPcgCapped;
          st->last_it = st->it;
        }
      }
    }
    gnew_sh = gnew;
  }
  __syncthreads();
  const double inv = gnew_sh > 0.0 ? 1.0 / gnew_sh : 0.0;
  for (int j = threadIdx.x; j < c; j += blockDim.x) st->t1[j] = gsh[j] * inv;
}

// w_{j+1} = (z_j - alpha_3 w_{j-1} - alpha_2 w_j) / alpha_1 (written over w_{j-1}),
// x += c_{j+1} eta w_{j+1}, and z_{j+1} = M^-1 v_{j+1} / gamma_{j+1} with eq. (3.5)
// (over z_j); partial sum(z_{j+1}).  Iteration `jit` runs even when the test stopped the
// iteration at jit, to apply its solution update.  init: z_1 only, and w, v_0 cleared.
template <typename T, int CM>
__global__ __launch_bounds__(kBlock) void k_minres_b(int n, T* __restrict__ z,
                                                     T* __restrict__ wprev,
                                                     T* __restrict__ wcur, T* __restrict__ x,
                                                     const T* __restrict__ v,
                                                     T* __restrict__ vzero,
                                                     const T* __restrict__ dinv,
                                                     const T* __restrict__ V, int64_t ldv,
                                                     int c, double delta, int init, int jit,
                                                     DevState* st, double* partials) {
  if (st->done && st->last_it != jit) return;
  __shared__ T sg[CM > 0 ? CM : 1];
  for (int j = threadIdx.x; j < CM; j += kBlock) sg[j] = j < c ? (T)st->g[j] : T(0);
  __syncthreads();
  const double gnew = st->rho;
  const T inv = gnew > 0.0 ? (T)(1.0 / gnew) : T(0);
  const double* mr = st->mr;
  const T ia1 = init ? T(0) : (T)(1.0 / mr[7]);
  const T a2 = init ? T(0) : (T)mr[8];
  const T a3 = init ? T(0) : (T)mr[9];
  const T ceta = init ? T(0) : (T)st->alpha;
  const T dl = (T)delta;
  double acc[1] = {0.0};
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    T vreg[CM > 0 ? CM : 1];
#pragma unroll
    for (int j = 0; j < CM; ++j) vreg[j] = V[l + (int64_t)j * ldv];
    T s = T(0);
#pragma unroll
    for (int j = 0; j < CM; ++j) s += vreg[j] * sg[j];
    if (init) {
      wprev[l] = T(0);
      wcur[l] = T(0);
      vzero[l] = T(0);
    } else {
      const T wn = (z[l] - a3 * wprev[l] - a2 * wcur[l]) * ia1;
      wprev[l] = wn;
      x[l] += ceta * wn;
    }
    const T zn = dinv[l] * (v[l] - dl * s) * inv;
    z[l] = zn;
    acc[0] += (double)zn;
  }
  write_partials<1>(acc, 1, partials);
}

template <typename T>
void launch_minres_a(int n, const T* q, const T* vcur, T* vprev, const T* dinv, const T* V,
                     int64_t ldv, int c, const double* Ginv, double delta, int trim,
                     double sig_over_n, int init, DevState* st, RedBuf rb, hipStream_t s) {
  const int grid = stream_grid(n);
#define ISIRA_MRA(CMV)                                                                       \
  k_minres_a<T, CMV><<<grid, kBlock, 0, s>>>(n, q, vcur, vprev, dinv, V, ldv, c, delta, trim, \
                                             sig_over_n, init, st, rb.partials)
  switch (pick_cm(c)) {
    ISIRA_CM_CASES(ISIRA_MRA)
  }
#undef ISIRA_MRA
  k_minres_fin_a<<<1, kFin, 0, s>>>(c, grid, rb.partials, Ginv, delta, init, st);
  HIP_LAUNCH_CHECK();
}

template <typename T>
void launch_minres_b(int n, T* z, T* wprev, T* wcur, T* x, const T* v, T* vzero, const T* dinv,
                     const T* V, int64_t ldv, int c, double delta, int init, int jit,
                     DevState* st, RedBuf rb, hipStream_t s) {
  const int grid = stream_grid(n);
#define ISIRA_MRB(CMV)                                                                      \
  k_minres_b<T, CMV><<<grid, kBlock, 0, s>>>(n, z, wprev, wcur, x, v, vzero, dinv, V, ldv, c, \
                                             delta, init, jit, st, rb.partials)
  switch (pick_cm(c)) {
    ISIRA_CM_CASES(ISIRA_MRB)
  }
#undef ISIRA_MRB
  HIP_LAUNCH_CHECK();
}
template void launch_minres_a<double>(int, const double*, const double*, double*, const double*,
                                      const double*, int64_t, int, const double*, double, int,
                                      double, int, DevState*, RedBuf, hipStream_t);
template void launch_minres_a<float>(int, const float*, const float*, float*, const float*,
                                     const float*, int64_t, int, const double*, double, int,
                                     double, int, DevState*, RedBuf, hipStream_t);
template void launch_minres_b<double>(int, double*, double*, double*, double*, const double*,
                                      double*, const double*, const double*, int64_t, int,
                                      double, int, int, DevState*, RedBuf, hipStream_t);
template void launch_minres_b<float>(int, float*, float*, float*, float*, const float*, float*,
                                     const float*, const float*, int64_t, int, double, int, int,
                                     DevState*, RedBuf, hipStream_t);

// ---- learned preconditioner variants ----

// x += alpha p; r -= alpha (q + delta V-hat t1) (q without the deflation term, t1 =
// V-hat^T p); partial ||r||^2; the finishing dispatch tests convergence.
template <typename T, int CM>
__global__ __launch_bounds__(kBlock) void k_pcg_update1_plain(
    int n, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
    const T* __restrict__ q, const T* __restrict__ V, int64_t ldv, int c, double delta,
    int trim, double sig_over_n, int init, DevState* st, double* partials) {
  if (st->done) return;
  __shared__ T st1[CM > 0 ? CM : 1];
  if constexpr (CM > 0) {
    for (int j = threadIdx.x; j < CM; j += kBlock) st1[j] = j < c ? (T)st->t1[j] : T(0);
    __syncthreads();
  }
  double acc[1] = {0.0};
  const T alpha = init ? T(0) : (T)st->alpha;
  const T dl = (T)delta;
  const T r1 = init ? T(0) : (T)(sig_over_n * st->sump);  // (sigma/n) 1-hat^T p
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    T rl = r[l];
    if (!init) {
      T vreg[CM > 0 ? CM : 1];
      T vt = T(0);
#pragma unroll
      for (int j = 0; j < CM; ++j) vreg[j] = V[l + (int64_t)j * ldv];
#pragma unroll
      for (int j = 0; j < CM; ++j) vt += vreg[j] * st1[j];
      x[l] += alpha * p[l];
      rl -= alpha * (q[l] + dl * vt + (l == trim ? T(0) : r1));
      r[l] = rl;
    }
    acc[0] += (double)rl * (double)rl;
  }
  write_partials<1>(acc, 1, partials);
}

__global__ __launch_bounds__(kFin) void k_pcg_fin1_plain(int nblk, const double* partials,
                                                           int init, DevState* st) {
  if (st->done) return;
  __shared__ double red[1];
  final_reduce(partials, 1, nblk, red);
  if (threadIdx.x == 0) {
    const double rr = red[0];
    st->rr = rr;
    if (init) {
      st->rr0 = rr;
      st->thresh2 = st->rtol2 * rr;
      st->it = 0;
      if (!(rr > 0.0)) st->done = 1;
    } else {
      st->it += 1;
      if (rr <= st->thresh2) {
        st->done = 1;
      } else if (st->it >= st->maxit) {
        st->done = 1;
        st->status = kPcgCapped;
      } else if (!isfinite(rr)) {
        st->done = 1;
        st->status = kPcgBreakdown;
      }
    }
  }
}

// After y = M r with dots t = V-hat^T y (st->t2[0..c)) and r^T y (st->t2[c]):
// g = G^-1 t, rho = r^T y - delta t^T g, beta.
__global__ void k_spai_finish_rho(int c, const double* Ginv, double delta, int init,
                                  DevState* st) {
  if (st->done) return;
  for (int j = threadIdx.x; j < c; j += blockDim.x) {
    double gj = 0.0;
    for (int i = 0; i < c; ++i) gj += Ginv[j + i * c] * st->t2[i];
    st->g[j] = gj;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tg = 0.0;
    for (int j = 0; j < c; ++j) tg += st->t2[j] * st->g[j];
    const double rho_new = st->t2[c] - delta * tg;
    if (!(rho_new > 0.0) || !isfinite(rho_new)) {
      st->done = 1;
      st->status = kPcgBreakdown;
    } else if (init) {
      st->rho = rho_new;
      st->beta = 0.0;
    } else {
      st->beta = rho_new / st->rho;
      st->rho = rho_new;
    }
  }
  next_t1(c, st->g, init, st);
}

void launch_spai_finish_rho(int c, const double* Ginv, double delta, int init, DevState* st,
                            hipStream_t s) {
  k_spai_finish_rho<<<1, 64, 0, s>>>(c, Ginv, delta, init, st);
  HIP_LAUNCH_CHECK();
}

// z = y - delta Y g; p = z + beta p; partial sum(p).
template <typename T, int CM>
__global__ __launch_bounds__(kBlock) void k_pcg_update2_learned(
    int n, const T* __restrict__ y, T* __restrict__ p, const T* __restrict__ Y, int64_t ldv,
    int c, const T* __restrict__ V, double delta, int init, DevState* st, double* partials) {
  if (st->done) return;
  __shared__ T sg[CM > 0 ? CM : 1];
  for (int j = threadIdx.x; j < CM; j += kBlock) sg[j] = j < c ? (T)st->g[j] : T(0);
  __syncthreads();
  double acc[1] = {0.0};
  const T beta = init ? T(0) : (T)st->beta;
  const T dl = (T)delta;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    T yreg[CM > 0 ? CM : 1];
#pragma unroll
    for (int j = 0; j < CM; ++j) yreg[j] = Y[l + (int64_t)j * ldv];
    T s = T(0);
#pragma unroll
    for (int j = 0; j < CM; ++j) s += yreg[j] * sg[j];
    const T z = y[l] - dl * s;
    const T pn = init ? z : z + beta * p[l];
    p[l] = pn;
    acc[0] += (double)pn;
  }
  write_partials<1>(acc, 1, partials);
}

template <typename T>
void launch_pcg_update1_plain(int n, T* x, T* r, const T* p, const T* q, const T* V,
                              int64_t ldv, int c, double delta, int trim, double sig_over_n,
                              int init, DevState* st, RedBuf rb, hipStream_t s, bool with_fin) {
  const int grid = stream_grid(n);
#define ISIRA_UPD1P(CMV)                                                                  \
  k_pcg_update1_plain<T, CMV><<<grid, kBlock, 0, s>>>(n, x, r, p, q, V, ldv, c, delta, trim, \
                                                      sig_over_n, init, st, rb.partials)
  switch (pick_cm(c)) {
    ISIRA_CM_CASES(ISIRA_UPD1P)
  }
#undef ISIRA_UPD1P
  if (with_fin) k_pcg_fin1_plain<<<1, kFin, 0, s>>>(grid, rb.partials, init, st);
  HIP_LAUNCH_CHECK();
}

// Pruned learned M = diag(mdiag) + the kept off-diagonal entries (CSR prp/pcol/pval, a few
// per row at the thresholds it is meant for): one thread per row.  u = M r; partials
// ||r||^2, r^T u and V-hat^T u in the layout of k_pcg_update1, so that k_pcg_fin1 forms
// g = G^-1 V-hat^T u and rho = r^T u - delta t2^T g (eq. (3.5)) as for Jacobi.  The trimmed
// row has a zero diagonal and no kept entries, so u is 0 there.
template <typename T, int CM>
__global__ __launch_bounds__(kBlock) void k_spai_sparse_step(
    int n, const T* __restrict__ r, T* __restrict__ u, const int32_t* __restrict__ prp,
    const int32_t* __restrict__ pcol, const float* __restrict__ pval,
    const T* __restrict__ mdiag, const T* __restrict__ V, int64_t ldv, int c, DevState* st,
    double* partials) {
  if (st->done) return;
  constexpr int NV = 2 + (CM > 0 ? CM : 0);
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    T vreg[CM > 0 ? CM : 1];
#pragma unroll
    for (int j = 0; j < CM; ++j) vreg[j] = V[l + (int64_t)j * ldv];
    const T rl = r[l];
    const int e0 = prp[l], e1 = prp[l + 1];
    T ul;
    if (e1 - e0 > kSpLongRow) {
      ul = u[l];  // summed by k_spai_long_rows
    } else {
      ul = mdiag[l] * rl;
      for (int e = e0; e < e1; ++e) ul += (T)pval[e] * r[pcol[e]];
      u[l] = ul;
    }
    acc[0] += (double)rl * (double)rl;
    acc[1] += (double)rl * (double)ul;
#pragma unroll
    for (int j = 0; j < CM; ++j) acc[2 + j] += (double)vreg[j] * (double)ul;
  }
  write_partials<NV>(acc, 2 + c, partials);
}

// u[l] = M_ll x[l] + sum of the kept m_lj x[j] for the listed long rows, one wave per row
// (lanes stride over the row, then a wave sum).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_spai_long_rows(int n_long, const int32_t* __restrict__ rows,
                                                           const T* __restrict__ x, T* __restrict__ u,
                                                           const int32_t* __restrict__ prp,
                                                           const int32_t* __restrict__ pcol,
                                                           const float* __restrict__ pval,
                                                           const T* __restrict__ mdiag,
                                                           const DevState* skip) {
  if (skip && skip->done) return;
  const int lane = threadIdx.x & 63;
  const int nw = (gridDim.x * kBlock) >> 6;
  for (int w = (blockIdx.x * kBlock + threadIdx.x) >> 6; w < n_long; w += nw) {
    const int l = rows[w];
    T acc = T(0);
    const int e1 = prp[l + 1];
    for (int e = prp[l] + lane; e < e1; e += 64) acc += (T)pval[e] * x[pcol[e]];
    acc = wave_sum(acc);
    if (lane == 0) u[l] = mdiag[l] * x[l] + acc;
  }
}

template <typename T>
static void launch_long_rows(int n_long, const int32_t* rows, const T* x, T* u, const int32_t* prp,
                             const int32_t* pcol, const float* pval, const T* mdiag,
                             const DevState* skip, hipStream_t s) {
  if (n_long <= 0) return;
  int grid = (n_long + kBlock / 64 - 1) / (kBlock / 64);
  if (grid > kStreamGrid) grid = kStreamGrid;
  k_spai_long_rows<T><<<grid, kBlock, 0, s>>>(n_long, rows, x, u, prp, pcol, pval, mdiag, skip);
}

template <typename T>
void launch_spai_sparse_step(int n, const T* r, T* u, const int32_t* prp, const int32_t* pcol,
                             const float* pval, const T* mdiag, const int32_t* plong, int n_long,
                             const T* V, int64_t ldv, int c, const double* Ginv, double delta,
                             int init, DevState* st, RedBuf rb, hipStream_t s) {
  const int grid = stream_grid(n);
  launch_long_rows<T>(n_long, plong, r, u, prp, pcol, pval, mdiag, st, s);
#define ISIRA_SPSTEP(CMV)                                                                    \
  k_spai_sparse_step<T, CMV><<<grid, kBlock, 0, s>>>(n, r, u, prp, pcol, pval, mdiag, V, ldv, c, \
                                                     st, rb.partials)
  switch (pick_cm(c)) {
    ISIRA_CM_CASES(ISIRA_SPSTEP)
  }
#undef ISIRA_SPSTEP
  k_pcg_fin1<<<1, kFin, 0, s>>>(c, grid, rb.partials, Ginv, delta, init, st);
  HIP_LAUNCH_CHECK();
}
template void launch_spai_sparse_step<double>(int, const double*, double*, const int32_t*,
                                              const int32_t*, const float*, const double*,
                                              const int32_t*, int, const double*, int64_t, int,
                                              const double*, double, int, DevState*, RedBuf,
                                              hipStream_t);
template void launch_spai_sparse_step<float>(int, const float*, float*, const int32_t*,
                                             const int32_t*, const float*, const float*,
                                             const int32_t*, int, const float*, int64_t, int,
                                             const double*, double, int, DevState*, RedBuf,
                                             hipStream_t);

template <typename T>
__global__ __launch_bounds__(kBlock) void k_spai_sparse_mv(int n, const T* __restrict__ x,
                                                           T* __restrict__ y,
                                                           const int32_t* __restrict__ prp,
                                                           const int32_t* __restrict__ pcol,
                                                           const float* __restrict__ pval,
                                                           const T* __restrict__ mdiag,
                                                           const DevState* skip) {
  if (skip && skip->done) return;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    const int e0 = prp[l], e1 = prp[l + 1];
    if (e1 - e0 > kSpLongRow) continue;  // summed by k_spai_long_rows
    T yl = mdiag[l] * x[l];
    for (int e = e0; e < e1; ++e) yl += (T)pval[e] * x[pcol[e]];
    y[l] = yl;
  }
}

template <typename T>
void launch_spai_sparse_mv(int n, const T* x, T* y, const int32_t* prp, const int32_t* pcol,
                           const float* pval, const T* mdiag, const int32_t* plong, int n_long,
                           const DevState* skip_if_done, hipStream_t s) {
  launch_long_rows<T>(n_long, plong, x, y, prp, pcol, pval, mdiag, skip_if_done, s);
  k_spai_sparse_mv<T><<<stream_grid(n), kBlock, 0, s>>>(n, x, y, prp, pcol, pval, mdiag,
                                                        skip_if_done);
  HIP_LAUNCH_CHECK();
}
template void launch_spai_sparse_mv<double>(int, const double*, double*, const int32_t*,
                                            const int32_t*, const float*, const double*,
                                            const int32_t*, int, const DevState*, hipStream_t);
template void launch_spai_sparse_mv<float>(int, const float*, float*, const int32_t*,
                                           const int32_t*, const float*, const float*,
                                           const int32_t*, int, const DevState*, hipStream_t);
// The partials (sum(p), V-hat^T p) are reduced by the next product's finishing dispatch.
template <typename T>
void launch_pcg_update2_learned(int n, const T* y, T* p, const T* Y, int64_t ldv, int c,
                                const T* V, double delta, int init, DevState* st, RedBuf rb,
                                hipStream_t s) {
  const int grid = stream_grid(n);
#define ISIRA_UPD2L(CMV)                                                                    \
  k_pcg_update2_learned<T, CMV><<<grid, kBlock, 0, s>>>(n, y, p, Y, ldv, c, V, delta, init, st, \
                                                        rb.partials)
  switch (pick_cm(c)) {
    ISIRA_CM_CASES(ISIRA_UPD2L)
  }
#undef ISIRA_UPD2L
  HIP_LAUNCH_CHECK();
}
template void launch_pcg_update1_plain<double>(int, double*, double*, const double*,
                                               const double*, const double*, int64_t, int,
                                               double, int, double, int, DevState*, RedBuf,
                                               hipStream_t, bool);
template void launch_pcg_update1_plain<float>(int, float*, float*, const float*, const float*,
                                              const float*, int64_t, int, double, int, double,
                                              int, DevState*, RedBuf, hipStream_t, bool);
template void launch_pcg_update2_learned<double>(int, const double*, double*, const double*,
                                                 int64_t, int, const double*, double, int,
                                                 DevState*, RedBuf, hipStream_t);
template void launch_pcg_update2_learned<float>(int, const float*, float*, const float*,
                                                int64_t, int, const float*, double, int,
                                                DevState*, RedBuf, hipStream_t);

// ------------------------------------------------------------------ right-hand side, enlarge

// r_in = trim(r - mean) in the inner precision (entry `trim` is 0); x = 0.  The mean is
// `mean`, or *mean_sum * inv_n when mean_sum is given (a sum left on the device).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_rhs_prep(int n, const double* __restrict__ r64,
                                                     double mean, const double* mean_sum,
                                                     double inv_n, int trim,
                                                     T* __restrict__ rin, T* __restrict__ x) {
  const double mu = mean_sum ? *mean_sum * inv_n : mean;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    rin[l] = (l == trim) ? T(0) : (T)(r64[l] - mu);
    x[l] = T(0);
  }
}
template <typename T>
void launch_rhs_prep(int n, const double* r64, double mean, const double* mean_sum,
                     double inv_n, int trim, T* rin, T* x, hipStream_t s) {
  k_rhs_prep<T><<<stream_grid(n), kBlock, 0, s>>>(n, r64, mean, mean_sum, inv_n, trim, rin, x);
  HIP_LAUNCH_CHECK();
}
template void launch_rhs_prep<double>(int, const double*, double, const double*, double, int,
                                      double*, double*, hipStream_t);
template void launch_rhs_prep<float>(int, const double*, double, const double*, double, int,
                                     float*, float*, hipStream_t);

// Resets the inner-iteration fields of the device state (the generic outputs red[] are
// kept: they may hold the Ritz residual the right-hand side is built from).
__global__ void k_pcg_reset(DevState* st, double rtol2, int maxit) {
  const int t = threadIdx.x;
  for (int j = t; j < kMaxC; j += blockDim.x) {
    st->t1[j] = 0.0;
    st->g[j] = 0.0;
  }
  for (int j = t; j < kMaxC + 1; j += blockDim.x) st->t2[j] = 0.0;
  if (t == 0) {
    st->alpha = st->beta = st->rho = st->pq = st->rr = st->rr0 = st->rmr = 0.0;
    st->thresh2 = 0.0;
    st->rtol2 = rtol2;
    st->sump = st->sumx = 0.0;
    st->it = 0;
    st->done = 0;
    st->status = 0;
    st->maxit = maxit;
  }
}
void launch_pcg_reset(DevState* st, double rtol2, int maxit, hipStream_t s) {
  k_pcg_reset<<<1, 64, 0, s>>>(st, rtol2, maxit);
  HIP_LAUNCH_CHECK();
}

// eq. (2.5): z = x - (1^T x / n) 1, in FP64 (x carries the trimmed zero in place).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sum(int n, const T* __restrict__ x,
                                                DevState* st, double* partials) {
  double acc[1] = {0.0};
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    acc[0] += (double)x[l];
  write_partials<1>(acc, 1, partials);
}
__global__ __launch_bounds__(kFin) void k_sum_fin(int nblk, const double* partials,
                                                    DevState* st) {
  __shared__ double red[1];
  final_reduce(partials, 1, nblk, red);
  if (threadIdx.x == 0) st->sumx = red[0];
}
template <typename T>
__global__ __launch_bounds__(kBlock) void k_enlarge(int n, const T* __restrict__ x,
                                                    double* __restrict__ z, const DevState* st) {
  const double mean = st->sumx / (double)n;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    z[l] = (double)x[l] - mean;
}
template <typename T>
void launch_enlarge(int n, const T* x, double* z, DevState* st, RedBuf rb, hipStream_t s) {
  const int grid = stream_grid(n);
  k_sum<T><<<grid, kBlock, 0, s>>>(n, x, st, rb.partials);
  k_sum_fin<<<1, kFin, 0, s>>>(grid, rb.partials, st);
  k_enlarge<T><<<grid, kBlock, 0, s>>>(n, x, z, st);
  HIP_LAUNCH_CHECK();
}
template void launch_enlarge<double>(int, const double*, double*, DevState*, RedBuf,
                                     hipStream_t);
template void launch_enlarge<float>(int, const float*, double*, DevState*, RedBuf, hipStream_t);

// ------------------------------------------------------------------ column dots, updates

// h_j = sum_l A[l,j] w_l z_l (j < na), then B's columns, then sum(z), then z^T z.  Tiles of
// kTile rows are staged in LDS; each wave owns a set of columns, so the per-workgroup sums
// need no atomics.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_multidot(int n, const T* __restrict__ A,
                                                     int64_t lda, int na,
                                                     const T* __restrict__ B, int64_t ldb,
                                                     int nb, const T* __restrict__ z,
                                                     const T* __restrict__ wz, int with_sum,
                                                     int with_self, double* h,
                                                     double* partials, const int32_t* skip) {
  if (skip && *skip) return;
  __shared__ T zt[kTile];
  __shared__ double acc[kMaxCols];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int ncol = na + nb;
  const int nv = ncol + with_sum + with_self;
  for (int v = tid; v < nv; v += kBlock) acc[v] = 0.0;
  const int ntiles = (n + kTile - 1) / kTile;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int base = tile * kTile;
    const int len = (n - base) < kTile ? (n - base) : kTile;
    __syncthreads();
    for (int i = tid; i < len; i += kBlock) {
      T zz = z[base + i];
      if (wz) zz *= wz[base + i];
      zt[i] = zz;
    }
    __syncthreads();
    // columns j = wid + 4 i; four of them in flight per wave
    int j = wid;
    for (; j + 12 < ncol; j += 16) {
      const T* c0 = (j < na) ? A + (int64_t)j * lda + base : B + (int64_t)(j - na) * ldb + base;
      const int j1 = j + 4, j2 = j + 8, j3 = j + 12;
      const T* c1 = (j1 < na) ? A + (int64_t)j1 * lda + base : B + (int64_t)(j1 - na) * ldb + base;
      const T* c2 = (j2 < na) ? A + (int64_t)j2 * lda + base : B + (int64_t)(j2 - na) * ldb + base;
      const T* c3 = (j3 < na) ? A + (int64_t)j3 * lda + base : B + (int64_t)(j3 - na) * ldb + base;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      for (int i = lane; i < len; i += 64) {
        const double zz = (double)zt[i];
        s0 += (double)c0[i] * zz;
        s1 += (double)c1[i] * zz;
        s2 += (double)c2[i] * zz;
        s3 += (double)c3[i] * zz;
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      s2 = wave_sum(s2);
      s3 = wave_sum(s3);
      if (lane == 0) {
        acc[j] += s0;
        acc[j1] += s1;
        acc[j2] += s2;
        acc[j3] += s3;
      }
    }
    for (; j < nv; j += 4) {
      double s = 0.0;
      if (j < ncol) {
        const T* colp = (j < na) ? A + (int64_t)j * lda + base : B + (int64_t)(j - na) * ldb + base;
        for (int i = lane; i < len; i += 64) s += (double)colp[i] * (double)zt[i];
      } else if (with_sum && j == ncol) {
        for (int i = lane; i < len; i += 64) s += (double)zt[i];
      } else {
        for (int i = lane; i < len; i += 64) s += (double)zt[i] * (double)zt[i];
      }
      s = wave_sum(s);
      if (lane == 0) acc[j] += s;
    }
  }
  __syncthreads();
  for (int v = tid; v < nv; v += kBlock) partials[(size_t)v * gridDim.x + blockIdx.x] = acc[v];
}

// h[v] = sum over workgroups of partials[v * nblk + b]; one wave per value, fixed order.
__global__ __launch_bounds__(64) void k_values_fin(int nv, int nblk, const double* partials,
                                                   double* h, const int32_t* skip = nullptr) {
  if (skip && *skip) return;
  const int v = blockIdx.x;
  if (v >= nv) return;
  const double* pv = partials + (size_t)v * nblk;
  double s = 0.0;
  int b = threadIdx.x;
  for (; b + 7 * 64 < nblk; b += 8 * 64) {  // eight loads in flight, summed in a fixed order
    double t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = pv[b + i * 64];
#pragma unroll
    for (int i = 0; i < 8; ++i) s += t[i];
  }
  for (; b < nblk; b += 64) s += pv[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) h[v] = s;
}

template <typename T>
void launch_multidot(int n, const T* A, int64_t lda, int na, const T* B, int64_t ldb, int nb,
                     const T* z, const T* wz, int with_sum, int with_self, double* h, RedBuf rb,
                     hipStream_t s, const int32_t* skip_if_done) {
  int grid = (n + kTile - 1) / kTile;
  if (grid > kStreamGrid) grid = kStreamGrid;
  k_multidot<T><<<grid, kBlock, 0, s>>>(n, A, lda, na, B, ldb, nb, z, wz, with_sum, with_self,
                                        h, rb.partials, skip_if_done);
  const int nv = na + nb + with_sum + with_self;
  k_values_fin<<<nv, 64, 0, s>>>(nv, grid, rb.partials, h, skip_if_done);
  HIP_LAUNCH_CHECK();
}
template void launch_multidot<double>(int, const double*, int64_t, int, const double*, int64_t,
                                      int, const double*, const double*, int, int, double*,
                                      RedBuf, hipStream_t, const int32_t*);
template void launch_multidot<float>(int, const float*, int64_t, int, const float*, int64_t, int,
                                     const float*, const float*, int, int, double*, RedBuf,
                                     hipStream_t, const int32_t*);

// z -= A hA + B hB (+ h_sum / n); optional ||z||^2 -> st->red[2].
__global__ __launch_bounds__(kBlock) void k_gemv_sub(int n, const double* __restrict__ A,
                                                     int64_t lda, int na,
                                                     const double* __restrict__ B, int64_t ldb,
                                                     int nb, const double* __restrict__ h,
                                                     int with_sum, double* __restrict__ z,
                                                     int with_norm, DevState* st,
                                                     double* partials, const int32_t* skip) {
  if (skip && *skip) return;
  __shared__ double sh[kMaxCols];
  const int ncol = na + nb;
  for (int v = threadIdx.x; v < ncol + with_sum; v += kBlock) sh[v] = h[v];
  __syncthreads();
  const double mean = with_sum ? sh[ncol] / (double)n : 0.0;
  double acc[1] = {0.0};
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    double s = 0.0;
    for (int j = 0; j < na; ++j) s += A[l + (int64_t)j * lda] * sh[j];
    for (int j = 0; j < nb; ++j) s += B[l + (int64_t)j * ldb] * sh[na + j];
    const double zl = z[l] - s - mean;
    z[l] = zl;
    acc[0] += zl * zl;
  }
  if (!with_norm) return;
  write_partials<1>(acc, 1, partials);
}

void launch_gemv_sub(int n, const double* A, int64_t lda, int na, const double* B, int64_t ldb,
                     int nb, const double* h, int with_sum, double* z, int with_norm,
                     DevState* st, RedBuf rb, hipStream_t s, const int32_t* skip) {
  k_gemv_sub<<<stream_grid(n), kBlock, 0, s>>>(n, A, lda, na, B, ldb, nb, h, with_sum, z,
                                               with_norm, st, rb.partials, skip);
  if (with_norm)
    k_values_fin<<<1, 64, 0, s>>>(1, stream_grid(n), rb.partials, st->red + 2, skip);
  HIP_LAUNCH_CHECK();
}

__global__ void k_dgks_decide(const double* h0sq, DevState* st) {
  if (threadIdx.x == 0) st->cgs_skip = (st->red[2] >= 0.5 * h0sq[0]) ? 1 : 0;
}
void launch_dgks_decide(const double* h0sq, DevState* st, hipStream_t s) {
  k_dgks_decide<<<1, 64, 0, s>>>(h0sq, st);
  HIP_LAUNCH_CHECK();
}

// (z and u may be the same vector)
__global__ __launch_bounds__(kBlock) void k_scale(int n, const double* z, double scale, double* u) {
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    u[l] = z[l] * scale;
}
void launch_scale(int n, const double* z, double scale, double* u, hipStream_t s) {
  k_scale<<<stream_grid(n), kBlock, 0, s>>>(n, z, scale, u);
  HIP_LAUNCH_CHECK();
}

// u = z / sqrt(*nrm2) with the squared norm left on the device (u = 0 when it is not > 0).
// (z and u may be the same vector: each entry is read before it is written, by one thread)
__global__ __launch_bounds__(kBlock) void k_scale_dev(int n, const double* z, const double* nrm2,
                                                      double* u) {
  const double v = *nrm2;
  const double sc = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    u[l] = z[l] * sc;
}
void launch_scale_dev(int n, const double* z, const double* nrm2, double* u, hipStream_t s) {
  k_scale_dev<<<stream_grid(n), kBlock, 0, s>>>(n, z, nrm2, u);
  HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ Ritz vectors, residuals

// r = W s - theta U s; partials ||r||^2 -> st->red[0], sum(r) -> st->red[1].
__global__ __launch_bounds__(kBlock) void k_ritz_residual(int n, const double* __restrict__ U,
                                                          const double* __restrict__ W,
                                                          int64_t ld, int k,
                                                          const double* __restrict__ svec,
                                                          double theta, double* __restrict__ r,
                                                          DevState* st, double* partials) {
  __shared__ double sh[ISIRA_MAX_BASIS];
  for (int j = threadIdx.x; j < k; j += kBlock) sh[j] = svec[j];
  __syncthreads();
  double acc[2] = {0.0, 0.0};
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    double y = 0.0, ly = 0.0;
    for (int j = 0; j < k; ++j) {
      y += U[l + (int64_t)j * ld] * sh[j];
      ly += W[l + (int64_t)j * ld] * sh[j];
    }
    const double rl = ly - theta * y;
    r[l] = rl;
    acc[0] += rl * rl;
    acc[1] += rl;
  }
  write_partials<2>(acc, 2, partials);
}
void launch_ritz_residual(int n, const double* U, const double* W, int64_t ld, int k,
                          const double* svec, double theta, double* r, DevState* st, RedBuf rb,
                          hipStream_t s) {
  k_ritz_residual<<<stream_grid(n), kBlock, 0, s>>>(n, U, W, ld, k, svec, theta, r, st,
                                                    rb.partials);
  k_values_fin<<<2, 64, 0, s>>>(2, stream_grid(n), rb.partials, st->red);
  HIP_LAUNCH_CHECK();
}

__global__ __launch_bounds__(kBlock) void k_ritz_vector(int n, const double* __restrict__ U,
                                                        int64_t ld, int k,
                                                        const double* __restrict__ svec,
                                                        double* __restrict__ y) {
  __shared__ double sh[ISIRA_MAX_BASIS];
  for (int j = threadIdx.x; j < k; j += kBlock) sh[j] = svec[j];
  __syncthreads();
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock) {
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += U[l + (int64_t)j * ld] * sh[j];
    y[l] = s;
  }
}
void launch_ritz_vector(int n, const double* U, int64_t ld, int k, const double* svec,
                        double* y, hipStream_t s) {
  k_ritz_vector<<<stream_grid(n), kBlock, 0, s>>>(n, U, ld, k, svec, y);
  HIP_LAUNCH_CHECK();
}

// U[:, 0:q] = U[:, 0:k] S in place, with S (k x q) stored row by row (St[i * q + j] = S(i, j)).
// Each workgroup stages a tile of 64 rows of U column-major in LDS (lane = row: conflict-free);
// each wave then forms eight output columns at a time.  The wave index is made provably
// uniform, so the eight entries S(i, j0:j0+8) of a row of S are one scalar load and every
// LDS read feeds eight FMAs.  All reads of a tile precede its writes, so the update is in place.
constexpr int kTsRows = 64;
constexpr int kTsCw = 8;
constexpr size_t kTsMfmaLds = 128 * 1024;  // LDS bytes of the matrix-core form's copy of S
__global__ __launch_bounds__(kBlock) void k_tsgemm_inplace(int n, double* __restrict__ U,
                                                           int64_t ld, int k,
                                                           const double* __restrict__ St,
                                                           int q) {
  extern __shared__ double ut[];  // k * kTsRows
  const int r = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntiles = (n + kTsRows - 1) / kTsRows;
  const int ngroups = (q + kTsCw - 1) / kTsCw;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int base = tile * kTsRows;
    const bool ok = base + r < n;
    __syncthreads();
    // eight columns in flight per wave
    for (int i0 = w; i0 < k; i0 += 32) {
      double t[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const int i = i0 + 4 * b;
        t[b] = (ok && i < k) ? U[base + r + (int64_t)i * ld] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < 8; ++b)
        if (i0 + 4 * b < k) ut[(i0 + 4 * b) * kTsRows + r] = t[b];
    }
    __syncthreads();
    for (int g = w; g < ngroups; g += 4) {
      const int j0 = g * kTsCw;
      double a[kTsCw];
#pragma unroll
      for (int jj = 0; jj < kTsCw; ++jj) a[jj] = 0.0;
      if (j0 + kTsCw <= q) {
#pragma unroll 4
        for (int i = 0; i < k; ++i) {
          const double u = ut[i * kTsRows + r];
          const double* sr = St + (int64_t)i * q + j0;
#pragma unroll
          for (int jj = 0; jj < kTsCw; ++jj) a[jj] += u * sr[jj];
        }
      } else {
        const int nj = q - j0;
        for (int i = 0; i < k; ++i) {
          const double u = ut[i * kTsRows + r];
          const double* sr = St + (int64_t)i * q + j0;
#pragma unroll
          for (int jj = 0; jj < kTsCw; ++jj)
            if (jj < nj) a[jj] += u * sr[jj];
        }
      }
      if (ok) {
#pragma unroll
        for (int jj = 0; jj < kTsCw; ++jj)
          if (j0 + jj < q) U[base + r + (int64_t)(j0 + jj) * ld] = a[jj];
      }
    }
  }
}
// The same product on the FP64 matrix cores.  S, zero-padded to kp = k rounded up to 4 rows
// and QP = NT * 16 columns, is staged once per workgroup in LDS.  A wave owns 16 rows of U
// and every output column: with the transposed product (U S)^T = S^T U^T, one
// v_mfma_f64_16x16x4 takes A = a 16 x 4 block of S^T from LDS (lane l: S(i0 + l/16,
// 16u + l%16)) and B = a 4 x 16 block of U^T (lane l: U(16t + l%16, i0 + l/16): four 128-byte
// row segments), and adds into the 16 x 16 block u of (U S)^T, whose lane l holds entries
// (16u + 4j + l/16, 16t + l%16), j = 0..3 -- so every store writes whole 128-byte segments.
// The B blocks of the next four k-steps are loaded while the current four are multiplied.
// A wave reads its 16 rows
// of all k columns before it writes any of them and no other wave touches those rows, so
// the update is in place.
typedef double dbl4 __attribute__((ext_vector_type(4)));
template <int NT, int THREADS>
__global__ __launch_bounds__(THREADS) void k_tsgemm_mfma(int n, double* U, int64_t ld, int k,
                                                         const double* __restrict__ St, int q) {
  extern __shared__ double sS[];
  constexpr int QP = NT * 16;
  const int kp = (k + 3) & ~3;
  for (int e = threadIdx.x; e < kp * QP; e += THREADS) {
    const int i = e / QP, j = e - i * QP;
    sS[e] = (i < k && j < q) ? St[(int64_t)i * q + j] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, c = lane & 15;
  constexpr int WPB = THREADS / 64;
  const int ntiles = (n + 15) >> 4;
  for (int t = blockIdx.x * WPB + (threadIdx.x >> 6); t < ntiles; t += gridDim.x * WPB) {
    const int row = t * 16 + c;
    const bool rok = row < n;
    const double* ur = U + row;
    dbl4 acc[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
    // B blocks of four k-steps (16 columns of U) are loaded together, one group ahead
    double bc[4], bn[4];
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int i = 4 * st + g;
      bc[st] = (rok && i < k) ? ur[(int64_t)i * ld] : 0.0;
    }
    for (int i0 = 0; i0 < kp; i0 += 16) {
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int i = i0 + 16 + 4 * st + g;
        bn[st] = (rok && i < k) ? ur[(int64_t)i * ld] : 0.0;
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        if (i0 + 4 * st < kp) {
          const double* srow = sS + (i0 + 4 * st + g) * QP + c;
#pragma unroll
          for (int u = 0; u < NT; ++u)
            acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(srow[u * 16], bc[st], acc[u], 0, 0, 0);
        }
      }
#pragma unroll
      for (int st = 0; st < 4; ++st) bc[st] = bn[st];
    }
    if (rok) {
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = u * 16 + 4 * j + g;
          if (col < q) U[row + (int64_t)col * ld] = acc[u][j];
        }
    }
  }
}

// More than four 16-column tiles: the tiles are shared out among G waves per 16-row tile
// (NTW tiles each, so that accumulators and S fragments stay within the registers of a
// 1024-thread workgroup); the G waves of a row tile sit in one workgroup, and a barrier
// between the multiplications and the stores keeps every read of U before any write.
template <int NTW, int G>
__global__ __launch_bounds__(1024) void k_tsgemm_mfma_g(int n, double* U, int64_t ld, int k,
                                                        const double* __restrict__ St, int q) {
  extern __shared__ double sS[];
  constexpr int QP = NTW * G * 16;
  constexpr int RT = 16 / G;  // row tiles per workgroup and round (16 waves, RT * G used)
  const int kp = (k + 3) & ~3;
  for (int e = threadIdx.x; e < kp * QP; e += 1024) {
    const int i = e / QP, j = e - i * QP;
    sS[e] = (i < k && j < q) ? St[(int64_t)i * q + j] : 0.0;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, c = lane & 15;
  const int rt = wave / G, cg = wave - rt * G;
  const bool active = rt < RT;
  const int ntiles = (n + 15) >> 4;
  for (int base = blockIdx.x * RT; base < ntiles; base += gridDim.x * RT) {
    const int t = base + rt;
    const int row = t * 16 + c;
    const bool rok = active && t < ntiles && row < n;
    const double* ur = U + row;
    dbl4 acc[NTW];
#pragma unroll
    for (int u = 0; u < NTW; ++u) acc[u] = dbl4{0.0, 0.0, 0.0, 0.0};
    if (active && t < ntiles) {
      double bc[4], bn[4];
#pragma unroll
      for (int st = 0; st < 4; ++st) {
        const int i = 4 * st + g;
        bc[st] = (rok && i < k) ? ur[(int64_t)i * ld] : 0.0;
      }
      for (int i0 = 0; i0 < kp; i0 += 16) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          const int i = i0 + 16 + 4 * st + g;
          bn[st] = (rok && i < k) ? ur[(int64_t)i * ld] : 0.0;
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          if (i0 + 4 * st < kp) {
            const double* srow = sS + (i0 + 4 * st + g) * QP + cg * NTW * 16 + c;
#pragma unroll
            for (int u = 0; u < NTW; ++u)
              acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(srow[u * 16], bc[st], acc[u], 0, 0, 0);
          }
        }
#pragma unroll
        for (int st = 0; st < 4; ++st) bc[st] = bn[st];
      }
    }
    __syncthreads();  // every wave of these row tiles has read its rows of U
    if (rok) {
#pragma unroll
      for (int u = 0; u < NTW; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = (cg * NTW + u) * 16 + 4 * j + g;
          if (col < q) U[row + (int64_t)col * ld] = acc[u][j];
        }
    }
  }
}

template <int NTW, int G>
static void launch_tsgemm_mfma_g(int n, double* U, int64_t ld, int k, const double* St, int q,
                                 size_t lds, hipStream_t s) {
  // set on every call (rotations are rare): the attribute is per device, and a process may
  // drive several; a failure shows as the launch's error
  (void)hipFuncSetAttribute((const void*)k_tsgemm_mfma_g<NTW, G>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTsMfmaLds);
  constexpr int RT = 16 / G;
  int grid = (((n + 15) >> 4) + RT - 1) / RT;
  if (grid > 1024) grid = 1024;
  k_tsgemm_mfma_g<NTW, G><<<grid, 1024, lds, s>>>(n, U, ld, k, St, q);
}

template <int NT>
static void launch_tsgemm_mfma_nt(int n, double* U, int64_t ld, int k, const double* St, int q,
                                  size_t lds, hipStream_t s) {
  constexpr int TH = 1024;  // up to four tiles: accumulators and S fragments fit
  (void)hipFuncSetAttribute((const void*)k_tsgemm_mfma<NT, TH>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTsMfmaLds);
  int grid = (((n + 15) >> 4) + (TH / 64) - 1) / (TH / 64);
  if (grid > 1024) grid = 1024;
  k_tsgemm_mfma<NT, TH><<<grid, TH, lds, s>>>(n, U, ld, k, St, q);
}

void launch_tsgemm_inplace(int n, double* U, int64_t ld, int k, const double* St, int q,
                           hipStream_t s) {
  const int nt = (q + 15) / 16;
  // tiles covered: nt itself up to 4; else NTW tiles for each of G waves per row tile
  const int ntw = nt <= 4 ? nt : ((nt == 5 || nt == 6 || nt == 9) ? 3 : 4);
  const int grp = nt <= 4 ? 1 : (nt <= 8 ? 2 : 3);
  const size_t lds = (size_t)((k + 3) & ~3) * ntw * grp * 16 * sizeof(double);
  if (lds <= kTsMfmaLds) {
    switch (nt) {
      case 1: launch_tsgemm_mfma_nt<1>(n, U, ld, k, St, q, lds, s); break;
      case 2: launch_tsgemm_mfma_nt<2>(n, U, ld, k, St, q, lds, s); break;
      case 3: launch_tsgemm_mfma_nt<3>(n, U, ld, k, St, q, lds, s); break;
      case 4: launch_tsgemm_mfma_nt<4>(n, U, ld, k, St, q, lds, s); break;
      case 5:
      case 6: launch_tsgemm_mfma_g<3, 2>(n, U, ld, k, St, q, lds, s); break;
      case 7:
      case 8: launch_tsgemm_mfma_g<4, 2>(n, U, ld, k, St, q, lds, s); break;
      case 9: launch_tsgemm_mfma_g<3, 3>(n, U, ld, k, St, q, lds, s); break;
      default: launch_tsgemm_mfma_g<4, 3>(n, U, ld, k, St, q, lds, s); break;
    }
    HIP_LAUNCH_CHECK();
    return;
  }
  // S too large for the LDS of one workgroup (k and q both near ISIRA_MAX_BASIS)
  int grid = (n + kTsRows - 1) / kTsRows;
  if (grid > 2048) grid = 2048;
  // k <= 192 needs up to 96 KB of dynamic LDS (set on every call, as above)
  (void)hipFuncSetAttribute((const void*)k_tsgemm_inplace,
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            ISIRA_MAX_BASIS * kTsRows * (int)sizeof(double));
  k_tsgemm_inplace<<<grid, kBlock, (size_t)k * kTsRows * sizeof(double), s>>>(n, U, ld, k, St, q);
  HIP_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ small elementwise helpers

template <typename T>
__global__ __launch_bounds__(kBlock) void k_masked_copy(int n, const double* __restrict__ src,
                                                        int trim, T* __restrict__ dst) {
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    dst[l] = (l == trim) ? T(0) : (T)src[l];
}
template <typename T>
void launch_masked_copy(int n, const double* src, int trim, T* dst, hipStream_t s) {
  k_masked_copy<T><<<stream_grid(n), kBlock, 0, s>>>(n, src, trim, dst);
  HIP_LAUNCH_CHECK();
}
template void launch_masked_copy<double>(int, const double*, int, double*, hipStream_t);
template void launch_masked_copy<float>(int, const double*, int, float*, hipStream_t);

// Jacobi part of Remark 3.2: M-hat_sigma^{-1} = 1 / (d - sigma), with 0 at the trimmed row.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_dinv(int n, const double* __restrict__ d,
                                                 double sigma, int trim, T* __restrict__ dinv) {
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    dinv[l] = (l == trim) ? T(0) : (T)(1.0 / (d[l] - sigma));
}
template <typename T>
void launch_dinv(int n, const double* d, double sigma, int trim, T* dinv, hipStream_t s) {
  k_dinv<T><<<stream_grid(n), kBlock, 0, s>>>(n, d, sigma, trim, dinv);
  HIP_LAUNCH_CHECK();
}
template void launch_dinv<double>(int, const double*, double, int, double*, hipStream_t);
template void launch_dinv<float>(int, const double*, double, int, float*, hipStream_t);

// dst[l] = src[idx[l]]
template <typename Ts, typename Td>
__global__ __launch_bounds__(kBlock) void k_gather(int n, const Ts* __restrict__ src,
                                                   const int32_t* __restrict__ idx,
                                                   Td* __restrict__ dst) {
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    dst[l] = (Td)src[idx[l]];
}
template <typename Ts, typename Td>
void launch_gather(int n, const Ts* src, const int32_t* idx, Td* dst, hipStream_t s) {
  k_gather<Ts, Td><<<stream_grid(n), kBlock, 0, s>>>(n, src, idx, dst);
  HIP_LAUNCH_CHECK();
}
template void launch_gather<double, double>(int, const double*, const int32_t*, double*,
                                            hipStream_t);
template void launch_gather<float, float>(int, const float*, const int32_t*, float*,
                                          hipStream_t);
template void launch_gather<double, float>(int, const double*, const int32_t*, float*,
                                           hipStream_t);
template void launch_gather<float, double>(int, const float*, const int32_t*, double*,
                                           hipStream_t);

// Replacement vectors from SplitMix64 (Steele, Lea and Flood 2014): entry with caller
// label o of draw number `draw` is output number draw*n + o of the generator seeded `seed`,
// mapped to [-1, 1) through its top 53 bits.
__device__ __forceinline__ double splitmix64_uniform(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
}
__global__ __launch_bounds__(kBlock) void k_fill_replacement(int n, uint64_t seed, uint64_t draw,
                                                             const int32_t* __restrict__ perm,
                                                             double* __restrict__ out) {
  for (int l = blockIdx.x * kBlock + threadIdx.x; l < n; l += gridDim.x * kBlock)
    out[l] = splitmix64_uniform(seed, draw * (uint64_t)n + (uint64_t)perm[l]);
}
void launch_fill_replacement(int n, uint64_t seed, uint64_t draw, const int32_t* perm,
                             double* out, hipStream_t s) {
  k_fill_replacement<<<stream_grid(n), kBlock, 0, s>>>(n, seed, draw, perm, out);
  HIP_LAUNCH_CHECK();
}

}  // namespace isira
