// Learned sparse approximate inverse (SPAI) preconditioner: the per-vertex / per-edge
// network that emits M on the pattern of L-hat, its hand-written backward pass and Adam.
//
// Network (F = 8 vertex features, H = 16 hidden units, weights rounded to BF16, FP32 math):
//   t_i = tanh(W1 f_i + b1),  h_i = tanh(W2 t_i + b2)                 (vertex MLP)
//   a_i = mean over neighbours j of h_j                                (aggregation)
//   s_i = wd . [h_i; a_i] + bd,  M_ii = softplus(s_i) / (d_i - sigma)   (diagonal head)
//   e_ij = [h_i + h_j; h_i * h_j; w_ij / sqrt(d_i d_j)]
//   g_ij = we . tanh(We e_ij + be) + ce                                (edge head)
//   m_ij = (1 - eps) tanh(g_ij) min(M_ii, M_jj) / max(n_i, n_j)
// e_ij is symmetric in (i, j), so M is symmetric; every row satisfies
// sum_j |m_ij| <= (1 - eps) M_ii, so M is strictly diagonally dominant with a positive
// diagonal, hence SPD.  The trimmed vertex gets M_ii = 0, which zeroes its row and column.
// Features: f = [1, log d_i, log n_i, mean_j log d_j, max_j log d_j, sigma / d_i, 1 / n_i,
// 1 if i is adjacent to the trimmed vertex].
#include <cmath>
#include <vector>

#include "spai.h"

namespace isira {
namespace spai {

constexpr int F = ISIRA_SPAI_F;
constexpr int H = ISIRA_SPAI_H;
constexpr int E = 2 * H + 1;
constexpr int oW1 = 0, ob1 = oW1 + H * F, oW2 = ob1 + H, ob2 = oW2 + H * H, owd = ob2 + H,
              obd = owd + 2 * H, oWe = obd + 1, obe = oWe + H * E, owe = obe + H, oce = owe + H,
              NP = oce + 1;
constexpr int NV_VERT = obd + 1;      // gradients reduced over vertices: params [0, oWe)
constexpr int NV_EDGE = NP - oWe;     // gradients reduced over edges:    params [oWe, NP)
constexpr float kEps = 0.05f;
// the neighbour mean sums rows longer than kNmChunk entries in pieces of kNmChunk entries
constexpr int kNmChunk = 1024;
static int64_t nm_part_elems(int64_t nnz) { return 2 * ((nnz + kNmChunk - 1) / kNmChunk) * H; }
static_assert(NV_VERT == oWe, "layout");
static_assert(NV_EDGE <= kSpaiRedValues && NV_VERT <= kSpaiRedValues && 64 <= kSpaiRedValues,
              "gradient reductions must fit the partials buffer");

__device__ __forceinline__ float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return x;  // inf / nan unchanged
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ void load_params(const float* __restrict__ params, float* sp) {
  for (int i = threadIdx.x; i < NP; i += blockDim.x) sp[i] = bf16_round(params[i]);
  __syncthreads();
}

__device__ __forceinline__ float softplusf(float x) {
  return fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}
__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

template <typename T>
__device__ __forceinline__ T wsum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wmax(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

static inline int grid_for(int64_t items, int per_block, int cap) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  return (int)(g > cap ? cap : g);
}

// ---------------------------------------------------------------------------- forward

__global__ __launch_bounds__(kBlock) void k_rowidx(int n, const int32_t* __restrict__ rp,
                                                   int32_t* __restrict__ rowidx) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kBlock + threadIdx.x) >> 6, nw = (gridDim.x * kBlock) >> 6;
  for (int r = wave; r < n; r += nw)
    for (int j = rp[r] + lane; j < rp[r + 1]; j += 64) rowidx[j] = r;
}

__global__ __launch_bounds__(kBlock) void k_features(int n, const int32_t* __restrict__ rp,
                                                     const int32_t* __restrict__ col,
                                                     const double* __restrict__ deg, int trim,
                                                     double sigma, float* __restrict__ feat) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kBlock + threadIdx.x) >> 6, nw = (gridDim.x * kBlock) >> 6;
  for (int i = wave; i < n; i += nw) {
    const int b = rp[i], e = rp[i + 1];
    float s = 0.0f, mx = -1e30f, adj = 0.0f;
    for (int j = b + lane; j < e; j += 64) {
      const int c = col[j];
      const float ld = logf((float)deg[c]);
      s += ld;
      mx = fmaxf(mx, ld);
      if (c == trim) adj = 1.0f;
    }
    s = wsum(s);
    mx = wmax(mx);
    adj = wmax(adj);
    if (lane == 0) {
      const float ni = (float)(e - b);
      const float di = (float)deg[i];
      float* f = feat + (size_t)i * F;
      f[0] = 1.0f;
      f[1] = logf(di);
      f[2] = logf(ni);
      f[3] = s / ni;
      f[4] = mx;
      f[5] = (float)(sigma / deg[i]);
      f[6] = 1.0f / ni;
      f[7] = adj;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_vertex_mlp(int n, const float* __restrict__ feat,
                                                       const float* __restrict__ params,
                                                       float* __restrict__ t1,
                                                       float* __restrict__ h) {
  __shared__ float sp[NP];
  load_params(params, sp);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    float f[F], t[H];
#pragma unroll
    for (int q = 0; q < F; ++q) f[q] = feat[(size_t)i * F + q];
#pragma unroll
    for (int o = 0; o < H; ++o) {
      float a = sp[ob1 + o];
#pragma unroll
      for (int q = 0; q < F; ++q) a += sp[oW1 + o * F + q] * f[q];
      t[o] = tanhf(a);
      t1[(size_t)i * H + o] = t[o];
    }
#pragma unroll
    for (int o = 0; o < H; ++o) {
      float a = sp[ob2 + o];
#pragma unroll
      for (int q = 0; q < H; ++q) a += sp[oW2 + o * H + q] * t[q];
      h[(size_t)i * H + o] = tanhf(a);
    }
  }
}

// a_i = mean_j h_j.  With divide_by_source = 1 it computes the plain gather-sum of x_j / n_j
// (used by the backward pass).  Rows of at most kNmChunk entries: H lanes per vertex, 64/H
// vertices per wave, four entries' loads issued together and summed in entry order.  Longer
// rows are skipped here and summed by k_nm_pieces + k_nm_long.
__device__ __forceinline__ float nm_term(const int32_t* __restrict__ rp,
                                         const float* __restrict__ x, int c, int k,
                                         int divide_by_source) {
  const float v = x[(size_t)c * H + k];
  return divide_by_source ? v / (float)(rp[c + 1] - rp[c]) : v;
}

__global__ __launch_bounds__(kBlock) void k_neighbour_mean(int n, const int32_t* __restrict__ rp,
                                                           const int32_t* __restrict__ col,
                                                           const float* __restrict__ x,
                                                           float* __restrict__ out,
                                                           int divide_by_source) {
  const int k = threadIdx.x % H;
  const int slot = (blockIdx.x * kBlock + threadIdx.x) / H;
  const int nslots = (gridDim.x * kBlock) / H;
  for (int i = slot; i < n; i += nslots) {
    const int b = rp[i], e = rp[i + 1];
    if (e - b > kNmChunk) continue;
    float s = 0.0f;
    int j = b;
    for (; j + 4 <= e; j += 4) {
      const int c0 = col[j], c1 = col[j + 1], c2 = col[j + 2], c3 = col[j + 3];
      const float v0 = nm_term(rp, x, c0, k, divide_by_source);
      const float v1 = nm_term(rp, x, c1, k, divide_by_source);
      const float v2 = nm_term(rp, x, c2, k, divide_by_source);
      const float v3 = nm_term(rp, x, c3, k, divide_by_source);
      s += v0;
      s += v1;
      s += v2;
      s += v3;
    }
    for (; j < e; ++j) s += nm_term(rp, x, col[j], k, divide_by_source);
    out[(size_t)i * H + k] = divide_by_source ? s : s / (float)(e - b);
  }
}

// Long rows (more than kNmChunk entries), first pass.  Stored entries are cut into chunks of
// kNmChunk; a chunk meets at most two long rows (one holding its first entry, one holding
// its last), since a long row cannot lie inside one chunk.  One wave per chunk: four groups
// of H lanes take every fourth entry of each long piece, the groups' sums are combined, and
// the piece's H sums go to part[(2 q + p) H ...] (p = 0: the row of the first entry, p = 1:
// the row of the last entry when it is another row).
__global__ __launch_bounds__(kBlock) void k_nm_pieces(int64_t nnz, const int32_t* __restrict__ rp,
                                                      const int32_t* __restrict__ col,
                                                      const int32_t* __restrict__ rowidx,
                                                      const float* __restrict__ x,
                                                      float* __restrict__ part,
                                                      int divide_by_source) {
  const int lane = threadIdx.x & 63, k = lane % H, g = lane / H;
  constexpr int G = 64 / H;
  const int64_t nch = (nnz + kNmChunk - 1) / kNmChunk;
  const int64_t wave = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kBlock) >> 6;
  for (int64_t q = wave; q < nch; q += nwaves) {
    const int64_t j0 = q * kNmChunk;
    const int64_t j1 = (j0 + kNmChunk < nnz) ? j0 + kNmChunk : nnz;
    const int r0 = rowidx[j0], r1 = rowidx[j1 - 1];
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const int r = p ? r1 : r0;
      if (p && r1 == r0) break;
      if (rp[r + 1] - rp[r] <= kNmChunk) continue;
      const int64_t a = rp[r] > j0 ? rp[r] : j0;
      const int64_t e = rp[r + 1] < j1 ? rp[r + 1] : j1;
      float s = 0.0f;
      int64_t j = a + g;
      for (; j + 3 * G < e; j += 4 * G) {  // four entries' loads in flight, summed in order
        const int c0 = col[j], c1 = col[j + G], c2 = col[j + 2 * G], c3 = col[j + 3 * G];
        const float v0 = nm_term(rp, x, c0, k, divide_by_source);
        const float v1 = nm_term(rp, x, c1, k, divide_by_source);
        const float v2 = nm_term(rp, x, c2, k, divide_by_source);
        const float v3 = nm_term(rp, x, c3, k, divide_by_source);
        s += v0;
        s += v1;
        s += v2;
        s += v3;
      }
      for (; j < e; j += G) s += nm_term(rp, x, col[j], k, divide_by_source);
#pragma unroll
      for (int o = H; o < 64; o <<= 1) s += __shfl_xor(s, o, 64);
      if (g == 0) part[((size_t)(2 * q + p)) * H + k] = s;
    }
  }
}

// Long rows, second pass: a row's H sums are its pieces' sums in chunk order (a thread per
// row and lane k of H; rows of at most kNmChunk entries are left to k_neighbour_mean).
__global__ __launch_bounds__(kBlock) void k_nm_long(int n, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ rowidx,
                                                    const float* __restrict__ part,
                                                    float* __restrict__ out,
                                                    int divide_by_source) {
  const int k = threadIdx.x % H;
  const int slot = (blockIdx.x * kBlock + threadIdx.x) / H;
  const int nslots = (gridDim.x * kBlock) / H;
  for (int i = slot; i < n; i += nslots) {
    const int b = rp[i], e = rp[i + 1];
    if (e - b <= kNmChunk) continue;
    const int q0 = b / kNmChunk, q1 = (e - 1) / kNmChunk;
    float s = 0.0f;
    int q = q0;
    for (; q + 4 <= q1 + 1; q += 4) {  // four pieces' loads in flight, summed in chunk order
      float v[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int pp = rowidx[(size_t)(q + t) * kNmChunk] == i ? 0 : 1;
        v[t] = part[((size_t)(2 * (q + t) + pp)) * H + k];
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) s += v[t];
    }
    for (; q <= q1; ++q) {
      const int pp = rowidx[(size_t)q * kNmChunk] == i ? 0 : 1;
      s += part[((size_t)(2 * q + pp)) * H + k];
    }
    out[(size_t)i * H + k] = divide_by_source ? s : s / (float)(e - b);
  }
}

// out_i for every row: short rows by k_neighbour_mean, long rows by pieces of kNmChunk
static void neighbour_mean(const SpaiWork& w, int n, int64_t nnz, const int32_t* rp,
                           const int32_t* col, const float* x, float* out, int divide_by_source,
                           hipStream_t s) {
  k_neighbour_mean<<<grid_for(n, kBlock / H, 8192), kBlock, 0, s>>>(n, rp, col, x, out,
                                                                    divide_by_source);
  const int64_t nch = (nnz + kNmChunk - 1) / kNmChunk;
  k_nm_pieces<<<grid_for(nch, kBlock / 64, 8192), kBlock, 0, s>>>(nnz, rp, col, w.rowidx, x,
                                                                  w.nm_part, divide_by_source);
  k_nm_long<<<grid_for(n, kBlock / H, 8192), kBlock, 0, s>>>(n, rp, w.rowidx, w.nm_part, out,
                                                             divide_by_source);
}

__global__ __launch_bounds__(kBlock) void k_diag_head(int n, const float* __restrict__ h,
                                                      const float* __restrict__ agg,
                                                      const double* __restrict__ deg,
                                                      double sigma, int trim,
                                                      const float* __restrict__ params,
                                                      float* __restrict__ sdiag,
                                                      float* __restrict__ diag32,
                                                      double* __restrict__ diag64) {
  __shared__ float sp[NP];
  load_params(params, sp);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    float s = sp[obd];
#pragma unroll
    for (int q = 0; q < H; ++q)
      s += sp[owd + q] * h[(size_t)i * H + q] + sp[owd + H + q] * agg[(size_t)i * H + q];
    sdiag[i] = s;
    const float m = (i == trim) ? 0.0f : softplusf(s) / (float)(deg[i] - sigma);
    diag32[i] = m;
    diag64[i] = (double)m;
  }
}

struct EdgeFwd {
  float u[H];
  float th, mn, mx;
};

__device__ __forceinline__ void edge_features(const float* hi, const float* hj, float wt,
                                              float* e) {
#pragma unroll
  for (int q = 0; q < H; ++q) {
    e[q] = hi[q] + hj[q];
    e[H + q] = hi[q] * hj[q];
  }
  e[2 * H] = wt;
}

__device__ __forceinline__ void edge_forward(const float* sp, const float* e, EdgeFwd& r) {
  float g = sp[oce];
#pragma unroll
  for (int o = 0; o < H; ++o) {
    float a = sp[obe + o];
#pragma unroll
    for (int q = 0; q < E; ++q) a += sp[oWe + o * E + q] * e[q];
    r.u[o] = tanhf(a);
    g += sp[owe + o] * r.u[o];
  }
  r.th = tanhf(g);
}

__device__ __forceinline__ float edge_weight(const void* w, int wdt, int j) {
  if (wdt == ISIRA_W_NONE) return 1.0f;
  if (wdt == ISIRA_W_F32) return ((const float*)w)[j];
  return (float)((const double*)w)[j];
}

__global__ __launch_bounds__(kBlock) void k_edge_values(int64_t nnz,
                                                        const int32_t* __restrict__ rowidx,
                                                        const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const void* w, int wdt,
                                                        const double* __restrict__ deg,
                                                        const float* __restrict__ h,
                                                        const float* __restrict__ diag32,
                                                        const float* __restrict__ params,
                                                        float* __restrict__ offd) {
  __shared__ float sp[NP];
  load_params(params, sp);
  for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * kBlock) {
    const int i = rowidx[j], c = col[j];
    float hi[H], hj[H], e[E];
#pragma unroll
    for (int q = 0; q < H; ++q) {
      hi[q] = h[(size_t)i * H + q];
      hj[q] = h[(size_t)c * H + q];
    }
    const float wt = (float)(edge_weight(w, wdt, (int)j) / sqrt(deg[i] * deg[c]));
    edge_features(hi, hj, wt, e);
    EdgeFwd r;
    edge_forward(sp, e, r);
    const float mn = fminf(diag32[i], diag32[c]);
    const float mx = (float)max(rp[i + 1] - rp[i], rp[c + 1] - rp[c]);
    offd[j] = (1.0f - kEps) * r.th * mn / mx;
  }
}

// ---------------------------------------------------------------------------- backward

// Rt[l*S + s] = r[s*n + perm[l]] (caller sample-major -> internal vertex-major)
__global__ __launch_bounds__(kBlock) void k_samples_in(int n, int S, const float* __restrict__ r,
                                                       const int32_t* __restrict__ perm,
                                                       float* __restrict__ Rt) {
  const int64_t tot = (int64_t)n * S;
  for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * kBlock) {
    const int l = (int)(t / S), s = (int)(t - (int64_t)l * S);
    Rt[t] = r[(size_t)s * n + perm[l]];
  }
}

// Yt[l][s] = M_ll Rt[l][s] + sum_j m_lj Rt[j][s]; row `trim` is zero.
__global__ __launch_bounds__(kBlock) void k_apply_multi(int n, int S, int Sp,
                                                        const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ col,
                                                        const float* __restrict__ diag,
                                                        const float* __restrict__ offd, int trim,
                                                        const float* __restrict__ Rt,
                                                        float* __restrict__ Yt) {
  const int rows_per = kBlock / Sp;
  const int rl = threadIdx.x / Sp, s = threadIdx.x % Sp;
  for (int base = blockIdx.x * rows_per; base < n; base += gridDim.x * rows_per) {
    const int l = base + rl;
    if (l >= n || s >= S) continue;
    float acc = 0.0f;
    if (l != trim) {
      acc = diag[l] * Rt[(size_t)l * S + s];
      for (int j = rp[l]; j < rp[l + 1]; ++j) acc += offd[j] * Rt[(size_t)col[j] * S + s];
    }
    Yt[(size_t)l * S + s] = acc;
  }
}

// per-sample ||z_s||^2 -> zz[s]; loss and G = dloss/dy.
__global__ __launch_bounds__(kBlock) void k_sample_norms(int n, int S, const float* __restrict__ Zt,
                                                         double* partials, unsigned* counter,
                                                         double* zz) {
  __shared__ double acc[64];
  for (int s = threadIdx.x; s < S; s += kBlock) acc[s] = 0.0;
  __syncthreads();
  // thread (row-slot, s): rows strided
  const int Sp = 64;
  const int rows_per = kBlock / Sp;
  const int rl = threadIdx.x / Sp, s = threadIdx.x % Sp;
  double loc = 0.0;
  if (s < S)
    for (int l = blockIdx.x * rows_per + rl; l < n; l += gridDim.x * rows_per) {
      const double v = Zt[(size_t)l * S + s];
      loc += v * v;
    }
  // reduce over the rows_per slots of each sample in fixed order
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = loc;
  __syncthreads();
  if (threadIdx.x < S) {
    double t = 0.0;
    for (int k = 0; k < rows_per; ++k) t += sh[k * Sp + threadIdx.x];
    partials[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x < S) {
    double t = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) t += partials[(size_t)threadIdx.x * gridDim.x + b];
    zz[threadIdx.x] = t;
  }
  if (threadIdx.x == 0) *counter = 0u;
}

__global__ __launch_bounds__(kBlock) void k_loss_grad_y(int n, int S, const float* __restrict__ Yt,
                                                        const float* __restrict__ Zt,
                                                        const double* __restrict__ zz,
                                                        float* __restrict__ Gt,
                                                        double* partials, unsigned* counter,
                                                        double* loss) {
  double loc = 0.0;
  const int64_t tot = (int64_t)n * S;
  for (int64_t t = blockIdx.x * (int64_t)kBlock + threadIdx.x; t < tot;
       t += (int64_t)gridDim.x * kBlock) {
    const int s = (int)(t % S);
    const double den = zz[s] > 0.0 ? zz[s] * S : 1.0;
    const double e = (double)Yt[t] - (double)Zt[t];
    loc += e * e / den;
    Gt[t] = (float)(2.0 * e / den);
  }
  __shared__ double sh4[4];
  loc = wsum(loc);
  if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = loc;
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) t += partials[b];
    *loss = t;
    *counter = 0u;
  }
}

// One wave per row i: for every stored entry (i, j) the gradient of the loss with respect
// to the shared value m_ij = m_ji is sum_s (G_i R_j + G_j R_i); it is pushed through the
// edge head.  Per row: dh_edge[i] (edge contributions to dL/dh_i) and cM[i] (to dL/dM_ii).
// Per entry with i < j: dpre (H), u (H) and dg for the edge-parameter reduction.
__global__ __launch_bounds__(kBlock) void k_edge_backward(
    int n, int S, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
    const void* w, int wdt, const double* __restrict__ deg, const float* __restrict__ h,
    const float* __restrict__ diag32, const float* __restrict__ Gt,
    const float* __restrict__ Rt, const float* __restrict__ params,
    float* __restrict__ dh_edge, float* __restrict__ cM, float* __restrict__ dpre_e,
    float* __restrict__ u_e, float* __restrict__ dg_e) {
  __shared__ float sp[NP];
  load_params(params, sp);
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * kBlock + threadIdx.x) >> 6, nw = (gridDim.x * kBlock) >> 6;
  for (int i = wave; i < n; i += nw) {
    const int b = rp[i], eend = rp[i + 1];
    float hi[H];
#pragma unroll
    for (int q = 0; q < H; ++q) hi[q] = h[(size_t)i * H + q];
    float dhi[H];
#pragma unroll
    for (int q = 0; q < H; ++q) dhi[q] = 0.0f;
    float cmi = 0.0f;
    const float Mi = diag32[i];
    const float ni = (float)(eend - b);
    for (int jj = b + lane; jj < eend; jj += 64) {
      const int c = col[jj];
      float dm = 0.0f;
      for (int s = 0; s < S; ++s)
        dm += Gt[(size_t)i * S + s] * Rt[(size_t)c * S + s] + Gt[(size_t)c * S + s] * Rt[(size_t)i * S + s];
      float hj[H], e[E];
#pragma unroll
      for (int q = 0; q < H; ++q) hj[q] = h[(size_t)c * H + q];
      const float wt = (float)(edge_weight(w, wdt, jj) / sqrt(deg[i] * deg[c]));
      edge_features(hi, hj, wt, e);
      EdgeFwd r;
      edge_forward(sp, e, r);
      const float Mj = diag32[c];
      const float mn = fminf(Mi, Mj);
      const float mx = fmaxf(ni, (float)(rp[c + 1] - rp[c]));
      const float dg = dm * (1.0f - kEps) * (1.0f - r.th * r.th) * mn / mx;
      const float dmn = dm * (1.0f - kEps) * r.th / mx;
      cmi += (Mi < Mj) ? dmn : ((Mi == Mj) ? 0.5f * dmn : 0.0f);
      float dpre[H];
#pragma unroll
      for (int o = 0; o < H; ++o) dpre[o] = dg * sp[owe + o] * (1.0f - r.u[o] * r.u[o]);
#pragma unroll
      for (int q = 0; q < H; ++q) {
        float d0 = 0.0f, d1 = 0.0f;
#pragma unroll
        for (int o = 0; o < H; ++o) {
          d0 += sp[oWe + o * E + q] * dpre[o];
          d1 += sp[oWe + o * E + H + q] * dpre[o];
        }
        dhi[q] += d0 + d1 * hj[q];
      }
      const bool own = i < c;
#pragma unroll
      for (int o = 0; o < H; ++o) {
        dpre_e[(size_t)jj * H + o] = own ? dpre[o] : 0.0f;
        u_e[(size_t)jj * H + o] = own ? r.u[o] : 0.0f;
      }
      dg_e[jj] = own ? dg : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < H; ++q) dhi[q] = wsum(dhi[q]);
    cmi = wsum(cmi);
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < H; ++q) dh_edge[(size_t)i * H + q] = dhi[q];
      cM[i] = cmi;
    }
  }
}

// dM_ii = sum_s G_i R_i + cM_i; ds_i; dh (diagonal + edge parts) and da.
__global__ __launch_bounds__(kBlock) void k_vertex_backward1(
    int n, int S, const float* __restrict__ Gt, const float* __restrict__ Rt,
    const float* __restrict__ cM, const float* __restrict__ sdiag, const double* __restrict__ deg,
    double sigma, int trim, const float* __restrict__ dh_edge, const float* __restrict__ params,
    float* __restrict__ ds, float* __restrict__ dh, float* __restrict__ da) {
  __shared__ float sp[NP];
  load_params(params, sp);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    float dM = cM[i];
    for (int s = 0; s < S; ++s) dM += Gt[(size_t)i * S + s] * Rt[(size_t)i * S + s];
    const float dsi = (i == trim) ? 0.0f : dM * sigmoidf(sdiag[i]) / (float)(deg[i] - sigma);
    ds[i] = dsi;
#pragma unroll
    for (int q = 0; q < H; ++q) {
      dh[(size_t)i * H + q] = dsi * sp[owd + q] + dh_edge[(size_t)i * H + q];
      da[(size_t)i * H + q] = dsi * sp[owd + H + q];
    }
  }
}

// dh += (gathered aggregation part); then the vertex-MLP backward -> dpre2, dpre1.
__global__ __launch_bounds__(kBlock) void k_vertex_backward2(
    int n, const float* __restrict__ dh, const float* __restrict__ dagg,
    const float* __restrict__ h, const float* __restrict__ t1, const float* __restrict__ params,
    float* __restrict__ dpre2, float* __restrict__ dpre1) {
  __shared__ float sp[NP];
  load_params(params, sp);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    float p2[H];
#pragma unroll
    for (int o = 0; o < H; ++o) {
      const float hv = h[(size_t)i * H + o];
      p2[o] = (dh[(size_t)i * H + o] + dagg[(size_t)i * H + o]) * (1.0f - hv * hv);
      dpre2[(size_t)i * H + o] = p2[o];
    }
#pragma unroll
    for (int q = 0; q < H; ++q) {
      float dt = 0.0f;
#pragma unroll
      for (int o = 0; o < H; ++o) dt += sp[oW2 + o * H + q] * p2[o];
      const float tv = t1[(size_t)i * H + q];
      dpre1[(size_t)i * H + q] = dt * (1.0f - tv * tv);
    }
  }
}

// Parameter gradients of the vertex MLP and the diagonal head: sums over vertices of outer
// products, in parameter order [W1 b1 W2 b2 wd bd].  Tiles of 64 vertices are staged in LDS;
// each thread owns fixed outputs, so the per-workgroup sums are deterministic.
constexpr int kRT = 64;
__global__ __launch_bounds__(kBlock) void k_vertex_param_grad(
    int n, const float* __restrict__ feat, const float* __restrict__ t1, const float* __restrict__ h,
    const float* __restrict__ agg, const float* __restrict__ ds, const float* __restrict__ dpre1,
    const float* __restrict__ dpre2, double* partials, unsigned* counter, float* __restrict__ grad) {
  __shared__ float sf[kRT][F], st[kRT][H], sh[kRT][H], sa[kRT][H], sd[kRT], s1[kRT][H], s2[kRT][H];
  double acc[(NV_VERT + kBlock - 1) / kBlock];
#pragma unroll
  for (int k = 0; k < (NV_VERT + kBlock - 1) / kBlock; ++k) acc[k] = 0.0;
  const int ntiles = (n + kRT - 1) / kRT;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int base = tile * kRT;
    const int len = min(kRT, n - base);
    __syncthreads();
    for (int e = threadIdx.x; e < kRT * H; e += kBlock) {
      const int r = e / H, q = e % H;
      const bool ok = r < len;
      const size_t gi = (size_t)(base + r) * H + q;
      st[r][q] = ok ? t1[gi] : 0.0f;
      sh[r][q] = ok ? h[gi] : 0.0f;
      sa[r][q] = ok ? agg[gi] : 0.0f;
      s1[r][q] = ok ? dpre1[gi] : 0.0f;
      s2[r][q] = ok ? dpre2[gi] : 0.0f;
      if (q < F) sf[r][q] = ok ? feat[(size_t)(base + r) * F + q] : 0.0f;
      if (q == 0) sd[r] = ok ? ds[base + r] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < (NV_VERT + kBlock - 1) / kBlock; ++k) {
      const int p = threadIdx.x + k * kBlock;
      if (p >= NV_VERT) break;
      double s = 0.0;
      if (p < ob1) {
        const int o = p / F, q = p % F;
        for (int r = 0; r < len; ++r) s += (double)(s1[r][o] * sf[r][q]);
      } else if (p < oW2) {
        const int o = p - ob1;
        for (int r = 0; r < len; ++r) s += (double)s1[r][o];
      } else if (p < ob2) {
        const int o = (p - oW2) / H, q = (p - oW2) % H;
        for (int r = 0; r < len; ++r) s += (double)(s2[r][o] * st[r][q]);
      } else if (p < owd) {
        const int o = p - ob2;
        for (int r = 0; r < len; ++r) s += (double)s2[r][o];
      } else if (p < owd + H) {
        const int q = p - owd;
        for (int r = 0; r < len; ++r) s += (double)(sd[r] * sh[r][q]);
      } else if (p < obd) {
        const int q = p - owd - H;
        for (int r = 0; r < len; ++r) s += (double)(sd[r] * sa[r][q]);
      } else {
        for (int r = 0; r < len; ++r) s += (double)sd[r];
      }
      acc[k] += s;
    }
  }
#pragma unroll
  for (int k = 0; k < (NV_VERT + kBlock - 1) / kBlock; ++k) {
    const int p = threadIdx.x + k * kBlock;
    if (p < NV_VERT) partials[(size_t)p * gridDim.x + blockIdx.x] = acc[k];
  }
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
  for (int p = threadIdx.x; p < NV_VERT; p += kBlock) {
    double s = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) s += partials[(size_t)p * gridDim.x + b];
    grad[p] = (float)s;
  }
  if (threadIdx.x == 0) *counter = 0u;
}

// Parameter gradients of the edge head, in parameter order [We be we ce], summed over the
// stored entries with i < j (each undirected edge once).
__global__ __launch_bounds__(kBlock) void k_edge_param_grad(
    int64_t nnz, const int32_t* __restrict__ rowidx, const int32_t* __restrict__ col,
    const void* w, int wdt, const double* __restrict__ deg, const float* __restrict__ h,
    const float* __restrict__ dpre_e, const float* __restrict__ u_e, const float* __restrict__ dg_e,
    double* partials, unsigned* counter, float* __restrict__ grad) {
  __shared__ float se[kRT][E], sp1[kRT][H], su[kRT][H], sg[kRT];
  constexpr int NK = (NV_EDGE + kBlock - 1) / kBlock;
  double acc[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) acc[k] = 0.0;
  const int64_t ntiles = (nnz + kRT - 1) / kRT;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t base = tile * kRT;
    const int len = (int)min((int64_t)kRT, nnz - base);
    __syncthreads();
    for (int r = threadIdx.x; r < kRT; r += kBlock) {
      if (r < len) {
        const int64_t j = base + r;
        const int i = rowidx[j], c = col[j];
        float hi[H], hj[H], e[E];
#pragma unroll
        for (int q = 0; q < H; ++q) {
          hi[q] = h[(size_t)i * H + q];
          hj[q] = h[(size_t)c * H + q];
        }
        edge_features(hi, hj, (float)(edge_weight(w, wdt, (int)j) / sqrt(deg[i] * deg[c])), e);
#pragma unroll
        for (int q = 0; q < E; ++q) se[r][q] = e[q];
#pragma unroll
        for (int o = 0; o < H; ++o) {
          sp1[r][o] = dpre_e[(size_t)j * H + o];
          su[r][o] = u_e[(size_t)j * H + o];
        }
        sg[r] = dg_e[j];
      } else {
#pragma unroll
        for (int q = 0; q < E; ++q) se[r][q] = 0.0f;
#pragma unroll
        for (int o = 0; o < H; ++o) sp1[r][o] = su[r][o] = 0.0f;
        sg[r] = 0.0f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const int p = threadIdx.x + k * kBlock;  // offset from oWe
      if (p >= NV_EDGE) break;
      double s = 0.0;
      if (p < obe - oWe) {
        const int o = p / E, q = p % E;
        for (int r = 0; r < len; ++r) s += (double)(sp1[r][o] * se[r][q]);
      } else if (p < owe - oWe) {
        const int o = p - (obe - oWe);
        for (int r = 0; r < len; ++r) s += (double)sp1[r][o];
      } else if (p < oce - oWe) {
        const int o = p - (owe - oWe);
        for (int r = 0; r < len; ++r) s += (double)(sg[r] * su[r][o]);
      } else {
        for (int r = 0; r < len; ++r) s += (double)sg[r];
      }
      acc[k] += s;
    }
  }
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int p = threadIdx.x + k * kBlock;
    if (p < NV_EDGE) partials[(size_t)p * gridDim.x + blockIdx.x] = acc[k];
  }
  __shared__ int last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
  for (int p = threadIdx.x; p < NV_EDGE; p += kBlock) {
    double s = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) s += partials[(size_t)p * gridDim.x + b];
    grad[oWe + p] = (float)s;
  }
  if (threadIdx.x == 0) *counter = 0u;
}

__global__ __launch_bounds__(kBlock) void k_adam(int count, float* __restrict__ p,
                                                 const float* __restrict__ g, float* __restrict__ m,
                                                 float* __restrict__ v, float lr, float b1, float b2,
                                                 float eps, float c1, float c2) {
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < count; i += gridDim.x * kBlock) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

__global__ __launch_bounds__(kBlock) void k_scatter_offd(int64_t nnz, const float* __restrict__ src,
                                                         const int32_t* __restrict__ map,
                                                         float* __restrict__ dst) {
  for (int64_t j = blockIdx.x * (int64_t)kBlock + threadIdx.x; j < nnz;
       j += (int64_t)gridDim.x * kBlock)
    dst[map[j]] = src[j];
}

}  // namespace spai
}  // namespace isira

// ---------------------------------------------------------------------------- host side

namespace isira {
namespace spai {

int32_t nparam() { return NP; }

int ensure(SpaiWork& w, int64_t n, int64_t nnz) {
  if (w.n == n && w.nnz == nnz && w.diag32) return 0;
  free_work(w);
  w.n = n;
  w.nnz = nnz;
  DevMem& m = *w.mem;
  int rc;
  if ((rc = dalloc(m, &w.diag32, n)) || (rc = dalloc(m, &w.diag64, n)) || (rc = dalloc(m, &w.offd, nnz)) ||
      (rc = dalloc(m, &w.feat, n * F)) || (rc = dalloc(m, &w.t1, n * H)) || (rc = dalloc(m, &w.h, n * H)) ||
      (rc = dalloc(m, &w.agg, n * H)) || (rc = dalloc(m, &w.sdiag, n)) || (rc = dalloc(m, &w.rowidx, nnz)) ||
      (rc = dalloc(m, &w.nm_part, nm_part_elems(nnz)))) {
    free_work(w);
    return rc;
  }
  return 0;
}

// bytes of the buffers ensure() allocates
size_t work_bytes(int64_t n, int64_t nnz) {
  return dev_round(n * 4) + dev_round(n * 8) + dev_round(nnz * 4) + dev_round(n * F * 4) +
         3 * dev_round(n * H * 4) + dev_round(n * 4) + dev_round(nnz * 4) +
         dev_round(nm_part_elems(nnz) * 4);
}

static int scratch(SpaiWork& w, size_t elems, float** out) {
  *out = nullptr;
  if (w.scratch_elems < elems) {
    dfree(*w.mem, w.scratch);
    w.scratch_elems = 0;
    const int rc = dalloc(*w.mem, &w.scratch, elems);
    if (rc) return rc;
    w.scratch_elems = elems;
  }
  *out = w.scratch;
  return 0;
}

int forward(SpaiWork& w, const int32_t* rp, const int32_t* col, const void* wts, int wdt,
            const double* deg, int n, int64_t nnz, double sigma, int trim, const float* params,
            hipStream_t s) {
  int rc = ensure(w, n, nnz);
  if (rc) return rc;
  const int gw = grid_for(n, kBlock / 64, 8192);
  k_rowidx<<<gw, kBlock, 0, s>>>(n, rp, w.rowidx);
  k_features<<<gw, kBlock, 0, s>>>(n, rp, col, deg, trim, sigma, w.feat);
  const int gv = grid_for(n, kBlock, 2048);
  k_vertex_mlp<<<gv, kBlock, 0, s>>>(n, w.feat, params, w.t1, w.h);
  neighbour_mean(w, n, nnz, rp, col, w.h, w.agg, 0, s);
  k_diag_head<<<gv, kBlock, 0, s>>>(n, w.h, w.agg, deg, sigma, trim, params, w.sdiag, w.diag32,
                                    w.diag64);
  k_edge_values<<<grid_for(nnz, kBlock, 8192), kBlock, 0, s>>>(nnz, w.rowidx, rp, col, wts, wdt,
                                                               deg, w.h, w.diag32, params, w.offd);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

int loss_grad(SpaiWork& w, const int32_t* rp, const int32_t* col, const void* wts, int wdt,
              const double* deg, int n, int64_t nnz, double sigma, int trim, const float* params,
              const int32_t* perm, const float* r, const float* z, int S, float* grad,
              double* loss_host, RedBuf rb, hipStream_t s) {
  if (S < 1 || S > 64) return -2;
  int frc = forward(w, rp, col, wts, wdt, deg, n, nnz, sigma, trim, params, s);
  if (frc) return frc;
  const size_t nS = (size_t)n * S;
  // 4 sample blocks, 6 per-vertex H-vectors + 2 scalars, per-entry dpre/u/dg, then 16-byte
  // aligned doubles zz[64] and the loss (65 doubles = 130 floats) with generous slack
  const size_t need = 4 * nS + (size_t)n * (6 * H + 2) + (size_t)nnz * (2 * H + 1) + 512;
  float* base = nullptr;
  const int src = scratch(w, need, &base);
  if (src) return src;
  float* Rt = base;
  float* Zt = Rt + nS;
  float* Yt = Zt + nS;
  float* Gt = Yt + nS;
  float* dh_edge = Gt + nS;
  float* cM = dh_edge + (size_t)n * H;
  float* ds = cM + n;
  float* dh = ds + n;
  float* da = dh + (size_t)n * H;
  float* dagg = da + (size_t)n * H;
  float* dpre2 = dagg + (size_t)n * H;
  float* dpre1 = dpre2 + (size_t)n * H;
  float* dpre_e = dpre1 + (size_t)n * H;
  float* u_e = dpre_e + (size_t)nnz * H;
  float* dg_e = u_e + (size_t)nnz * H;
  double* dscal = (double*)(((uintptr_t)(dg_e + nnz) + 15) & ~(uintptr_t)15);  // zz[64], loss
  double* zz = dscal;
  double* dloss = dscal + 64;
  const int gS = grid_for((int64_t)nS, kBlock, 4096);
  k_samples_in<<<gS, kBlock, 0, s>>>(n, S, r, perm, Rt);
  k_samples_in<<<gS, kBlock, 0, s>>>(n, S, z, perm, Zt);
  int Sp = 1;
  while (Sp < S) Sp <<= 1;
  k_apply_multi<<<grid_for(n, kBlock / Sp, 8192), kBlock, 0, s>>>(n, S, Sp, rp, col, w.diag32,
                                                                  w.offd, trim, Rt, Yt);
  k_sample_norms<<<grid_for(n, kBlock / 64, kSpaiRedGrid), kBlock, 0, s>>>(n, S, Zt, rb.partials,
                                                                 rb.counters + 20, zz);
  k_loss_grad_y<<<grid_for((int64_t)nS, kBlock, kSpaiRedGrid), kBlock, 0, s>>>(n, S, Yt, Zt, zz, Gt,
                                                                      rb.partials,
                                                                      rb.counters + 21, dloss);
  const int gw = grid_for(n, kBlock / 64, 8192);
  k_edge_backward<<<gw, kBlock, 0, s>>>(n, S, rp, col, wts, wdt, deg, w.h, w.diag32, Gt, Rt,
                                        params, dh_edge, cM, dpre_e, u_e, dg_e);
  const int gv = grid_for(n, kBlock, 2048);
  k_vertex_backward1<<<gv, kBlock, 0, s>>>(n, S, Gt, Rt, cM, w.sdiag, deg, sigma, trim, dh_edge,
                                           params, ds, dh, da);
  neighbour_mean(w, n, nnz, rp, col, da, dagg, 1, s);
  k_vertex_backward2<<<gv, kBlock, 0, s>>>(n, dh, dagg, w.h, w.t1, params, dpre2, dpre1);
  k_vertex_param_grad<<<grid_for(n, kRT, kSpaiRedGrid), kBlock, 0, s>>>(n, w.feat, w.t1, w.h, w.agg, ds,
                                                               dpre1, dpre2, rb.partials,
                                                               rb.counters + 22, grad);
  k_edge_param_grad<<<grid_for(nnz, kRT, kSpaiRedGrid), kBlock, 0, s>>>(nnz, w.rowidx, col, wts, wdt, deg,
                                                               w.h, dpre_e, u_e, dg_e, rb.partials,
                                                               rb.counters + 23, grad);
  if (hipMemcpyAsync(loss_host, dloss, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return -1;
  if (hipStreamSynchronize(s) != hipSuccess) return -1;
  return 0;
}

void adam(float* p, const float* g, float* m, float* v, int count, float lr, float b1, float b2,
          float eps, int step, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  k_adam<<<grid_for(count, kBlock, 1024), kBlock, 0, s>>>(count, p, g, m, v, lr, b1, b2, eps, c1, c2);
}

void scatter_offd(int64_t nnz, const float* src, const int32_t* map, float* dst, hipStream_t s) {
  k_scatter_offd<<<grid_for(nnz, kBlock, 8192), kBlock, 0, s>>>(nnz, src, map, dst);
}

}  // namespace spai
}  // namespace isira
