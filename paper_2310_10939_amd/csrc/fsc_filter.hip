// The learned polynomial-filter form: device kernels.
//
// The plain method computes M^t X0 (Algorithm 1); here gamma^t is replaced by
// p(gamma) = sum_{j=0..8} c_j T*_j(gamma) with T*_j the Chebyshev polynomials
// shifted to [0, 1].  In z-space (Z = D^{-1/2} Y) the basis blocks follow the
// three-term recurrence
//   B_0 = Z0,  B_1 = 2 M_z B_0 - B_0,  B_{j+1} = 4 M_z B_j - 2 B_j - B_{j-1},
// where M_z Z = Z/2 + (1/(2d)) (.) (A Z) is the same operator as one
// PowerMethod step, so each basis block costs one sparse product (the tile
// kernel with a Chebyshev epilogue).  The epilogue also accumulates the
// column Rayleigh quotients <B_j, M B_j> / <B_j, B_j> (y-space) used as
// features.  The filtered embedding is E(c) = sum_j c_j B_j with
// c_0 = 1 - sum_{j>0} c_j (so p(1) = 1).
//
// Training statistics: for labels of the non-isolated vertices, the
// within-cluster and total scatter of E(c) (the k-means cost of Sec. 2.2 and
// its one-cluster value) are quadratic forms c^T W c and c^T T c.  With
// G_ij = sum_v <B_i[v], B_j[v]>, S_ic = sum_{v in C_c} B_i[v] and m_c = |C_c|:
//   W_ij = G_ij - sum_c <S_ic, S_jc> / m_c,
//   T_ij = G_ij - <S_i, S_j> / m   (S_i = sum_c S_ic, m = sum_c m_c),
// all in FP64 from the FP32 blocks, each sum in a fixed order.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"
#include "fsc_tiles.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace fsc {

// Rayleigh-quotient statistics: each block writes its partial sums; the
// one-block cheb_stats_finish kernel, launched after the step on the same
// stream, writes per column q rayleigh[step * LH + q] = sum d z m / sum d z z
// (no block of the step waits on a device-scope fence).
template <int LH>
__device__ __forceinline__ void cheb_stats_epilogue(const StatsArgs& sa, const double* st) {
  __shared__ double red[kBlock / FSC_WAVE];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) {
    const double v = block_sum<kBlock>(st[q], red);
    if (threadIdx.x == 0) sa.partials[(int64_t)blockIdx.x * 2 * LH + q] = v;
  }
}

template <int LH>
__global__ __launch_bounds__(kBlock) void cheb_stats_finish(StatsArgs sa, int grid) {
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ double tot[2 * LH];
  const int32_t nlong = sa.meta[1];
  double v[2 * LH];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) v[q] = 0.0;
  for (int32_t g = threadIdx.x; g < grid; g += kBlock)
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) v[q] += sa.partials[(int64_t)g * 2 * LH + q];
  for (int32_t g = threadIdx.x; g < nlong; g += kBlock)
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) v[q] += sa.lnorm[(int64_t)g * 2 * LH + q];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) {
    const double s = block_sum<kBlock>(v[q], red);
    if (threadIdx.x == 0) tot[q] = s;
  }
  __syncthreads();
  if (threadIdx.x < LH) {
    const int q = threadIdx.x;
    sa.rayleigh[(int64_t)sa.step * LH + q] = tot[q] > 0.0 ? tot[LH + q] / tot[q] : 0.0;
  }
}

// One Chebyshev step: zout = first ? 2 M_z z - z : 4 M_z z - 2 z - zprev.
template <typename W, int LH_>
struct ChebOp {
  static constexpr int LH = LH_;
  static constexpr bool STATS = true;
  using A = float;
  struct Pre {
    float z[LH_];
    float zm[LH_];
    float h;
    double d;
  };
  const W* val;
  const float* zin;
  const float* zprev;
  float* zout;
  const float* hinv;
  const double* deg;
  int first;
  __device__ __forceinline__ void init() {}
  template <class SA>
  __device__ __forceinline__ void epilogue(const SA& sa, const double* st) const {
    cheb_stats_epilogue<LH_>(sa, st);
  }
  template <int U>
  __device__ __forceinline__ void accumulate(const int32_t* col, int64_t j0, int32_t stride, int64_t end,
                                             float* acc) const {
    int32_t c[U];
    float w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + (int64_t)u * stride;
      const bool ok = j < end;
      c[u] = ok ? nt_load(col + j) : -1;
      w[u] = ok ? load_weight<W, float>(val, j) : 0.f;
    }
    float z[U][LH_];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (c[u] >= 0) {
        rowio<float, LH_>::load(zin + (int64_t)c[u] * LH_, z[u]);
      } else {
#pragma unroll
        for (int q = 0; q < LH_; ++q) z[u][q] = 0.f;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < LH_; ++q) {
        if constexpr (std::is_void<W>::value) acc[q] += z[u][q];
        else acc[q] += w[u] * z[u][q];
      }
  }
  __device__ __forceinline__ void prefetch(int32_t r, Pre& p) const {
    rowio<float, LH_>::load(zin + (int64_t)r * LH_, p.z);
    if (first) {
#pragma unroll
      for (int q = 0; q < LH_; ++q) p.zm[q] = 0.f;
    } else {
      rowio<float, LH_>::load(zprev + (int64_t)r * LH_, p.zm);
    }
    p.h = hinv[r];
    p.d = deg[r];
  }
  __device__ __forceinline__ void finish(int32_t r, const float* acc, const Pre& p, double* st) const {
    float out[LH_];
#pragma unroll
    for (int q = 0; q < LH_; ++q) {
      const float m = fma_acc(p.h, acc[q], 0.5f * p.z[q]);
      out[q] = first ? 2.f * m - p.z[q] : 4.f * m - 2.f * p.z[q] - p.zm[q];
      st[q] += p.d * (double)p.z[q] * (double)p.z[q];
      st[LH_ + q] += p.d * (double)p.z[q] * (double)m;
    }
    if (zout) rowio<float, LH_>::store(zout + (int64_t)r * LH_, out);
  }
};

// ---------------------------------------------------------------------------
// Gram matrix of the basis blocks over the non-isolated vertices:
// G_ij = sum_{v: d_v > 0} <B_i[v], B_j[v]>, written to out[81] (both
// triangles).
// ---------------------------------------------------------------------------
struct Blocks {
  const float* b[9];
};

constexpr int kGram = 45;

__global__ __launch_bounds__(kBlock) void gram_kernel(Blocks B, const double* __restrict__ deg, int32_t n, int l,
                                                      int LH, double* __restrict__ partials,
                                                      int32_t* __restrict__ counter, double* __restrict__ out) {
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ int is_last;
  double acc[kGram];
#pragma unroll
  for (int i = 0; i < kGram; ++i) acc[i] = 0.0;
  for (int32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    if (!(deg[r] > 0.0)) continue;
    for (int q = 0; q < l; ++q) {
      double b[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) b[i] = (double)B.b[i][(int64_t)r * LH + q];
      int idx = 0;
#pragma unroll
      for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = i; j < 9; ++j) acc[idx++] += b[i] * b[j];
    }
  }
#pragma unroll
  for (int i = 0; i < kGram; ++i) {
    const double v = block_sum<kBlock>(acc[i], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * kGram + i] = v;
  }
  if (threadIdx.x == 0) {
    __threadfence();
    is_last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (threadIdx.x < kGram) {
    double s = 0.0;
    for (int g = 0; g < (int)gridDim.x; ++g) s += partials[(int64_t)g * kGram + threadIdx.x];
    const int k = threadIdx.x;
    int i = 0, base = 0;
    while (k >= base + (9 - i)) {
      base += 9 - i;
      ++i;
    }
    const int j = i + (k - base);
    out[i * 9 + j] = s;
    out[j * 9 + i] = s;
  }
  if (threadIdx.x == 0) *counter = 0;
}

// ---------------------------------------------------------------------------
// Per-cluster sums of the basis blocks.  Block g takes rows
// [g * chunk, (g + 1) * chunk); thread e < 9l owns component e = i * l + q
// (block B_i, column q) and thread 9l counts the rows: each walks the chunk's
// rows in order and adds to its own LDS column acc[c][e], so no two threads
// touch one word and the sums are deterministic.  part[g][c][e].
// ---------------------------------------------------------------------------
constexpr int kSumsRowsLds = 1024;  // labels and degree flags of this many rows staged at a time

__global__ __launch_bounds__(kBlock) void cluster_sums_kernel(Blocks B, const int32_t* __restrict__ labels,
                                                              const double* __restrict__ deg, int32_t n, int l,
                                                              int LH, int k, int32_t chunk,
                                                              double* __restrict__ part) {
  extern __shared__ double acc[];  // k * E
  __shared__ int32_t lab[kSumsRowsLds];
  __shared__ const float* bp[9];
  const int E = 9 * l + 1;
  if (threadIdx.x < 9) {
#pragma unroll
    for (int i = 0; i < 9; ++i)
      if ((int)threadIdx.x == i) bp[i] = B.b[i];
  }
  for (int i = threadIdx.x; i < k * E; i += kBlock) acc[i] = 0.0;
  const int32_t r0 = blockIdx.x * chunk;
  const int32_t r1 = min(n, r0 + chunk);
  const int e = threadIdx.x;
  for (int32_t s0 = r0; s0 < r1; s0 += kSumsRowsLds) {
    const int32_t cnt = min(kSumsRowsLds, r1 - s0);
    __syncthreads();
    // -1 marks a row in no cluster: an isolated vertex (or a label outside
    // [0, k), which the k-means labels never are)
    for (int i = threadIdx.x; i < cnt; i += kBlock) {
      const int32_t c = labels[s0 + i];
      lab[i] = deg[s0 + i] > 0.0 && c >= 0 && c < k ? c : -1;
    }
    __syncthreads();
    if (e < E) {
      const bool is_count = e == E - 1;
      const float* src = is_count ? nullptr : bp[e / l] + (e % l);
      int32_t i = 0;
      for (; i + 8 <= cnt; i += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = is_count ? 1.0 : (double)src[(int64_t)(s0 + i + u) * LH];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = lab[i + u];
          if (c >= 0) acc[c * E + e] += v[u];
        }
      }
      for (; i < cnt; ++i) {
        const int c = lab[i];
        if (c >= 0) acc[c * E + e] += is_count ? 1.0 : (double)src[(int64_t)(s0 + i) * LH];
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k * E; i += kBlock) part[(int64_t)blockIdx.x * k * E + i] = acc[i];
}

// W and T from G (gram[81]) and the per-block cluster sums (one block).
__global__ __launch_bounds__(kBlock) void scatter_finish_kernel(const double* __restrict__ part, int nblk, int l,
                                                                int k, const double* __restrict__ gram,
                                                                double* __restrict__ within,
                                                                double* __restrict__ total) {
  extern __shared__ double S[];  // k * E cluster sums, then E totals
  const int E = 9 * l + 1;
  for (int i = threadIdx.x; i < k * E; i += kBlock) {
    double s = 0.0;
    for (int g = 0; g < nblk; ++g) s += part[(int64_t)g * k * E + i];
    S[i] = s;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < E; e += kBlock) {
    double s = 0.0;
    for (int c = 0; c < k; ++c) s += S[c * E + e];
    S[k * E + e] = s;
  }
  __syncthreads();
  if (threadIdx.x < 81) {
    const int i = threadIdx.x / 9, j = threadIdx.x % 9;
    double wb = 0.0;
    for (int c = 0; c < k; ++c) {
      const double* Sc = S + c * E;
      const double m = Sc[E - 1];
      if (!(m > 0.0)) continue;
      double dot = 0.0;
      for (int q = 0; q < l; ++q) dot += Sc[i * l + q] * Sc[j * l + q];
      wb += dot / m;
    }
    const double* St = S + k * E;
    const double m = St[E - 1];
    double tb = 0.0;
    if (m > 0.0) {
      for (int q = 0; q < l; ++q) tb += St[i * l + q] * St[j * l + q];
      tb /= m;
    }
    within[threadIdx.x] = gram[threadIdx.x] - wb;
    total[threadIdx.x] = gram[threadIdx.x] - tb;
  }
}

// ---------------------------------------------------------------------------
// Features: log n, log k, log mean degree, log(1 + degree CV), log(max/mean degree)
// (over non-isolated vertices) and the column-mean Rayleigh quotients of
// B_0..B_3, centred and scaled by fixed constants.
// ---------------------------------------------------------------------------
__constant__ float kFeatShift[9] = {12.f, 2.f, 3.f, 1.f, 5.f, 0.f, 0.f, 0.f, 0.f};
__constant__ float kFeatScale[9] = {2.f, 1.f, 1.f, 1.f, 2.f, 1.f, 1.f, 1.f, 1.f};

__global__ __launch_bounds__(kBlock) void features_kernel(const double* __restrict__ deg, int32_t n, int k, int l,
                                                          int LH, const double* __restrict__ ray,
                                                          double* __restrict__ partials,
                                                          int32_t* __restrict__ counter, float* __restrict__ feat) {
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ int is_last;
  double s1 = 0.0, s2 = 0.0, mx = 0.0, cnt = 0.0;
  for (int32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    const double d = deg[r];
    if (d > 0.0) {
      s1 += d;
      s2 += d * d;
      mx = fmax(mx, d);
      cnt += 1.0;
    }
  }
  s1 = block_sum<kBlock>(s1, red);
  s2 = block_sum<kBlock>(s2, red);
  cnt = block_sum<kBlock>(cnt, red);
  // block max through negated sums is not exact; use a shuffle max
  for (int m = 32; m >= 1; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m, FSC_WAVE));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x / 64] = mx;
  __syncthreads();
  double bm = 0.0;
  for (int i = 0; i < kBlock / FSC_WAVE; ++i) bm = fmax(bm, red[i]);
  if (threadIdx.x == 0) {
    partials[blockIdx.x * 4 + 0] = s1;
    partials[blockIdx.x * 4 + 1] = s2;
    partials[blockIdx.x * 4 + 2] = bm;
    partials[blockIdx.x * 4 + 3] = cnt;
    __threadfence();
    is_last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last || threadIdx.x != 0) return;
  __threadfence();
  double a = 0.0, b2 = 0.0, m = 0.0, c = 0.0;
  for (int g = 0; g < (int)gridDim.x; ++g) {
    a += partials[g * 4 + 0];
    b2 += partials[g * 4 + 1];
    m = fmax(m, partials[g * 4 + 2]);
    c += partials[g * 4 + 3];
  }
  const double mean = c > 0.0 ? a / c : 1.0;
  const double var = c > 0.0 ? fmax(b2 / c - mean * mean, 0.0) : 0.0;
  double raw[9];
  raw[0] = log((double)n);
  raw[1] = log((double)k);
  raw[2] = log(mean);
  raw[3] = log1p(sqrt(var) / mean);
  raw[4] = log(fmax(m, 1e-300) / mean);
  for (int j = 0; j < 4; ++j) {
    double s = 0.0;
    for (int q = 0; q < l; ++q) s += ray[j * LH + q];
    raw[5 + j] = s / l;
  }
  for (int i = 0; i < 9; ++i) feat[i] = (float)((raw[i] - kFeatShift[i]) / kFeatScale[i]);
  *counter = 0;
}

// Chebyshev coefficients of gamma^8 on [0, 1]: with x = 2 gamma - 1 = cos u,
// gamma^8 = cos^16(u/2) = (C(16,8) + 2 sum_j C(16, 8-j) cos(j u)) / 2^16.
__constant__ float kGamma8[9] = {12870.f / 65536.f, 11440.f / 32768.f, 8008.f / 32768.f,
                                 4368.f / 32768.f,  1820.f / 32768.f,  560.f / 32768.f,
                                 120.f / 32768.f,   16.f / 32768.f,    1.f / 32768.f};

// S = sum_j c_j B_j, c_0 = 1 - sum_{j>0} c_j (c_rest = c_1..c_8 on device),
// or the coefficients of gamma^8 when c_rest is null.
__global__ void combine_kernel(Blocks B, const float* __restrict__ c_rest, int64_t count, float* __restrict__ S) {
  float c[9];
  if (c_rest) {
    float sum = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      c[j + 1] = c_rest[j];
      sum += c_rest[j];
    }
    c[0] = 1.f - sum;
  } else {
#pragma unroll
    for (int j = 0; j < 9; ++j) c[j] = kGamma8[j];
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 9; ++j) s += c[j] * B.b[j][i];
    S[i] = s;
  }
}

// used = 1 when (a) the filtered block's column-mean Rayleigh quotient (row
// row_f) is below that of M^8 X0 (row row_ref): the filter concentrated the
// block on the top of the spectrum less than the same budget of plain
// PowerMethod steps does; or (b) the normalised k-means cost of the filtered
// embedding exceeds kmax (its clusters are not tight); or (c) a coefficient
// is not finite.  diag (optional): rho_f, rho_8, normalised cost, used.
__global__ void fallback_kernel(const double* __restrict__ ray, int l, int LH, int row_f, int row_ref,
                                const double* __restrict__ kcost, double kmax, const float* __restrict__ c_rest,
                                int32_t* __restrict__ used, double* __restrict__ diag) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double rf = 0.0, rr = 0.0;
  for (int q = 0; q < l; ++q) {
    rf += ray[row_f * LH + q];
    rr += ray[row_ref * LH + q];
  }
  rf /= l;
  rr /= l;
  const double kc = *kcost;
  bool bad = !(rf >= rr) || !(kc <= kmax);
  for (int j = 0; j < 8; ++j) bad = bad || !isfinite(c_rest[j]);
  *used = bad ? 1 : 0;
  if (diag) {
    diag[0] = rf;
    diag[1] = rr;
    diag[2] = kc;
    diag[3] = bad ? 1.0 : 0.0;
  }
}

// ===========================================================================
// Host side
// ===========================================================================
template <typename W, int LH>
static int cheb_steps_typed(Context* ctx, EmbedIO* io, float* const* basis, int nsteps, double* ray,
                            hipStream_t s) {
  const fsc_csr* g = io->g;
  TileArgs ta;
  ta.row_ptr = g->row_ptr;
  ta.col = g->col_idx;
  ta.n = (int32_t)g->n;
  ta.nb = io->plan.nb;
  ta.desc = io->plan.desc;
  ta.chunks = io->plan.chunks;
  ta.meta = io->plan.meta;
  ta.lcount = io->lcount;
  ta.lnorm = io->lnorm;
  ta.lpart = io->lpart;
  ta.xcd_order = ctx->tune.xcd_order;
  StatsArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.partials = io->partials;
  sa.lnorm = io->lnorm;
  sa.meta = io->plan.meta;
  sa.rayleigh = ray;
  for (int j = 0; j < nsteps; ++j) {
    ChebOp<W, LH> op;
    op.val = reinterpret_cast<const W*>(g->val);
    op.zin = basis[j];
    op.zprev = j > 0 ? basis[j - 1] : nullptr;
    op.zout = basis[j + 1];
    op.hinv = reinterpret_cast<const float*>(io->hinv);
    op.deg = io->deg;
    op.first = j == 0;
    sa.step = j;
    auto* ev = timing_start(ctx, s);
    if (ctx->tune.unroll == 4)
      hipLaunchKernelGGL((tile_kernel<4, ChebOp<W, LH>>), dim3(io->grid), dim3(kBlock), 0, s, op, ta, sa);
    else
      hipLaunchKernelGGL((tile_kernel<8, ChebOp<W, LH>>), dim3(io->grid), dim3(kBlock), 0, s, op, ta, sa);
    timing_stop(ev, s);
    hipLaunchKernelGGL((cheb_stats_finish<LH>), dim3(1), dim3(kBlock), 0, s, sa, io->grid);
  }
  return check_hip(hipGetLastError(), "chebyshev step launch");
}

// Rayleigh statistics of one block x (no output): ray row `row`.
template <typename W, int LH>
static int rayleigh_typed(Context* ctx, EmbedIO* io, const float* x, double* ray, int row, hipStream_t s) {
  const fsc_csr* g = io->g;
  TileArgs ta;
  ta.row_ptr = g->row_ptr;
  ta.col = g->col_idx;
  ta.n = (int32_t)g->n;
  ta.nb = io->plan.nb;
  ta.desc = io->plan.desc;
  ta.chunks = io->plan.chunks;
  ta.meta = io->plan.meta;
  ta.lcount = io->lcount;
  ta.lnorm = io->lnorm;
  ta.lpart = io->lpart;
  ta.xcd_order = ctx->tune.xcd_order;
  StatsArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.partials = io->partials;
  sa.lnorm = io->lnorm;
  sa.meta = io->plan.meta;
  sa.rayleigh = ray;
  sa.step = row;
  ChebOp<W, LH> op;
  op.val = reinterpret_cast<const W*>(g->val);
  op.zin = x;
  op.zprev = nullptr;
  op.zout = nullptr;
  op.hinv = reinterpret_cast<const float*>(io->hinv);
  op.deg = io->deg;
  op.first = 1;
  hipLaunchKernelGGL((tile_kernel<4, ChebOp<W, LH>>), dim3(io->grid), dim3(kBlock), 0, s, op, ta, sa);
  hipLaunchKernelGGL((cheb_stats_finish<LH>), dim3(1), dim3(kBlock), 0, s, sa, io->grid);
  return check_hip(hipGetLastError(), "rayleigh launch");
}

template <typename W>
static int cheb_dispatch(Context* ctx, EmbedIO* io, float* const* basis, int nsteps, double* ray, hipStream_t s) {
  switch (io->LH) {
    case 1: return cheb_steps_typed<W, 1>(ctx, io, basis, nsteps, ray, s);
    case 2: return cheb_steps_typed<W, 2>(ctx, io, basis, nsteps, ray, s);
    case 4: return cheb_steps_typed<W, 4>(ctx, io, basis, nsteps, ray, s);
    default: return cheb_steps_typed<W, 8>(ctx, io, basis, nsteps, ray, s);
  }
}

template <typename W>
static int ray_dispatch(Context* ctx, EmbedIO* io, const float* x, double* ray, int row, hipStream_t s) {
  switch (io->LH) {
    case 1: return rayleigh_typed<W, 1>(ctx, io, x, ray, row, s);
    case 2: return rayleigh_typed<W, 2>(ctx, io, x, ray, row, s);
    case 4: return rayleigh_typed<W, 4>(ctx, io, x, ray, row, s);
    default: return rayleigh_typed<W, 8>(ctx, io, x, ray, row, s);
  }
}

int cheb_basis_run(Context* ctx, EmbedIO* io, float* const* basis, double* ray, hipStream_t s) {
  // basis[0] is the start block Z0 (io->z[0] after embed_run with t = 0)
  if (io->g->val) return cheb_dispatch<float>(ctx, io, basis, 8, ray, s);
  return cheb_dispatch<void>(ctx, io, basis, 8, ray, s);
}

int rayleigh_run(Context* ctx, EmbedIO* io, const float* x, double* ray, int row, hipStream_t s) {
  if (io->g->val) return ray_dispatch<float>(ctx, io, x, ray, row, s);
  return ray_dispatch<void>(ctx, io, x, ray, row, s);
}

int gram_run(Context* ctx, const EmbedIO* io, float* const* basis, double* partials, int32_t* counter, double* out,
             hipStream_t s) {
  Blocks B;
  for (int j = 0; j < 9; ++j) B.b[j] = basis[j];
  const int32_t n = (int32_t)io->g->n;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, ctx->num_cu * 2));
  hipLaunchKernelGGL(gram_kernel, dim3(grid), dim3(kBlock), 0, s, B, io->deg, n, io->l, io->LH, partials, counter, out);
  return check_hip(hipGetLastError(), "gram launch");
}

// Blocks of the cluster-sums kernel: about 256 rows each, at most kSumsGrid.
constexpr int kSumsGrid = 512;

static int sums_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, kSumsGrid)); }

size_t scatter_workspace_bytes(int64_t n, int l, int k) {
  return align_up((size_t)sums_grid(n) * k * (9 * l + 1) * 8);
}

int scatter_run(const EmbedIO* io, float* const* basis, const int32_t* labels, int k, const double* gram,
                double* sums, double* within, double* total, hipStream_t s) {
  Blocks B;
  for (int j = 0; j < 9; ++j) B.b[j] = basis[j];
  const int32_t n = (int32_t)io->g->n;
  const int l = io->l, E = 9 * l + 1;
  const int grid = sums_grid(n);
  const int32_t chunk = (n + grid - 1) / grid;
  // LDS: k * E doubles (at most 64 * 73 * 8 = 37 KB) plus the staged labels
  hipLaunchKernelGGL(cluster_sums_kernel, dim3(grid), dim3(kBlock), (size_t)k * E * 8, s, B, labels, io->deg, n, l,
                     io->LH, k, chunk, sums);
  int rc = check_hip(hipGetLastError(), "cluster sums launch");
  if (rc) return rc;
  hipLaunchKernelGGL(scatter_finish_kernel, dim3(1), dim3(kBlock), (size_t)(k + 1) * E * 8, s, sums, grid, l, k, gram,
                     within, total);
  return check_hip(hipGetLastError(), "scatter finish launch");
}

int features_run(Context* ctx, const EmbedIO* io, int k, const double* ray, double* partials, int32_t* counter,
                 float* feat, hipStream_t s) {
  const int32_t n = (int32_t)io->g->n;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, ctx->num_cu * 2));
  hipLaunchKernelGGL(features_kernel, dim3(grid), dim3(kBlock), 0, s, io->deg, n, k, io->l, io->LH, ray, partials,
                     counter, feat);
  return check_hip(hipGetLastError(), "features launch");
}

int combine_run(const EmbedIO* io, float* const* basis, const float* c_rest, float* S, hipStream_t s) {
  Blocks B;
  for (int j = 0; j < 9; ++j) B.b[j] = basis[j];
  const int64_t count = io->g->n * io->LH;
  const int grid = (int)std::min<int64_t>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(combine_kernel, dim3(grid), dim3(256), 0, s, B, c_rest, count, S);
  return check_hip(hipGetLastError(), "combine launch");
}

int fallback_run(const EmbedIO* io, const double* ray, int row_f, int row_ref, const double* kcost, double kmax,
                 const float* c_rest, int32_t* used, double* diag, hipStream_t s) {
  hipLaunchKernelGGL(fallback_kernel, dim3(1), dim3(64), 0, s, ray, io->l, io->LH, row_f, row_ref, kcost, kmax, c_rest,
                     used, diag);
  return check_hip(hipGetLastError(), "fallback launch");
}

}  // namespace fsc
