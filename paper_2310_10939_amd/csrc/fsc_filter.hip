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
// features.  The Gram statistics <B_i, B_j>, <B_i, Y>, <Y, Y> (FP64, over the
// l columns) are what the trainer needs; the filtered embedding is
// S = sum_j c_j B_j with c_0 = 1 - sum_{j>0} c_j (so p(1) = 1).
#include "fsc_device.hpp"
#include "fsc_internal.hpp"
#include "fsc_tiles.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace fsc {

// Rayleigh-quotient epilogue: the last block writes, per column q,
// rayleigh[step * LH + q] = sum d z m / sum d z z.
template <int LH>
__device__ __forceinline__ void cheb_stats_epilogue(const StatsArgs& sa, const double* st) {
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ double tot[2 * LH];
  __shared__ int is_last;
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) {
    const double v = block_sum<kBlock>(st[q], red);
    if (threadIdx.x == 0) sa.partials[(int64_t)blockIdx.x * 2 * LH + q] = v;
  }
  if (threadIdx.x == 0) {
    __threadfence();
    const int prev = atomicAdd(sa.counter, 1);
    is_last = (prev == (int)gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const int32_t nlong = sa.meta[1];
  double v[2 * LH];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) v[q] = 0.0;
  for (int32_t g = threadIdx.x; g < (int32_t)gridDim.x; g += kBlock)
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
  if (threadIdx.x == 0) *sa.counter = 0;
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
      const float m = 0.5f * p.z[q] + p.h * acc[q];
      out[q] = first ? 2.f * m - p.z[q] : 4.f * m - 2.f * p.z[q] - p.zm[q];
      st[q] += p.d * (double)p.z[q] * (double)p.z[q];
      st[LH_ + q] += p.d * (double)p.z[q] * (double)m;
    }
    if (zout) rowio<float, LH_>::store(zout + (int64_t)r * LH_, out);
  }
};

// ---------------------------------------------------------------------------
// Gram statistics: G_ij = sum_v d_v <B_i[v], B_j[v]>, h_i = <B_i, Y>, yy.
// out: [0..81) G (both triangles), [81..90) h, [90] yy.
// ---------------------------------------------------------------------------
struct Blocks {
  const float* b[9];
};

constexpr int kGram = 45 + 9 + 1;

__global__ __launch_bounds__(kBlock) void gram_kernel(Blocks B, const float* __restrict__ Y,
                                                      const double* __restrict__ deg, int32_t n, int l, int LH,
                                                      double* __restrict__ partials, int32_t* __restrict__ counter,
                                                      double* __restrict__ out) {
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ int is_last;
  double acc[kGram];
#pragma unroll
  for (int i = 0; i < kGram; ++i) acc[i] = 0.0;
  for (int32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    const double d = deg[r];
    for (int q = 0; q < l; ++q) {
      double b[9];
#pragma unroll
      for (int i = 0; i < 9; ++i) b[i] = (double)B.b[i][(int64_t)r * LH + q];
      const double y = Y ? (double)Y[(int64_t)r * LH + q] : 0.0;
      int idx = 0;
#pragma unroll
      for (int i = 0; i < 9; ++i)
#pragma unroll
        for (int j = i; j < 9; ++j) acc[idx++] += d * b[i] * b[j];
#pragma unroll
      for (int i = 0; i < 9; ++i) acc[45 + i] += d * b[i] * y;
      acc[54] += d * y * y;
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
    if (k < 45) {
      int i = 0, base = 0;
      while (k >= base + (9 - i)) {
        base += 9 - i;
        ++i;
      }
      const int j = i + (k - base);
      out[i * 9 + j] = s;
      out[j * 9 + i] = s;
    } else {
      out[81 + (k - 45)] = s;
    }
  }
  if (threadIdx.x == 0) *counter = 0;
}

// ---------------------------------------------------------------------------
// Features: log n, log k, log mean degree, degree CV, log(max/mean degree)
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
  raw[3] = sqrt(var) / mean;
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
  sa.counter = io->counter;
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
  sa.counter = io->counter;
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

int gram_run(Context* ctx, const EmbedIO* io, float* const* basis, const float* Y, double* partials,
             int32_t* counter, double* out, hipStream_t s) {
  Blocks B;
  for (int j = 0; j < 9; ++j) B.b[j] = basis[j];
  const int32_t n = (int32_t)io->g->n;
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, ctx->num_cu * 2));
  hipLaunchKernelGGL(gram_kernel, dim3(grid), dim3(kBlock), 0, s, B, Y, io->deg, n, io->l, io->LH, partials, counter,
                     out);
  return check_hip(hipGetLastError(), "gram launch");
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
