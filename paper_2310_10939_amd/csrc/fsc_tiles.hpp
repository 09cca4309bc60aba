// Device-side tile machinery of the sparse product, shared by the single-graph
// and the batched kernels: the row operators (degree pass, one PowerMethod
// step) and the short-tile body.  See fsc_embed.hip for the tile layout.
#pragma once

#include <type_traits>

#include "fsc_device.hpp"
#include "fsc_internal.hpp"

namespace fsc {

constexpr int kBlock = 256;

struct StatsArgs;
template <int LH>
__device__ __forceinline__ void stats_epilogue(const StatsArgs& sa, const double* st);

__device__ __forceinline__ int64_t lower_bound_i64(const int64_t* a, int64_t len, int64_t x) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Lanes per row for a tile of R rows holding nz nonzeros: every row of the
// tile in one pass of the block, and no more lanes than the mean row length.
__device__ __forceinline__ int lanes_per_row(int64_t R, int64_t nz) {
  if (R <= 0) return 1;
  int g1 = 1;
  while (g1 * 2 * R <= kBlock && g1 < FSC_WAVE) g1 *= 2;
  const int64_t mean = nz / R;
  int g2 = 1;
  while (g2 < mean && g2 < FSC_WAVE) g2 *= 2;
  return g1 < g2 ? g1 : g2;
}

// ---------------------------------------------------------------------------
// Row-reduction operators
// ---------------------------------------------------------------------------
// acc += sum_u w[u] * Z[c[u]] over U gathered rows (c[u] < 0: skipped); all
// U loads are issued before the first use.
template <typename S, typename W, int LH, int U, typename A>
__device__ __forceinline__ void gather_rows(const S* __restrict__ z, const int32_t* c, const A* w, A* acc) {
  A zr[U][LH];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (c[u] >= 0) {
      rowio<S, LH>::load(z + (int64_t)c[u] * LH, zr[u]);
    } else {
#pragma unroll
      for (int q = 0; q < LH; ++q) zr[u][q] = A(0);
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int q = 0; q < LH; ++q) {
      if constexpr (std::is_void<W>::value) acc[q] += zr[u][q];
      else acc[q] += w[u] * zr[u][q];
    }
}

template <typename W, typename A>
__device__ __forceinline__ A load_weight(const W* val, int64_t j) {
  if constexpr (std::is_void<W>::value) {
    return A(1);
  } else if constexpr (std::is_same<W, bf16_t>::value) {
    return static_cast<A>(bf16_to_f32(nt_load(reinterpret_cast<const uint16_t*>(val) + j)));
  } else {
    return static_cast<A>(nt_load(val + j));
  }
}

// Degrees: d_v = sum of the weights of row v (Sec. 2; the graph has no
// self-loops, so this is sum_{u != v} w(u, v)), accumulated in FP64.  The
// epilogue writes d, 1/(2d), d^{-1/2} and the k-means eligibility mask.
template <typename W, typename HA>
struct DegreeOp {
  static constexpr int LH = 1;
  static constexpr bool STATS = false;
  using A = double;
  struct Pre {};
  const W* val;
  double* deg;
  HA* hinv;
  double* isq;
  uint8_t* elig;
  __device__ __forceinline__ void init() {}
  template <class SA>
  __device__ __forceinline__ void epilogue(const SA&, const double*) const {}
  template <int U>
  __device__ __forceinline__ void accumulate(const int32_t*, int64_t j0, int32_t stride, int64_t end,
                                             double* acc) const {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + (int64_t)u * stride;
      if (j < end) acc[0] += load_weight<W, double>(val, j);
    }
  }
  __device__ __forceinline__ void prefetch(int32_t, Pre&) const {}
  __device__ __forceinline__ void finish(int32_t r, const double* acc, const Pre&, double*) const {
    const double d = acc[0];
    deg[r] = d;
    hinv[r] = d > 0.0 ? static_cast<HA>(0.5 / d) : HA(0);
    isq[r] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    elig[r] = d > 0.0 ? 1 : 0;
  }
};

// a * b + c with one rounding, for the accumulation type
__device__ __forceinline__ float fma_acc(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One PowerMethod step in z-space with a per-column scale c (1 unless the
// iterate is re-normalised):
//   Z'_r = c (.) (Z_r / 2 + hinv_r (A Z)_r).
// With STATS the epilogue accumulates, per column, sum_r d_r Z'_r^2 (the
// y-space squared norm of the stored iterate) and sum_r d_r Z_r (Z_r/2 +
// hinv_r (A Z)_r) (y_{i-1}^T M y_{i-1}, the Rayleigh numerator).
template <typename S, typename W, int LH_, bool STATS_>
struct StepOp {
  static constexpr int LH = LH_;
  static constexpr bool STATS = STATS_;
  using A = typename elem<S>::acc;
  struct Pre {
    A z[LH_];
    A h;
    double d;
  };
  const W* val;
  const W* sval;   // weights in slab order (column-slab product only)
  const S* zin;
  S* zout;
  const A* hinv;
  const double* deg;
  const A* scale;  // per-column scale of this step (device), or null for 1
  A cs[LH_];
  __device__ __forceinline__ void init() {
#pragma unroll
    for (int q = 0; q < LH_; ++q) cs[q] = scale ? scale[q] : A(1);
  }
  template <int U>
  __device__ __forceinline__ void accumulate(const int32_t* col, int64_t j0, int32_t stride, int64_t end,
                                             A* acc) const {
    int32_t c[U];
    A w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + (int64_t)u * stride;
      const bool ok = j < end;
      c[u] = ok ? nt_load(col + j) : -1;
      w[u] = ok ? load_weight<W, A>(val, j) : A(0);
    }
    gather_rows<S, W, LH_, U>(zin, c, w, acc);
  }
  // The same over positions reg + off[u] of the slab-ordered copy (off < 0:
  // none); reg is uniform, so the loads take a scalar base and 32-bit offsets.
  // The stored index plus cbase is the column (16-bit slab-local indices
  // with the slab's first column, or 32-bit columns with 0).  UNIT: every
  // weight there is 1, so none is loaded.
  template <int U, bool UNIT, typename CI>
  __device__ __forceinline__ void accumulate_at(const CI* scol, int64_t reg, const int32_t* off, int32_t cbase,
                                                A* acc) const {
    const CI* cp = scol + reg;
    int32_t c[U];
    A w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) c[u] = off[u] >= 0 ? cbase + (int32_t)nt_load(cp + off[u]) : -1;
    if constexpr (std::is_void<W>::value || UNIT) {
#pragma unroll
      for (int u = 0; u < U; ++u) w[u] = A(1);
      gather_rows<S, void, LH_, U>(zin, c, w, acc);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) w[u] = off[u] >= 0 ? load_weight<W, A>(sval + reg, off[u]) : A(0);
      gather_rows<S, W, LH_, U>(zin, c, w, acc);
    }
  }
  // Two rows at once (offsets off0 into acc0, off1 into acc1): every index,
  // weight and row load of both is issued before the first use; each row's
  // sum is built in the same order as by accumulate_at.
  template <int U, bool UNIT, typename CI>
  __device__ __forceinline__ void accumulate_at2(const CI* scol, int64_t reg, const int32_t* off0,
                                                 const int32_t* off1, int32_t cbase, A* acc0, A* acc1) const {
    const CI* cp = scol + reg;
    int32_t c[2 * U];
    A w[2 * U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      c[u] = off0[u] >= 0 ? cbase + (int32_t)nt_load(cp + off0[u]) : -1;
      c[U + u] = off1[u] >= 0 ? cbase + (int32_t)nt_load(cp + off1[u]) : -1;
    }
    if constexpr (std::is_void<W>::value || UNIT) {
#pragma unroll
      for (int u = 0; u < 2 * U; ++u) w[u] = A(1);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        w[u] = off0[u] >= 0 ? load_weight<W, A>(sval + reg, off0[u]) : A(0);
        w[U + u] = off1[u] >= 0 ? load_weight<W, A>(sval + reg, off1[u]) : A(0);
      }
    }
    A zr[2 * U][LH_];
#pragma unroll
    for (int u = 0; u < 2 * U; ++u) {
      if (c[u] >= 0) {
        rowio<S, LH_>::load(zin + (int64_t)c[u] * LH_, zr[u]);
      } else {
#pragma unroll
        for (int q = 0; q < LH_; ++q) zr[u][q] = A(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < LH_; ++q) {
        if constexpr (std::is_void<W>::value || UNIT) {
          acc0[q] += zr[u][q];
          acc1[q] += zr[U + u][q];
        } else {
          acc0[q] += w[u] * zr[u][q];
          acc1[q] += w[U + u] * zr[U + u][q];
        }
      }
  }
  __device__ __forceinline__ void prefetch(int32_t r, Pre& p) const {
    rowio<S, LH_>::load(zin + (int64_t)r * LH_, p.z);
    p.h = hinv[r];
    if constexpr (STATS_) p.d = deg[r];
  }
  template <class SA>
  __device__ __forceinline__ void epilogue(const SA& sa, const double* st) const {
    stats_epilogue<LH_>(sa, st);
  }
  __device__ __forceinline__ void finish(int32_t r, const A* acc, const Pre& p, double* st) const {
    A zn[LH_];
#pragma unroll
    for (int q = 0; q < LH_; ++q) {
      // one explicit fused multiply-add, so every kernel that inlines this
      // rounds the same way
      const A m = fma_acc(p.h, acc[q], A(0.5) * p.z[q]);
      zn[q] = cs[q] * m;
      if constexpr (STATS_) {
        // statistics of the value that is actually stored
        zn[q] = elem<S>::to_acc(elem<S>::from_acc(zn[q]));
        st[q] += p.d * (double)zn[q] * (double)zn[q];
        st[LH_ + q] += p.d * (double)p.z[q] * (double)m;
      }
    }
    rowio<S, LH_>::store(zout + (int64_t)r * LH_, zn);
  }
};

// ---------------------------------------------------------------------------
// Tile arguments and the short-tile body
// ---------------------------------------------------------------------------
struct TileArgs {
  const int64_t* row_ptr;
  const int32_t* col;
  int32_t n;
  int32_t nb;
  const TileDesc* desc;
  const LongChunk* chunks;
  const int32_t* meta;
  void* lpart;        // A[chunks][LH]
  int32_t* lcount;    // [long rows]
  double* lnorm;      // [long rows][2*LH] (STATS)
  int xcd_order;      // 1: each XCD takes a contiguous range of short tiles
};

template <int LH, typename A>
__device__ __forceinline__ void group_reduce(A* acc, int G) {
  for (int m = G >> 1; m >= 1; m >>= 1)
#pragma unroll
    for (int q = 0; q < LH; ++q) acc[q] += shfl_xor(acc[q], m);
}

template <int kU, class Op>
__device__ __forceinline__ void short_tile(const Op& op, const TileArgs& ta, const TileDesc d, double* st) {
  constexpr int LH = Op::LH;
  using A = typename Op::A;
  const int G = d.G;
  const int ngroups = kBlock / G;
  const int gid = threadIdx.x / G, lane = threadIdx.x % G;
  for (int32_t rbase = d.r0; rbase < d.r1; rbase += ngroups) {
    const int32_t r = rbase + gid;
    const bool active = r < d.r1;
    A acc[LH];
#pragma unroll
    for (int q = 0; q < LH; ++q) acc[q] = A(0);
    typename Op::Pre pre;
    if (active) {
      if (lane == 0) op.prefetch(r, pre);
      const int64_t a = ta.row_ptr[r], b = ta.row_ptr[r + 1];
      for (int64_t j0 = a + lane; j0 < b; j0 += (int64_t)G * kU)
        op.template accumulate<kU>(ta.col, j0, G, b, acc);
    }
    group_reduce<LH, A>(acc, G);
    if (active && lane == 0) op.finish(r, acc, pre, st);
  }
}

// ---------------------------------------------------------------------------
// Column statistics of a step, finished by one block after the step.
// state: [0..LH) prev_sq, [LH..2LH) cum (product of applied scales),
//        [2LH..3LH) next scale (FP64), [3LH..4LH) next scale in the step's
//        accumulation type.
// ---------------------------------------------------------------------------
struct StatsArgs {
  double* partials;     // [grid][2*LH]
  const double* lnorm;  // [long rows][2*LH]
  const int32_t* meta;  // meta[1] = long rows
  double* state;
  double* sqnorm;       // optional (t+1) x l
  double* rayleigh;     // optional t x l
  int step, t, l, renorm;
  int acc_is_double;
};

constexpr int kFinish = 256;  // threads of the statistics finish

// The column statistics of a step from their block sums tot[0..2LH): the
// squared norms, the Rayleigh quotients of the previous step, the scales.
template <int LH>
__device__ void stats_apply(const StatsArgs& sa, const double* tot);

template <int LH>
__device__ void stats_finish(const StatsArgs& sa, int grid) {
  __shared__ double red[2 * LH * (kFinish / FSC_WAVE)];
  __shared__ double tot[2 * LH];
  const int32_t nlong = sa.step > 0 ? sa.meta[1] : 0;
  double v[2 * LH];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) v[q] = 0.0;
  for (int32_t g = threadIdx.x; g < grid; g += kFinish)
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) v[q] += sa.partials[(int64_t)g * 2 * LH + q];
  for (int32_t g = threadIdx.x; g < nlong; g += kFinish)
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) v[q] += sa.lnorm[(int64_t)g * 2 * LH + q];
  block_sum_n<kFinish, 2 * LH>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) tot[q] = v[q];
  __syncthreads();
  stats_apply<LH>(sa, tot);
}

// The same finish by one block of a later kernel (a block that has no other
// work there): one sum at a time, so that it adds few registers to that
// kernel.  Each sum is formed as above (per thread in the same order, then
// the wave sums, then the wave totals in order), so the bits are the same.
template <int LH>
__device__ void stats_finish_lean(const StatsArgs& sa, int grid) {
  static_assert(kFinish == kBlock, "the finishing block has the finish's width");
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ double tot[2 * LH];
  const int32_t nlong = sa.step > 0 ? sa.meta[1] : 0;
#pragma unroll 1
  for (int q = 0; q < 2 * LH; ++q) {
    double v = 0.0;
    for (int32_t g = threadIdx.x; g < grid; g += kBlock) v += sa.partials[(int64_t)g * 2 * LH + q];
    for (int32_t g = threadIdx.x; g < nlong; g += kBlock) v += sa.lnorm[(int64_t)g * 2 * LH + q];
    const double t = block_sum<kBlock>(v, red);
    if (threadIdx.x == 0) tot[q] = t;
  }
  __syncthreads();
  stats_apply<LH>(sa, tot);
}

// A step's statistics left to be finished inside the next step kernel
// (grid = 0: none): its partials come from `grid` blocks.
struct PendingFinish {
  StatsArgs sa;
  int grid;
};

template <int LH>
__device__ void stats_apply(const StatsArgs& sa, const double* tot) {
  if (threadIdx.x < LH) {
    const int q = threadIdx.x;
    double* prev_sq = sa.state;
    double* cum = sa.state + LH;
    double* next = sa.state + 2 * LH;
    const double sq = tot[q];
    if (sa.step == 0) {
      cum[q] = 1.0;
    } else {
      cum[q] *= next[q];
      if (sa.rayleigh && q < sa.l) {
        const double den = prev_sq[q];
        sa.rayleigh[(int64_t)(sa.step - 1) * sa.l + q] = den > 0.0 ? tot[LH + q] / den : 0.0;
      }
    }
    if (sa.sqnorm && q < sa.l) sa.sqnorm[(int64_t)sa.step * sa.l + q] = sq / (cum[q] * cum[q]);
    prev_sq[q] = sq;
    double c = 1.0;
    if (sa.renorm) {
      if (sa.step + 1 < sa.t) c = sq > 0.0 ? 1.0 / sqrt(sq) : 1.0;
      else c = 1.0 / cum[q];  // the last step restores the un-normalised scale
    }
    next[q] = c;
    if (sa.acc_is_double) reinterpret_cast<double*>(sa.state + 3 * LH)[q] = c;
    else reinterpret_cast<float*>(sa.state + 3 * LH)[q] = (float)c;
  }
}

// Writes this block's partial statistics.  They are finished by
// stats_finish_kernel, launched after the kernel on the same stream, or by a
// block of the next step kernel (PendingFinish): a last-block finish inside
// the same kernel would need a device-scope release by every block, which
// writes back its XCD's L2 and cost 15% of a power step.
// Called by every thread of every block.
template <int LH>
__device__ __forceinline__ void stats_epilogue(const StatsArgs& sa, const double* st) {
  __shared__ double red[kBlock / FSC_WAVE];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) {
    const double v = block_sum<kBlock>(st[q], red);
    if (threadIdx.x == 0) sa.partials[(int64_t)blockIdx.x * 2 * LH + q] = v;
  }
}

// One block: the statistics of a step from the `grid` partials of the kernel
// that wrote them (in a fixed order, so deterministic).
template <int LH>
__global__ __launch_bounds__(kFinish) void stats_finish_kernel(StatsArgs sa, int grid) {
  stats_finish<LH>(sa, grid);
}

// ---------------------------------------------------------------------------
// Row-reduction operators run by the tile kernel
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// The tile kernel: short tiles, then long-row chunks, then the operator's
// statistics epilogue
// ---------------------------------------------------------------------------
template <int kU, class Op>
__device__ __forceinline__ void long_chunk(const Op& op, const TileArgs& ta, int32_t ci) {
  constexpr int LH = Op::LH;
  using A = typename Op::A;
  __shared__ A wred[kBlock / FSC_WAVE][LH];
  __shared__ int is_last;
  const LongChunk ch = ta.chunks[ci];
  A acc[LH];
#pragma unroll
  for (int q = 0; q < LH; ++q) acc[q] = A(0);
  for (int64_t j0 = ch.start + threadIdx.x; j0 < ch.end; j0 += (int64_t)kBlock * kU)
    op.template accumulate<kU>(ta.col, j0, kBlock, ch.end, acc);
  group_reduce<LH, A>(acc, FSC_WAVE);
  const int w = threadIdx.x / FSC_WAVE;
  if ((threadIdx.x & (FSC_WAVE - 1)) == 0)
#pragma unroll
    for (int q = 0; q < LH; ++q) wred[w][q] = acc[q];
  __syncthreads();
  A* lpart = reinterpret_cast<A*>(ta.lpart);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < LH; ++q) {
      A sum = A(0);
      for (int i = 0; i < kBlock / FSC_WAVE; ++i) sum += wred[i][q];
      lpart[(int64_t)ci * LH + q] = sum;
    }
    __threadfence();
    const int prev = atomicAdd(&ta.lcount[ch.lid], 1);
    is_last = (prev == ch.count - 1);
  }
  __syncthreads();
  if (is_last && threadIdx.x == 0) {
    __threadfence();
    A tot[LH];
#pragma unroll
    for (int q = 0; q < LH; ++q) tot[q] = A(0);
    for (int c = 0; c < ch.count; ++c)
#pragma unroll
      for (int q = 0; q < LH; ++q) tot[q] += lpart[(int64_t)(ch.first + c) * LH + q];
    double lst[2 * LH];
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) lst[q] = 0.0;
    typename Op::Pre pre;
    op.prefetch(ch.row, pre);
    op.finish(ch.row, tot, pre, lst);
    if constexpr (Op::STATS) {
#pragma unroll
      for (int q = 0; q < 2 * LH; ++q) ta.lnorm[(int64_t)ch.lid * 2 * LH + q] = lst[q];
    }
    ta.lcount[ch.lid] = 0;  // ready for the next step
  }
  __syncthreads();
}

template <int kU, class Op>
__global__ __launch_bounds__(kBlock) void tile_kernel(Op op_in, TileArgs ta, StatsArgs sa) {
  constexpr int LH = Op::LH;
  Op op = op_in;
  op.init();
  const int32_t nb = ta.nb;
  const int32_t ntiles = nb + ta.meta[0];
  double st[2 * LH];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) st[q] = 0.0;

  if (ta.xcd_order) {
    // blocks are dispatched to the 8 XCDs round-robin: give XCD x the
    // contiguous range [x*nb/8, (x+1)*nb/8) of short tiles
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3, per = gridDim.x >> 3;
    const int32_t lo = (int32_t)((int64_t)nb * x / 8), hi = (int32_t)((int64_t)nb * (x + 1) / 8);
    for (int32_t tile = lo + slot; tile < hi; tile += per) short_tile<kU>(op, ta, ta.desc[tile], st);
  } else {
    for (int32_t tile = blockIdx.x; tile < nb; tile += gridDim.x) short_tile<kU>(op, ta, ta.desc[tile], st);
  }
  for (int32_t tile = nb + blockIdx.x; tile < ntiles; tile += gridDim.x) long_chunk<kU>(op, ta, tile - nb);
  if constexpr (Op::STATS) op.epilogue(sa, st);
}

}  // namespace fsc
