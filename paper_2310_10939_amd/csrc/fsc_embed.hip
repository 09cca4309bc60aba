// The embedding D^{-1/2} Y of FastSpectralCluster (Algorithm 2) on gfx950.
//
// Everything runs in z-space, Z = D^{-1/2} Y: one PowerMethod step
// (Algorithm 1) with the halved signless Laplacian M = (I + D^{-1/2} A
// D^{-1/2}) / 2 (Sec. 2) becomes
//     Z' = Z / 2 + (1 / (2 d)) (.) (A Z),
// so the degree scaling is one multiply per row and Z_t is the embedding
// itself.  The sparse product is the only pass over the graph per step.
//
// Sparse product layout ("tiles"): the nonzeros are cut into buckets of
// tile_nnz; bucket b owns the rows whose first nonzero lies in
// [b*tile_nnz, (b+1)*tile_nnz).  A bucket holds at most 2*tile_nnz nonzeros of
// rows no longer than tile_nnz, plus possibly one longer last row; such long
// rows are cut into chunks of tile_nnz processed by separate tiles whose
// partial sums are combined, in chunk order, by the tile that finishes last.
// A short tile streams its nonzeros with fully coalesced reads of col/val,
// gathers the l-wide rows of Z, stages the weighted rows in LDS and then sums
// each matrix row with a lane group sized to the tile's mean row length
// (wave-shuffle reduction).  The grid is persistent: block g takes tiles g,
// g + grid, ... so per-block statistics are deterministic.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>
#include <type_traits>

namespace fsc {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Tile plan
// ---------------------------------------------------------------------------
__device__ __forceinline__ int64_t lower_bound_i64(const int64_t* a, int64_t len, int64_t x) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void plan_buckets(const int64_t* __restrict__ row_ptr, int32_t n, int32_t nb, int32_t NB,
                             int32_t* __restrict__ rb, int32_t* __restrict__ nch) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t r0 = min<int64_t>(lower_bound_i64(row_ptr, (int64_t)n + 1, (int64_t)b * NB), n);
  const int64_t r1 = min<int64_t>(lower_bound_i64(row_ptr, (int64_t)n + 1, (int64_t)(b + 1) * NB), n);
  rb[b] = (int32_t)r0;
  if (b == nb - 1) rb[nb] = n;
  int32_t c = 0;
  if (r1 > r0) {
    const int64_t len = row_ptr[r1] - row_ptr[r1 - 1];
    if (len > NB) c = (int32_t)((len + NB - 1) / NB);
  }
  nch[b] = c;
}

// Exclusive scans of nch and of (nch > 0), one block.
__global__ __launch_bounds__(1024) void plan_scan(const int32_t* __restrict__ nch, int32_t nb,
                                                  int32_t* __restrict__ choff, int32_t* __restrict__ lid,
                                                  int32_t* __restrict__ meta) {
  __shared__ int32_t sa[1024], sb[1024];
  int32_t carry_a = 0, carry_b = 0;
  for (int32_t base = 0; base < nb; base += 1024) {
    const int32_t i = base + threadIdx.x;
    const int32_t va = i < nb ? nch[i] : 0;
    const int32_t vb = i < nb ? (nch[i] > 0) : 0;
    sa[threadIdx.x] = va;
    sb[threadIdx.x] = vb;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      int32_t xa = threadIdx.x >= off ? sa[threadIdx.x - off] : 0;
      int32_t xb = threadIdx.x >= off ? sb[threadIdx.x - off] : 0;
      __syncthreads();
      sa[threadIdx.x] += xa;
      sb[threadIdx.x] += xb;
      __syncthreads();
    }
    if (i < nb) {
      choff[i] = carry_a + sa[threadIdx.x] - va;
      lid[i] = carry_b + sb[threadIdx.x] - vb;
    }
    carry_a += sa[1023];
    carry_b += sb[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    choff[nb] = carry_a;
    lid[nb] = carry_b;
    meta[0] = carry_a;
    meta[1] = carry_b;
  }
}

__global__ void plan_chunks(const int64_t* __restrict__ row_ptr, int32_t nb, int32_t NB,
                            const int32_t* __restrict__ rb, const int32_t* __restrict__ nch,
                            const int32_t* __restrict__ choff, const int32_t* __restrict__ lid,
                            LongChunk* __restrict__ chunks) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb || nch[b] == 0) return;
  const int32_t r = rb[b + 1] - 1;
  const int64_t rs = row_ptr[r], re = row_ptr[r + 1];
  const int32_t cnt = nch[b], first = choff[b];
  for (int32_t c = 0; c < cnt; ++c) {
    LongChunk ch;
    ch.start = rs + (int64_t)c * NB;
    ch.end = min<int64_t>(ch.start + NB, re);
    ch.row = r;
    ch.lid = lid[b];
    ch.index = c;
    ch.count = cnt;
    ch.first = first;
    ch.pad = 0;
    chunks[first + c] = ch;
  }
}

__global__ void fill_i32(int32_t* p, int64_t count, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// Row-reduction operators run by the tile kernel
// ---------------------------------------------------------------------------
// Degrees: d_v = sum of the weights of row v (Sec. 2; the graph has no
// self-loops, so this is sum_{u != v} w(u, v)), accumulated in FP64.  The
// epilogue writes d, 1/(2d), d^{-1/2} and the k-means eligibility mask.
template <typename W, typename HA>
struct DegreeOp {
  static constexpr int LH = 1;
  static constexpr bool STATS = false;
  using A = double;
  const W* val;
  double* deg;
  HA* hinv;
  double* isq;
  uint8_t* elig;
  __device__ __forceinline__ void init() {}
  template <int U>
  __device__ __forceinline__ void gather_many(const int64_t* j, const int32_t*, const bool* ok,
                                              double (*out)[1]) const {
#pragma unroll
    for (int u = 0; u < U; ++u) out[u][0] = ok[u] ? weight<W, double>::get(val, j[u]) : 0.0;
  }
  __device__ __forceinline__ void finish(int32_t r, const double* acc, double*) const {
    const double d = acc[0];
    deg[r] = d;
    hinv[r] = d > 0.0 ? static_cast<HA>(0.5 / d) : HA(0);
    isq[r] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    elig[r] = d > 0.0 ? 1 : 0;
  }
};

// One PowerMethod step in z-space with an optional per-column scale c:
//   Z'_r = c (.) (Z_r / 2 + hinv_r (A Z)_r).
// With STATS the epilogue accumulates, per column, sum_r d_r Z'_r^2 and
// sum_r d_r Z_r (Z_r/2 + hinv_r (A Z)_r) (y-space norm and the numerator of
// the Rayleigh quotient of the previous iterate).
template <typename S, typename W, int LH_, bool STATS_>
struct StepOp {
  static constexpr int LH = LH_;
  static constexpr bool STATS = STATS_;
  using A = typename elem<S>::acc;
  const W* val;
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
  __device__ __forceinline__ void gather_many(const int64_t* j, const int32_t* c, const bool* ok,
                                              A (*out)[LH_]) const {
    A w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) w[u] = ok[u] ? weight<W, A>::get(val, j[u]) : A(0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (ok[u]) {
        rowio<S, LH_>::load(zin + (int64_t)c[u] * LH_, out[u]);
      } else {
#pragma unroll
        for (int q = 0; q < LH_; ++q) out[u][q] = A(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int q = 0; q < LH_; ++q) out[u][q] *= w[u];
  }
  __device__ __forceinline__ void finish(int32_t r, const A* acc, double* st) const {
    A z[LH_], zn[LH_];
    rowio<S, LH_>::load(zin + (int64_t)r * LH_, z);
    const A h = hinv[r];
#pragma unroll
    for (int q = 0; q < LH_; ++q) {
      const A m = A(0.5) * z[q] + h * acc[q];
      zn[q] = cs[q] * m;
      if constexpr (STATS_) {
        // statistics from the value that is actually stored
        zn[q] = elem<S>::to_acc(elem<S>::from_acc(zn[q]));
        const double d = deg[r];
        st[q] += d * (double)zn[q] * (double)zn[q];
        st[LH_ + q] += d * (double)z[q] * (double)m;
      }
    }
    rowio<S, LH_>::store(zout + (int64_t)r * LH_, zn);
  }
};

// ---------------------------------------------------------------------------
// The tile kernel
// ---------------------------------------------------------------------------
struct TileArgs {
  const int64_t* row_ptr;
  const int32_t* col;
  int32_t n;
  int32_t nb;
  int32_t NB;
  const int32_t* rb;
  const LongChunk* chunks;
  const int32_t* meta;
  double* partials;   // [grid][2*LH] (STATS)
  void* lpart;        // A[chunks][LH]
  int32_t* lcount;    // [long rows]
  double* lnorm;      // [long rows][2*LH] (STATS)
};

template <int LH, typename A>
__device__ __forceinline__ void group_reduce(A* acc, int G) {
  for (int m = G >> 1; m >= 1; m >>= 1)
#pragma unroll
    for (int q = 0; q < LH; ++q) acc[q] += shfl_xor(acc[q], m);
}

template <class Op>
__global__ __launch_bounds__(kBlock) void tile_kernel(Op op_in, TileArgs ta) {
  constexpr int LH = Op::LH;
  Op op = op_in;
  op.init();
  using A = typename Op::A;
  constexpr int U = 4;  // nonzeros in flight per thread
  extern __shared__ __align__(16) unsigned char smem_raw[];
  A* prod = reinterpret_cast<A*>(smem_raw);  // [2*NB][LH]
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ A wred[kBlock / FSC_WAVE][LH];
  __shared__ int is_last;

  const int tid = threadIdx.x;
  const int32_t NB = ta.NB;
  const int32_t nb = ta.nb;
  const int32_t ntiles = nb + ta.meta[0];
  double st[2 * LH];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) st[q] = 0.0;

  for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    if (tile < nb) {
      // ------------------------------ short tile ----------------------------
      const int32_t r0 = ta.rb[tile];
      int32_t r1 = ta.rb[tile + 1];
      if (r1 > r0 && ta.row_ptr[r1] - ta.row_ptr[r1 - 1] > NB) --r1;  // long last row
      const int64_t s = ta.row_ptr[r0];
      const int32_t ne = (int32_t)(ta.row_ptr[r1] - s);
      // phase 1: stream nonzeros, gather, weight, stage in LDS
      for (int32_t base = 0; base < ne; base += kBlock * U) {
        int64_t jj[U];
        int32_t cc[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t j = base + u * kBlock + tid;
          ok[u] = j < ne;
          jj[u] = s + j;
          cc[u] = ok[u] ? ta.col[s + j] : 0;
        }
        A v[U][LH];
        op.template gather_many<U>(jj, cc, ok, v);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int32_t j = base + u * kBlock + tid;
          if (ok[u]) {
#pragma unroll
            for (int q = 0; q < LH; ++q) prod[j * LH + q] = v[u][q];
          }
        }
      }
      __syncthreads();
      // phase 2: one lane group per row
      const int32_t R = r1 - r0;
      if (R > 0) {
        int G = 1;
        {
          const int32_t fit = kBlock / R;          // groups that fit in one pass
          const int32_t mean = ne / R;
          int g1 = 1;
          while (g1 * 2 <= fit && g1 < FSC_WAVE) g1 *= 2;
          int g2 = 1;
          while (g2 * 4 < mean && g2 < FSC_WAVE) g2 *= 2;
          G = g1 < g2 ? g1 : g2;
        }
        const int ngroups = kBlock / G;
        const int gid = tid / G, lane = tid % G;
        for (int32_t rbase = r0; rbase < r1; rbase += ngroups) {
          const int32_t r = rbase + gid;
          const bool active = r < r1;
          A acc[LH];
#pragma unroll
          for (int q = 0; q < LH; ++q) acc[q] = A(0);
          if (active) {
            const int32_t a = (int32_t)(ta.row_ptr[r] - s), e = (int32_t)(ta.row_ptr[r + 1] - s);
            for (int32_t j = a + lane; j < e; j += G)
#pragma unroll
              for (int q = 0; q < LH; ++q) acc[q] += prod[j * LH + q];
          }
          group_reduce<LH, A>(acc, G);
          if (active && lane == 0) op.finish(r, acc, st);
        }
      }
      __syncthreads();
    } else {
      // ------------------------------ long-row chunk -------------------------
      const int32_t ci = tile - nb;
      const LongChunk ch = ta.chunks[ci];
      A acc[LH];
#pragma unroll
      for (int q = 0; q < LH; ++q) acc[q] = A(0);
      for (int64_t base = ch.start; base < ch.end; base += kBlock * U) {
        int64_t jj[U];
        int32_t cc[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t j = base + u * kBlock + tid;
          ok[u] = j < ch.end;
          jj[u] = j;
          cc[u] = ok[u] ? ta.col[j] : 0;
        }
        A v[U][LH];
        op.template gather_many<U>(jj, cc, ok, v);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int q = 0; q < LH; ++q) acc[q] += v[u][q];
      }
      // block reduction in a fixed order
      group_reduce<LH, A>(acc, FSC_WAVE);
      const int w = tid / FSC_WAVE;
      if ((tid & (FSC_WAVE - 1)) == 0)
#pragma unroll
        for (int q = 0; q < LH; ++q) wred[w][q] = acc[q];
      __syncthreads();
      A* lpart = reinterpret_cast<A*>(ta.lpart);
      if (tid == 0) {
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
      if (is_last && tid == 0) {
        __threadfence();
        A tot[LH];
#pragma unroll
        for (int q = 0; q < LH; ++q) tot[q] = A(0);
        for (int c = 0; c < ch.count; ++c)
#pragma unroll
          for (int q = 0; q < LH; ++q)
            tot[q] += lpart[(int64_t)(ch.first + c) * LH + q];
        double lst[2 * LH];
#pragma unroll
        for (int q = 0; q < 2 * LH; ++q) lst[q] = 0.0;
        op.finish(ch.row, tot, lst);
        if constexpr (Op::STATS) {
#pragma unroll
          for (int q = 0; q < 2 * LH; ++q) ta.lnorm[(int64_t)ch.lid * 2 * LH + q] = lst[q];
        }
        ta.lcount[ch.lid] = 0;  // ready for the next step
      }
      __syncthreads();
    }
  }
  if constexpr (Op::STATS) {
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) {
      const double v = block_sum<kBlock>(st[q], red);
      if (tid == 0) ta.partials[(int64_t)blockIdx.x * 2 * LH + q] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Start block: Z0 = D^{-1/2} X0, X0 Gaussian (Algorithm 2) or given.
// ---------------------------------------------------------------------------
template <typename S, int LH>
__global__ __launch_bounds__(kBlock) void start_block(int32_t n, int32_t l, uint32_t k0, uint32_t k1,
                                                      const double* __restrict__ x0,
                                                      const double* __restrict__ isq,
                                                      const double* __restrict__ deg, S* __restrict__ z,
                                                      double* __restrict__ partials, int stats) {
  using A = typename elem<S>::acc;
  __shared__ double red[kBlock / FSC_WAVE];
  double st[LH];
#pragma unroll
  for (int q = 0; q < LH; ++q) st[q] = 0.0;
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double s = isq[i];
    A row[LH];
#pragma unroll
    for (int q = 0; q < LH; ++q) {
      double x = 0.0;
      if (q < l) {
        if (x0) {
          x = x0[(int64_t)i * l + q];
        } else {
          const u32x4 r = philox4x32_10(u32x4{(uint32_t)i, 0u, (uint32_t)q, 0u}, k0, k1);
          const double u1 = uniform53(r.x, r.y), u2 = uniform53(r.z, r.w);
          x = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
        }
      }
      row[q] = elem<S>::to_acc(elem<S>::from_acc(static_cast<A>(s * x)));
      st[q] += deg[i] * (double)row[q] * (double)row[q];
    }
    rowio<S, LH>::store(z + (int64_t)i * LH, row);
  }
  if (stats) {
#pragma unroll
    for (int q = 0; q < LH; ++q) {
      const double v = block_sum<kBlock>(st[q], red);
      if (threadIdx.x == 0) {
        partials[(int64_t)blockIdx.x * 2 * LH + q] = v;
        partials[(int64_t)blockIdx.x * 2 * LH + LH + q] = 0.0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Column statistics after step `step` (0 = the start block), one block.
// state: [0] prev_sq, [1] cum (product of applied scales), [2] next scale.
// ---------------------------------------------------------------------------
template <int LH>
__global__ __launch_bounds__(kBlock) void finish_stats(const double* __restrict__ partials, int32_t grid,
                                                      const double* __restrict__ lnorm,
                                                      const int32_t* __restrict__ meta, int step, int t, int l,
                                                      int renorm, double* __restrict__ state,
                                                      double* __restrict__ sqnorm, double* __restrict__ rayleigh,
                                                      float* __restrict__ scale_f, double* __restrict__ scale_d) {
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ double tot[2 * LH];
  const int32_t nlong = step > 0 ? meta[1] : 0;
  for (int q = 0; q < 2 * LH; ++q) {
    double v = 0.0;
    for (int32_t g = threadIdx.x; g < grid; g += kBlock) v += partials[(int64_t)g * 2 * LH + q];
    for (int32_t g = threadIdx.x; g < nlong; g += kBlock) v += lnorm[(int64_t)g * 2 * LH + q];
    v = block_sum<kBlock>(v, red);
    if (threadIdx.x == 0) tot[q] = v;
  }
  __syncthreads();
  if (threadIdx.x < LH) {
    const int q = threadIdx.x;
    double* prev_sq = state;
    double* cum = state + LH;
    double* next = state + 2 * LH;
    const double sq = tot[q];
    double c_applied = 1.0;
    if (step == 0) {
      cum[q] = 1.0;
    } else {
      c_applied = next[q];
      cum[q] *= c_applied;
      if (rayleigh && q < l) {
        const double den = prev_sq[q];
        rayleigh[(int64_t)(step - 1) * l + q] = den > 0.0 ? tot[LH + q] / den : 0.0;
      }
    }
    if (sqnorm && q < l) sqnorm[(int64_t)step * l + q] = sq / (cum[q] * cum[q]);
    prev_sq[q] = sq;
    double c = 1.0;
    if (renorm) {
      if (step + 1 < t) c = sq > 0.0 ? 1.0 / sqrt(sq) : 1.0;
      else c = 1.0 / cum[q];  // the last step restores the un-normalised scale
    }
    next[q] = c;
    if (scale_f) scale_f[q] = (float)c;
    if (scale_d) scale_d[q] = c;
  }
}

// ---------------------------------------------------------------------------
// Output conversions
// ---------------------------------------------------------------------------
template <typename S, int LH>
__global__ void unpad_rows(const S* __restrict__ z, int32_t n, int32_t l, S* __restrict__ out) {
  const int64_t total = (int64_t)n * l;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / l;
    const int q = (int)(i - r * l);
    out[i] = z[r * LH + q];
  }
}

template <typename S, int LH>
__global__ void rows_to_points(const S* __restrict__ z, int32_t n, int32_t KD, float* __restrict__ out) {
  const int64_t total = (int64_t)n * KD;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / KD;
    const int q = (int)(i - r * KD);
    float v = 0.f;
    if (q < LH) v = (float)elem<S>::to_acc(z[r * LH + q]);
    out[i] = v;
  }
}

// ---------------------------------------------------------------------------
// Validation: bad row pointer, column out of range, self-loop, weight < 0 or
// not finite.  flags: [0] row_ptr, [1] column, [2] self-loop, [3] weight.
// ---------------------------------------------------------------------------
template <typename W>
__global__ void validate_kernel(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                const W* __restrict__ val, int32_t n, int64_t nnz, int32_t* flags) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += stride) {
    const int64_t a = row_ptr[r], b = row_ptr[r + 1];
    if (a < 0 || b < a || b > nnz || (r == 0 && a != 0) || (r == n - 1 && b != nnz)) {
      atomicOr(&flags[0], 1);
      continue;
    }
    for (int64_t j = a; j < b; ++j)
      if (col[j] == r) atomicOr(&flags[2], 1);
  }
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += stride) {
    const int32_t c = col[j];
    if (c < 0 || c >= n) atomicOr(&flags[1], 1);
    if constexpr (!std::is_void<W>::value) {
      const double w = weight<W, double>::get(val, j);
      if (!(w >= 0.0) || isinf(w)) atomicOr(&flags[3], 1);
    }
  }
}

// ===========================================================================
// Host side
// ===========================================================================
// LDS per block of the tile kernel: 2*NB staged products of LH values, and
// 2*NB FP64 weights in the degree pass that shares the plan.
static size_t tile_lds_bytes(int NB, int LH, int vec_dtype) {
  const size_t row = (size_t)LH * (vec_dtype == FSC_F64 ? 8 : 4);
  return (size_t)2 * NB * std::max<size_t>(row, 8);
}

static int default_tile_nnz(int LH, int vec_dtype) {
  int nb = 2048;
  while (nb > 256 && tile_lds_bytes(nb, LH, vec_dtype) > 32768) nb >>= 1;
  return nb;
}

int max_tile_nnz(int l, int vec_dtype) {
  const int LH = padded_width(l);
  int nb = 1 << 16;
  while (nb > 64 && tile_lds_bytes(nb, LH, vec_dtype) > 60 * 1024) nb >>= 1;
  return nb;
}

size_t embed_workspace_bytes(const Context* ctx, const fsc_csr* g, int l, int vec_dtype, int tile_nnz) {
  const int LH = padded_width(l);
  const int NB = tile_nnz > 0 ? tile_nnz : default_tile_nnz(LH, vec_dtype);
  const int64_t n = g->n;
  const int64_t nb = g->nnz / NB + 1;
  const size_t se = vec_dtype == FSC_F64 ? 8 : vec_dtype == FSC_F32 ? 4 : 2;
  const size_t ae = vec_dtype == FSC_F64 ? 8 : 4;
  const int grid = 4096;
  size_t b = 0;
  b += align_up(n * 8) * 2 + align_up(n * ae) + align_up(n);       // deg, isq, hinv, elig
  b += 2 * align_up(n * LH * se);                                  // z ping-pong
  b += align_up((size_t)grid * 2 * LH * 8);                        // partials
  b += align_up(4 * LH * 8) + align_up(LH * 8) + align_up(LH * 4); // state, scales
  b += align_up(nb * 2 * LH * 8);                                  // lnorm
  b += align_up((2 * nb + 1) * std::max<size_t>(LH * ae, 8));      // lpart (FP64 for degrees)
  b += align_up(nb * 4);                                           // lcount
  b += align_up((nb + 1) * 4) * 4 + align_up((2 * nb + 1) * sizeof(LongChunk)) + align_up(16);  // plan
  b += 16 * 256;                                                   // alignment slack
  return b;
}

int embed_bind_workspace(Context* ctx, Arena* a, EmbedIO* io) {
  const fsc_csr* g = io->g;
  const int LH = io->LH;
  const int NB = io->tile_nnz > 0 ? io->tile_nnz : default_tile_nnz(LH, io->vec_dtype);
  io->tile_nnz = NB;
  const int64_t n = g->n;
  const int64_t nb = g->nnz / NB + 1;
  const size_t se = io->vec_dtype == FSC_F64 ? 8 : io->vec_dtype == FSC_F32 ? 4 : 2;
  const size_t ae = io->vec_dtype == FSC_F64 ? 8 : 4;
  io->deg = a->take<double>(n);
  io->isq = a->take<double>(n);
  io->hinv = a->take<char>(n * ae);
  io->elig = a->take<uint8_t>(n);
  io->z[0] = a->take<char>(n * LH * se);
  io->z[1] = a->take<char>(n * LH * se);
  io->partials = a->take<double>((size_t)4096 * 2 * LH);
  io->state = a->take<double>(4 * LH);
  io->lnorm = a->take<double>(nb * 2 * LH);
  io->lpart = a->take<char>((2 * nb + 1) * std::max<size_t>(LH * ae, 8));
  io->lcount = a->take<int32_t>(nb);
  io->plan.nb = (int32_t)nb;
  io->plan.tile_nnz = NB;
  io->plan.rb = a->take<int32_t>(nb + 1);
  io->plan.nch = a->take<int32_t>(nb + 1);
  io->plan.choff = a->take<int32_t>(nb + 1);
  io->plan.lid = a->take<int32_t>(nb + 1);
  io->plan.max_chunks = (int32_t)(2 * nb + 1);
  io->plan.chunks = a->take<LongChunk>(2 * nb + 1);
  io->plan.meta = a->take<int32_t>(4);
  if (a->used > a->size) return fail(FSC_E_NOMEM, "workspace arena too small");
  return FSC_OK;
}

template <class Op>
static int launch_tiles(Context* ctx, const Op& op, const TileArgs& ta, int grid, hipStream_t s) {
  const size_t lds = (size_t)2 * ta.NB * Op::LH * sizeof(typename Op::A);
  hipLaunchKernelGGL(tile_kernel<Op>, dim3(grid), dim3(kBlock), lds, s, op, ta);
  return check_hip(hipGetLastError(), "tile_kernel launch");
}

static int persistent_grid(Context* ctx, int nb) {
  // enough resident blocks to cover the chip several times over, but never
  // more tiles-worth of blocks than there are short tiles plus long chunks
  int g = ctx->num_cu * 8;
  if (g > 4096) g = 4096;
  const int cap = 2 * nb + 1;
  return g < cap ? g : cap;
}

template <typename S, typename W, int LH>
static int run_steps(Context* ctx, EmbedIO* io, TileArgs ta, hipStream_t s, bool stats) {
  using A = typename elem<S>::acc;
  const fsc_csr* g = io->g;
  A* scale = reinterpret_cast<A*>(io->state + 3 * LH);  // next step's scale, as A
  for (int step = 1; step <= io->t; ++step) {
    const S* zin = reinterpret_cast<const S*>(io->z[(step - 1) & 1]);
    S* zout = reinterpret_cast<S*>(io->z[step & 1]);
    int rc;
    if (stats) {
      StepOp<S, W, LH, true> op;
      op.val = reinterpret_cast<const W*>(g->val);
      op.zin = zin;
      op.zout = zout;
      op.hinv = reinterpret_cast<const A*>(io->hinv);
      op.deg = io->deg;
      op.scale = scale;
      auto* ev = timing_start(ctx, s);
      rc = launch_tiles(ctx, op, ta, io->grid, s);
      timing_stop(ev, s);
      if (rc) return rc;
      hipLaunchKernelGGL(finish_stats<LH>, dim3(1), dim3(kBlock), 0, s, io->partials, io->grid, io->lnorm,
                         io->plan.meta, step, io->t, io->l, io->renorm, io->state, io->sqnorm_trace,
                         io->rayleigh_trace,
                         std::is_same<A, float>::value ? reinterpret_cast<float*>(scale) : nullptr,
                         std::is_same<A, double>::value ? reinterpret_cast<double*>(scale) : nullptr);
      rc = check_hip(hipGetLastError(), "finish_stats launch");
    } else {
      StepOp<S, W, LH, false> op;
      op.val = reinterpret_cast<const W*>(g->val);
      op.zin = zin;
      op.zout = zout;
      op.hinv = reinterpret_cast<const A*>(io->hinv);
      op.deg = io->deg;
      op.scale = nullptr;
      auto* ev = timing_start(ctx, s);
      rc = launch_tiles(ctx, op, ta, io->grid, s);
      timing_stop(ev, s);
    }
    if (rc) return rc;
  }
  io->zt = io->z[io->t & 1];
  return FSC_OK;
}

template <typename S, typename W, int LH>
static int run_embed_typed(Context* ctx, EmbedIO* io, hipStream_t s) {
  using A = typename elem<S>::acc;
  const fsc_csr* g = io->g;
  const int32_t n = (int32_t)g->n;
  const int32_t nb = io->plan.nb;
  const int32_t NB = io->plan.tile_nnz;
  int rc;
  // tile plan
  {
    const int blocks = (nb + 255) / 256;
    hipLaunchKernelGGL(plan_buckets, dim3(blocks), dim3(256), 0, s, g->row_ptr, n, nb, NB, io->plan.rb,
                       io->plan.nch);
    hipLaunchKernelGGL(plan_scan, dim3(1), dim3(1024), 0, s, io->plan.nch, nb, io->plan.choff, io->plan.lid,
                       io->plan.meta);
    hipLaunchKernelGGL(plan_chunks, dim3(blocks), dim3(256), 0, s, g->row_ptr, nb, NB, io->plan.rb,
                       io->plan.nch, io->plan.choff, io->plan.lid, io->plan.chunks);
    hipLaunchKernelGGL(fill_i32, dim3((nb + 255) / 256), dim3(256), 0, s, io->lcount, (int64_t)nb, 0);
    if ((rc = check_hip(hipGetLastError(), "plan kernels"))) return rc;
  }
  io->grid = persistent_grid(ctx, nb);
  TileArgs ta;
  ta.row_ptr = g->row_ptr;
  ta.col = g->col_idx;
  ta.n = n;
  ta.nb = nb;
  ta.NB = NB;
  ta.rb = io->plan.rb;
  ta.chunks = io->plan.chunks;
  ta.meta = io->plan.meta;
  ta.partials = io->partials;
  ta.lcount = io->lcount;
  ta.lnorm = io->lnorm;
  // degrees (FP64), 1/(2d), d^{-1/2}, eligibility
  {
    TileArgs td = ta;
    td.lpart = io->lpart;  // FP64 chunk partials: sized for A = double only when vec is f64
    DegreeOp<W, A> op;
    op.val = reinterpret_cast<const W*>(g->val);
    op.deg = io->deg;
    op.hinv = reinterpret_cast<A*>(io->hinv);
    op.isq = io->isq;
    op.elig = io->elig;
    if ((rc = launch_tiles(ctx, op, td, io->grid, s))) return rc;
  }
  ta.lpart = io->lpart;
  const bool stats = io->renorm || io->sqnorm_trace || io->rayleigh_trace;
  // start block
  {
    const uint64_t seed = io->seed;
    hipLaunchKernelGGL((start_block<S, LH>), dim3(io->grid), dim3(kBlock), 0, s, n, io->l,
                       (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), io->x0, io->isq, io->deg,
                       reinterpret_cast<S*>(io->z[0]), io->partials, stats ? 1 : 0);
    if ((rc = check_hip(hipGetLastError(), "start_block launch"))) return rc;
    if (stats) {
      A* scale = reinterpret_cast<A*>(io->state + 3 * LH);
      hipLaunchKernelGGL(finish_stats<LH>, dim3(1), dim3(kBlock), 0, s, io->partials, io->grid, io->lnorm,
                         io->plan.meta, 0, io->t, io->l, io->renorm, io->state, io->sqnorm_trace,
                         io->rayleigh_trace,
                         std::is_same<A, float>::value ? reinterpret_cast<float*>(scale) : nullptr,
                         std::is_same<A, double>::value ? reinterpret_cast<double*>(scale) : nullptr);
      if ((rc = check_hip(hipGetLastError(), "finish_stats launch"))) return rc;
    }
  }
  return run_steps<S, W, LH>(ctx, io, ta, s, stats);
}

template <typename S, typename W>
static int run_embed_lh(Context* ctx, EmbedIO* io, hipStream_t s) {
  switch (io->LH) {
    case 1: return run_embed_typed<S, W, 1>(ctx, io, s);
    case 2: return run_embed_typed<S, W, 2>(ctx, io, s);
    case 4: return run_embed_typed<S, W, 4>(ctx, io, s);
    case 8: return run_embed_typed<S, W, 8>(ctx, io, s);
  }
  return fail(FSC_E_UNSUPPORTED, "unsupported block width");
}

template <typename S>
static int run_embed_val(Context* ctx, EmbedIO* io, hipStream_t s) {
  const fsc_csr* g = io->g;
  if (!g->val) return run_embed_lh<S, void>(ctx, io, s);
  switch (g->val_dtype) {
    case FSC_F64:
      if (std::is_same<S, double>::value) return run_embed_lh<S, double>(ctx, io, s);
      break;
    case FSC_F32: return run_embed_lh<S, float>(ctx, io, s);
    case FSC_BF16:
      if (!std::is_same<S, double>::value) return run_embed_lh<S, bf16_t>(ctx, io, s);
      break;
  }
  return fail(FSC_E_UNSUPPORTED, "unsupported combination of weight and vector dtypes "
                                 "(f64 vectors take f64/f32 weights, f32/bf16 vectors take f32/bf16 weights)");
}

int embed_run(Context* ctx, EmbedIO* io, hipStream_t s) {
  switch (io->vec_dtype) {
    case FSC_F64: return run_embed_val<double>(ctx, io, s);
    case FSC_F32: return run_embed_val<float>(ctx, io, s);
    case FSC_BF16: return run_embed_val<bf16_t>(ctx, io, s);
  }
  return fail(FSC_E_ARG, "vec_dtype must be FSC_F64, FSC_F32 or FSC_BF16");
}

template <typename S>
static int unpad_typed(const EmbedIO* io, void* out, hipStream_t s) {
  const int32_t n = (int32_t)io->g->n;
  const int64_t total = (int64_t)n * io->l;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
  const S* z = reinterpret_cast<const S*>(io->zt);
  S* o = reinterpret_cast<S*>(out);
  switch (io->LH) {
    case 1: hipLaunchKernelGGL((unpad_rows<S, 1>), dim3(blocks), dim3(256), 0, s, z, n, io->l, o); break;
    case 2: hipLaunchKernelGGL((unpad_rows<S, 2>), dim3(blocks), dim3(256), 0, s, z, n, io->l, o); break;
    case 4: hipLaunchKernelGGL((unpad_rows<S, 4>), dim3(blocks), dim3(256), 0, s, z, n, io->l, o); break;
    case 8: hipLaunchKernelGGL((unpad_rows<S, 8>), dim3(blocks), dim3(256), 0, s, z, n, io->l, o); break;
  }
  return check_hip(hipGetLastError(), "unpad_rows launch");
}

int embed_unpad(Context*, const EmbedIO* io, void* out, hipStream_t s) {
  if (io->g->n == 0) return FSC_OK;
  switch (io->vec_dtype) {
    case FSC_F64: return unpad_typed<double>(io, out, s);
    case FSC_F32: return unpad_typed<float>(io, out, s);
    case FSC_BF16: return unpad_typed<bf16_t>(io, out, s);
  }
  return fail(FSC_E_ARG, "bad vec_dtype");
}

template <typename S>
static int points_typed(const EmbedIO* io, float* pts, hipStream_t s) {
  const int32_t n = (int32_t)io->g->n;
  const int KD = kmeans_width(io->l);
  const int64_t total = (int64_t)n * KD;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
  const S* z = reinterpret_cast<const S*>(io->zt);
  switch (io->LH) {
    case 1: hipLaunchKernelGGL((rows_to_points<S, 1>), dim3(blocks), dim3(256), 0, s, z, n, KD, pts); break;
    case 2: hipLaunchKernelGGL((rows_to_points<S, 2>), dim3(blocks), dim3(256), 0, s, z, n, KD, pts); break;
    case 4: hipLaunchKernelGGL((rows_to_points<S, 4>), dim3(blocks), dim3(256), 0, s, z, n, KD, pts); break;
    case 8: hipLaunchKernelGGL((rows_to_points<S, 8>), dim3(blocks), dim3(256), 0, s, z, n, KD, pts); break;
  }
  return check_hip(hipGetLastError(), "rows_to_points launch");
}

int embed_to_points(Context*, const EmbedIO* io, float* pts, hipStream_t s) {
  switch (io->vec_dtype) {
    case FSC_F64: return points_typed<double>(io, pts, s);
    case FSC_F32: return points_typed<float>(io, pts, s);
    case FSC_BF16: return points_typed<bf16_t>(io, pts, s);
  }
  return fail(FSC_E_ARG, "bad vec_dtype");
}

int validate_csr(Context* ctx, const fsc_csr* g, hipStream_t s) {
  int rc;
  hipLaunchKernelGGL(fill_i32, dim3(1), dim3(64), 0, s, ctx->error_flag, (int64_t)4, 0);
  const int32_t n = (int32_t)g->n;
  const int blocks = (int)std::min<int64_t>((std::max<int64_t>(g->n, g->nnz) + 255) / 256, 8192);
  if (!g->val) {
    hipLaunchKernelGGL(validate_kernel<void>, dim3(blocks), dim3(256), 0, s, g->row_ptr, g->col_idx,
                       (const void*)nullptr, n, g->nnz, ctx->error_flag);
  } else if (g->val_dtype == FSC_F64) {
    hipLaunchKernelGGL(validate_kernel<double>, dim3(blocks), dim3(256), 0, s, g->row_ptr, g->col_idx,
                       (const double*)g->val, n, g->nnz, ctx->error_flag);
  } else if (g->val_dtype == FSC_F32) {
    hipLaunchKernelGGL(validate_kernel<float>, dim3(blocks), dim3(256), 0, s, g->row_ptr, g->col_idx,
                       (const float*)g->val, n, g->nnz, ctx->error_flag);
  } else {
    hipLaunchKernelGGL(validate_kernel<bf16_t>, dim3(blocks), dim3(256), 0, s, g->row_ptr, g->col_idx,
                       (const bf16_t*)g->val, n, g->nnz, ctx->error_flag);
  }
  if ((rc = check_hip(hipGetLastError(), "validate launch"))) return rc;
  if ((rc = check_hip(hipMemcpyAsync(ctx->host_flag, ctx->error_flag, 4 * sizeof(int32_t),
                                     hipMemcpyDeviceToHost, s), "validate copy")))
    return rc;
  if ((rc = check_hip(hipStreamSynchronize(s), "validate sync"))) return rc;
  const int32_t* f = ctx->host_flag;
  if (f[0]) return fail(FSC_E_GRAPH, "row_ptr is not a valid CSR row pointer");
  if (f[1]) return fail(FSC_E_GRAPH, "column index out of range");
  if (f[2]) return fail(FSC_E_GRAPH, "graph has a self-loop");
  if (f[3]) return fail(FSC_E_GRAPH, "weight is negative, NaN or infinite");
  return FSC_OK;
}

}  // namespace fsc
