// Builds the column-slab layout of a graph for the sparse product (the
// layout is described in fsc_slab.hpp).  Three kernels, all on the caller's
// stream and free of host synchronisation:
//   slab_count_kernel  per tile: nonzeros of its short rows, its long rows and
//                      their chunks;
//   slab_scan_kernel   exclusive scans of those over the tiles;
//   slab_build_kernel  per tile: segment lengths per (row, slab), rows sorted
//                      by length per slab (counting sort in LDS), diagonal
//                      starts, the scatter of the nonzeros into slab order,
//                      and the long-row chunks.
// The wave form replaces the last kernel by slab_wave_build_kernel (no sort:
// each 64-row group's nonzeros slab by slab, row by row).
// The layout is a function of the CSR alone: rows are sorted stably, and a
// row's nonzeros keep their CSR order within its segment.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>
#include <type_traits>

namespace fsc {

static_assert(kSlabLong < 1024, "the length and diagonal scans use one block pass");
static_assert(kSlabLong <= 255, "the wave form stores segment lengths in a byte");
static_assert(kSlabRows == 1024, "one build thread per row of a tile");

// Slab of column c: slabs are S consecutive columns.
__device__ __forceinline__ int slab_of(int32_t c, int32_t S, int last) {
  // S is a power of two in the phase and wave forms: a shift, not a division
  const int p = c < 0 ? 0 : ((S & (S - 1)) == 0 ? c >> (__ffs(S) - 1) : c / S);
  return p > last ? last : p;
}

// The per-vertex quantities of the degree pass (Sec. 2), written by the
// builders for the short rows (which they read anyway) and by
// slab_long_degree_kernel for the long ones: d = sum of the row's weights
// (FP64), 1/(2d), d^{-1/2} (0 for an isolated vertex) and the k-means
// eligibility d > 0.
struct DegreeOut {
  double* deg;
  float* hinv;
  double* isq;
  uint8_t* elig;
};

__device__ __forceinline__ void write_degree(const DegreeOut& o, int32_t r, double d) {
  o.deg[r] = d;
  o.hinv[r] = d > 0.0 ? static_cast<float>(0.5 / d) : 0.f;
  o.isq[r] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  o.elig[r] = d > 0.0 ? 1 : 0;
}

// Degrees of the long rows: one block per row (its first chunk names it).
template <typename W>
__global__ __launch_bounds__(256) void slab_long_degree_kernel(const int64_t* __restrict__ row_ptr,
                                                               const W* __restrict__ val,
                                                               const LongChunk* __restrict__ chunks,
                                                               const int32_t* __restrict__ meta, DegreeOut o) {
  __shared__ double red[256 / FSC_WAVE];
  const int32_t nch = meta[0];
  for (int32_t c = blockIdx.x; c < nch; c += gridDim.x) {
    const LongChunk ch = chunks[c];
    if (ch.index != 0) continue;
    const int64_t a = row_ptr[ch.row], b = row_ptr[ch.row + 1];
    double sum = 0.0;
    for (int64_t j = a + threadIdx.x; j < b; j += 256) sum += weight<W, double>::get(val, j);
    sum = block_sum<256>(sum, red);
    if (threadIdx.x == 0) write_degree(o, ch.row, sum);
  }
}

__global__ __launch_bounds__(256) void slab_count_kernel(const int64_t* __restrict__ row_ptr, int32_t n,
                                                         int32_t rows, int64_t* __restrict__ tshort,
                                                         int32_t* __restrict__ tlong, int32_t* __restrict__ tchunks) {
  __shared__ int64_t l64[256 / FSC_WAVE];
  __shared__ int32_t l32[256 / FSC_WAVE];
  const int32_t T = blockIdx.x;
  const int32_t r0 = T * rows;
  const int32_t R = min(rows, n - r0);
  int64_t sh = 0;
  int32_t nl = 0, nc = 0;
  for (int32_t rl = threadIdx.x; rl < R; rl += 256) {
    const int64_t len = row_ptr[r0 + rl + 1] - row_ptr[r0 + rl];
    if (len > kSlabLong) {
      ++nl;
      nc += (int32_t)((len + kSlabChunk - 1) / kSlabChunk);
    } else {
      sh += len;
    }
  }
  int64_t t64;
  int32_t t32;
  block_scan_inclusive<256, int64_t>(sh, l64, &t64);
  if (threadIdx.x == 0) tshort[T] = t64;
  block_scan_inclusive<256, int32_t>(nl, l32, &t32);
  if (threadIdx.x == 0) tlong[T] = t32;
  block_scan_inclusive<256, int32_t>(nc, l32, &t32);
  if (threadIdx.x == 0) tchunks[T] = t32;
}

__global__ __launch_bounds__(1024) void slab_scan_kernel(const int64_t* __restrict__ tshort,
                                                         const int32_t* __restrict__ tlong,
                                                         const int32_t* __restrict__ tchunks, int32_t ntiles,
                                                         int64_t* __restrict__ toff, int32_t* __restrict__ loff,
                                                         int32_t* __restrict__ coff, int32_t* __restrict__ meta) {
  __shared__ int64_t l64[1024 / FSC_WAVE];
  __shared__ int32_t la[1024 / FSC_WAVE], lb[1024 / FSC_WAVE];
  int64_t c64 = 0;
  int32_t ca = 0, cb = 0;
  for (int32_t base = 0; base < ntiles; base += 1024) {
    const int32_t i = base + threadIdx.x;
    const int64_t v = i < ntiles ? tshort[i] : 0;
    const int32_t va = i < ntiles ? tlong[i] : 0;
    const int32_t vb = i < ntiles ? tchunks[i] : 0;
    int64_t t64;
    int32_t ta, tb;
    const int64_t iv = block_scan_inclusive<1024, int64_t>(v, l64, &t64);
    const int32_t ia = block_scan_inclusive<1024, int32_t>(va, la, &ta);
    const int32_t ib = block_scan_inclusive<1024, int32_t>(vb, lb, &tb);
    if (i < ntiles) {
      toff[i] = c64 + iv - v;
      loff[i] = ca + ia - va;
      coff[i] = cb + ib - vb;
    }
    c64 += t64;
    ca += ta;
    cb += tb;
  }
  if (threadIdx.x == 0) {
    toff[ntiles] = c64;
    loff[ntiles] = ca;
    coff[ntiles] = cb;
    meta[0] = cb;
    meta[1] = ca;
  }
}

// Four consecutive column indices / weights starting at j0 (j0 a multiple of
// 4): one 16-byte (weights: 16- or 8-byte) load when `vec` says the arrays
// are 16-byte aligned and the quad lies inside them, else element by element
// inside [a, b) (0 elsewhere).
__device__ __forceinline__ void quad_cols(const int32_t* col, int64_t j0, int64_t a, int64_t b, bool vec,
                                          int32_t (&c)[4]) {
  if (vec) {
    const int4 v = *reinterpret_cast<const int4*>(col + j0);
    c[0] = v.x;
    c[1] = v.y;
    c[2] = v.z;
    c[3] = v.w;
  } else {
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = j0 + u >= a && j0 + u < b ? col[j0 + u] : 0;
  }
}
template <typename W> struct quad_w;
template <> struct quad_w<void> {
  __device__ static void get(const void*, int64_t, int64_t, int64_t, bool, float (&w)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = 1.0f;
  }
};
template <> struct quad_w<float> {
  __device__ static void get(const float* v, int64_t j0, int64_t a, int64_t b, bool vec, float (&w)[4]) {
    if (vec) {
      const float4 x = *reinterpret_cast<const float4*>(v + j0);
      w[0] = x.x;
      w[1] = x.y;
      w[2] = x.z;
      w[3] = x.w;
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = j0 + u >= a && j0 + u < b ? v[j0 + u] : 0.f;
    }
  }
};
template <> struct quad_w<bf16_t> {
  __device__ static void get(const bf16_t* v, int64_t j0, int64_t a, int64_t b, bool vec, float (&w)[4]) {
    if (vec) {
      const uint2 x = *reinterpret_cast<const uint2*>(v + j0);
      w[0] = bf16_to_f32((uint16_t)(x.x & 0xffffu));
      w[1] = bf16_to_f32((uint16_t)(x.x >> 16));
      w[2] = bf16_to_f32((uint16_t)(x.y & 0xffffu));
      w[3] = bf16_to_f32((uint16_t)(x.y >> 16));
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) w[u] = j0 + u >= a && j0 + u < b ? bf16_to_f32(v[j0 + u].bits) : 0.f;
    }
  }
};

constexpr int kBuild = 1024;  // threads of the build kernel: one per row of a tile
constexpr int kBuildU = 8;    // nonzeros of a row loaded at once
constexpr int kBuildQ = 4;    // quads of a row whose loads are issued together
constexpr int kGroupQ = 8;    // group form: rounds of 8 nonzeros per row whose loads are issued together

// Weight j as a float (1 without weights).
template <typename W> __device__ __forceinline__ float weight_at(const W* v, int64_t j);
template <> __device__ __forceinline__ float weight_at<void>(const void*, int64_t) { return 1.0f; }
template <> __device__ __forceinline__ float weight_at<float>(const float* v, int64_t j) { return v[j]; }
template <> __device__ __forceinline__ float weight_at<bf16_t>(const bf16_t* v, int64_t j) {
  return bf16_to_f32(v[j].bits);
}

// The group form's view of a row: eight lanes of a wave take one row, lane g
// the nonzeros g, g + 8, ... of it, so that each round of a group reads 8
// consecutive entries.  In a round, the lanes that hold nonzeros of one slab
// come from one ballot per bit of the slab index, restricted to the group;
// their rank among those lanes is their order in CSR order.
struct GroupRow {
  int64_t a;  // first nonzero
  int len;    // nonzeros (0 for a long row or a row past the tile)
  bool shortrow;
  int mlen;   // the longest of the wave's 8 rows of this round
};

// Row i * 8 + lane / 8 of the wave's 64, whose bounds [a, b) are held by the
// lane of that index (the lanes' own rows).
__device__ __forceinline__ GroupRow group_row(int64_t a, int64_t b, int i, int32_t rg, int32_t R) {
  const int src = i * 8 + (threadIdx.x % FSC_WAVE) / 8;
  GroupRow gr;
  gr.a = __shfl(a, src, FSC_WAVE);
  const int64_t e = __shfl(b, src, FSC_WAVE);
  gr.shortrow = rg < R && e - gr.a <= kSlabLong;
  gr.len = gr.shortrow ? (int)(e - gr.a) : 0;
  int m = gr.len;
#pragma unroll
  for (int o = 8; o < FSC_WAVE; o <<= 1) m = max(m, __shfl_xor(m, o, FSC_WAVE));
  gr.mlen = m;
  return gr;
}

// Lanes of this lane's group whose nonzero (ok) lies in the same slab p.
__device__ __forceinline__ uint64_t group_match(bool ok, int p, int sbits, uint64_t gmask) {
  uint64_t m = __ballot(ok) & gmask;
  for (int bit = 0; bit < sbits; ++bit) {
    const bool set = (p >> bit) & 1;
    const uint64_t on = __ballot(set);
    m &= set ? on : ~on;
  }
  return m;
}

// NT threads; tiles of at most NT rows.  Row form (GROUP false): one thread
// per row.  Group form (GROUP true, NT = 512): eight lanes per row, so that
// the reads of the indices and weights are coalesced; the layout is the
// same.  With NT = 512 the block's 53 KB of LDS let three blocks share a CU.
template <typename W, typename CI, int NT, bool GROUP>
__global__ __launch_bounds__(NT) void slab_build_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const W* __restrict__ val, int32_t n,
    int32_t rows, int32_t S, int32_t nslab, const int64_t* __restrict__ toff, const int32_t* __restrict__ loff,
    const int32_t* __restrict__ coff, CI* __restrict__ scol, W* __restrict__ sval, uint16_t* __restrict__ sperm,
    int32_t* __restrict__ sbase, int32_t* __restrict__ smax, int64_t* __restrict__ sreg,
    LongChunk* __restrict__ chunks, uint8_t* __restrict__ tunit, DegreeOut dout, int64_t nnz, int aligned) {
  // Per-slab arrays in LDS have strides of 2 more than their length, so that
  // one row's (or one length's) entries of different slabs fall in different
  // banks.
  constexpr int RS = NT + 2;
  constexpr int LS = kSlabLong + 2;
  __shared__ uint16_t cnt[kSlabMax * RS];   // segment length, later the scatter cursor
  __shared__ uint16_t spos[kSlabMax * RS];  // sorted position of each row per slab
  // per wave: rows of each length, then its cursor (aligned: the group form
  // passes floats through it first)
  __shared__ __align__(16) uint16_t hist[NT / FSC_WAVE * (kSlabLong + 1)];
  __shared__ int32_t baseL[kSlabMax * LS];
  __shared__ int32_t totL[kSlabMax];
  __shared__ int64_t regL[kSlabMax + 1];
  __shared__ int32_t scan32[NT / FSC_WAVE];
  __shared__ int tile_unit;
  const int32_t T = blockIdx.x;
  const int32_t r0 = T * rows;
  const int32_t R = min(rows, n - r0);
  const int last = nslab - 1;
  const int rl = threadIdx.x;  // this thread's row (rows <= NT)
  int64_t a = 0, b = 0;
  if (rl < R) {
    a = row_ptr[r0 + rl];
    b = row_ptr[r0 + rl + 1];
  }
  const bool shortrow = rl < R && b - a <= kSlabLong;
  for (int i = threadIdx.x; i < nslab * RS; i += NT) cnt[i] = 0;
  __syncthreads();
  // A short row's nonzeros in CSR order, kBuildQ aligned quads at a time
  // (one 16-byte load per quad where the arrays allow it): its segment
  // length in every slab, its degree (its weights are read here anyway), and
  // whether every weight of the tile's short rows is exactly 1.
  int unit = 1;
  const int wave = threadIdx.x / FSC_WAVE, lane = threadIdx.x % FSC_WAVE;
  const int g = lane & 7;
  const uint64_t gmask = (uint64_t)0xff << (lane & ~7);
  const uint64_t lower = ((uint64_t)1 << lane) - 1;
  int sbits = 0;
  while ((1 << sbits) <= last) ++sbits;
  if constexpr (GROUP) {
    // group form: while every weight of a row so far is exactly 1 its degree
    // is their count (the same bits as adding them one by one); from its
    // first other weight on, the group's first lane adds the round's weights
    // in CSR order, passed through LDS (the histograms' space, free until
    // the sort)
    float* wb = reinterpret_cast<float*>(hist) + wave * FSC_WAVE;
    for (int i = 0; i < FSC_WAVE / 8; ++i) {
      const int32_t rg = wave * FSC_WAVE + i * 8 + lane / 8;
      const GroupRow gr = group_row(a, b, i, rg, R);
      double dsum = 0.0;
      bool exact = true;  // every weight of the row so far is 1: dsum counts them
      for (int u0 = 0; u0 < gr.mlen; u0 += 8 * kGroupQ) {
        int32_t c[kGroupQ];
        float w[kGroupQ];
#pragma unroll
        for (int q = 0; q < kGroupQ; ++q) {
          const int e = u0 + 8 * q + g;
          c[q] = e < gr.len ? col[gr.a + e] : 0;
          w[q] = e < gr.len ? weight_at<W>(val, gr.a + e) : 1.0f;
        }
#pragma unroll
        for (int q = 0; q < kGroupQ; ++q) {
          const int e = u0 + 8 * q + g;
          const bool ok = e < gr.len;
          const int p = slab_of(c[q], S, last);
          const uint64_t m = group_match(ok, p, sbits, gmask);
          const bool other = ok && w[q] != 1.0f;
          if (ok) {
            if (other) unit = 0;
            if ((m & lower) == 0) cnt[p * RS + rg] = (uint16_t)(cnt[p * RS + rg] + __popcll(m));
          }
          if constexpr (!std::is_void<W>::value) {
            const int k1 = gr.len - (u0 + 8 * q);  // the row's nonzeros in this round (if below 8)
            exact = exact && (__ballot(other) & gmask) == 0;
            if (exact) {
              if (g == 0 && k1 > 0) dsum += (double)min(k1, 8);
            } else {
              wb[lane] = w[q];
              __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
              if (g == 0) {
                const float4 x0 = *reinterpret_cast<const float4*>(wb + lane);
                const float4 x1 = *reinterpret_cast<const float4*>(wb + lane + 4);
                const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
                for (int k = 0; k < 8; ++k)
                  if (k < k1) dsum += (double)x[k];
              }
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
      }
      if (g == 0 && gr.shortrow) write_degree(dout, r0 + rg, std::is_void<W>::value ? (double)gr.len : dsum);
    }
  } else if (shortrow) {
    double dsum = 0.0;
    for (int64_t g0 = a & ~(int64_t)3; g0 < b; g0 += 4 * kBuildQ) {
      int32_t c[kBuildQ][4];
      float w[kBuildQ][4];
#pragma unroll
      for (int q = 0; q < kBuildQ; ++q) {
        const int64_t j0 = g0 + 4 * q;
        const bool vec = aligned && j0 + 4 <= nnz;
        quad_cols(col, j0, a, b, vec, c[q]);
        quad_w<W>::get(val, j0, a, b, vec, w[q]);
      }
#pragma unroll
      for (int q = 0; q < kBuildQ; ++q) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t j = g0 + 4 * q + u;
          if (j < a || j >= b) continue;
          if (w[q][u] != 1.0f) unit = 0;
          dsum += (double)w[q][u];
          cnt[slab_of(c[q][u], S, last) * RS + rl] += 1;
        }
      }
    }
    write_degree(dout, r0 + rl, dsum);
  }
  {
    int32_t nonunit;
    block_scan_inclusive<NT, int32_t>(unit ? 0 : 1, scan32, &nonunit);
    if (threadIdx.x == 0) {
      tile_unit = nonunit == 0;
      tunit[T] = nonunit == 0 ? 1 : 0;  // such a tile skips the weight stream, so its weights are not copied
    }
  }
  __syncthreads();
  // Rows by decreasing segment length, in row order within a length (a
  // stable counting sort), one wave per slab: the wave counts its slab's
  // rows of every length, turns the counts into the start of each length in
  // the sorted order (the number of rows longer than L, which is also the
  // height of diagonal L) and the diagonal starts, and places the rows 64 at
  // a time.  In a group of 64 rows, the lanes that share a lane's length
  // come from one ballot per bit of the lengths (a lane keeps the lanes that
  // agree with it on every bit); the first lane of each length then speaks
  // for them all, so neither the count nor the placement loops over the
  // lengths or needs an atomic.  Only the wave touches its slab's arrays and
  // its own histogram, and a wave's LDS accesses take effect in program
  // order, so no block barrier is needed until all slabs are done.
  {
    constexpr int LPL = (kSlabLong + 1 + FSC_WAVE - 1) / FSC_WAVE;  // lengths per lane
    uint16_t* h = hist + wave * (kSlabLong + 1);
    for (int p = wave; p < nslab; p += NT / FSC_WAVE) {
      int32_t* bl = baseL + p * LS;
      const uint16_t* cp = cnt + p * RS;
      for (int L = lane; L <= kSlabLong; L += FSC_WAVE) h[L] = 0;
      int mx = 0, sum = 0;
      for (int r = lane; r < R; r += FSC_WAVE) {
        const int L = cp[r];
        mx = max(mx, L);
        sum += L;
      }
#pragma unroll
      for (int o = 32; o >= 1; o >>= 1) {
        mx = max(mx, __shfl_xor(mx, o, FSC_WAVE));
        sum += __shfl_xor(sum, o, FSC_WAVE);
      }
      const int32_t maxlen = mx;
      int nbits = 0;
      while ((1 << nbits) <= maxlen) ++nbits;
      auto same_length = [nbits](int L, bool ok) {
        uint64_t m = __ballot(ok);
        for (int bit = 0; bit < nbits; ++bit) {
          const bool set = (L >> bit) & 1;
          const uint64_t on = __ballot(set);
          m &= set ? on : ~on;
        }
        return m;
      };
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      for (int r0w = 0; r0w < R; r0w += FSC_WAVE) {
        const int r = r0w + lane;
        const bool ok = r < R;
        const int L = ok ? (int)cp[r] : 0;
        const uint64_t m = same_length(L, ok);
        if (ok && (m & lower) == 0) h[L] = (uint16_t)(h[L] + __popcll(m));
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
      // start[L] = rows longer than L: a suffix sum over the lengths, lane l
      // holding lengths [l * LPL, (l + 1) * LPL)
      int32_t hv[LPL], tl = 0;
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        const int L = lane * LPL + i;
        hv[i] = L <= kSlabLong ? h[L] : 0;
        tl += hv[i];
      }
      int32_t incl = tl;
#pragma unroll
      for (int o = 1; o < FSC_WAVE; o <<= 1) {
        const int32_t x = __shfl_up(incl, o, FSC_WAVE);
        if (lane >= o) incl += x;
      }
      const int32_t all = __shfl(incl, FSC_WAVE - 1, FSC_WAVE);
      int32_t after = all - incl;  // rows in the lanes above: longer
      int32_t start[LPL];
#pragma unroll
      for (int i = LPL - 1; i >= 0; --i) {
        start[i] = after;
        after += hv[i];
      }
      // diagonal starts: bl[0] = 0, bl[k + 1] = sum over k' <= k of the
      // height of diagonal k' (start[k'] for k' < maxlen, else 0)
      int32_t dl = 0, dv[LPL];
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        const int k = lane * LPL + i;
        dv[i] = k < maxlen ? start[i] : 0;
        dl += dv[i];
      }
      int32_t dincl = dl;
#pragma unroll
      for (int o = 1; o < FSC_WAVE; o <<= 1) {
        const int32_t x = __shfl_up(dincl, o, FSC_WAVE);
        if (lane >= o) dincl += x;
      }
      int32_t run = dincl - dl;
      const int64_t tp = (int64_t)T * nslab + p;
      int32_t* gb = sbase + tp * (kSlabLong + 1);
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        const int k = lane * LPL + i;
        run += dv[i];
        if (k < kSlabLong) bl[k + 1] = run;
        if (k + 1 <= maxlen) gb[k + 1] = run;
      }
      if (lane == 0) {
        bl[0] = 0;
        gb[0] = 0;
        smax[tp] = maxlen;
        totL[p] = sum;
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      // the cursor of each length starts at its start
#pragma unroll
      for (int i = 0; i < LPL; ++i) {
        const int L = lane * LPL + i;
        if (L <= kSlabLong) h[L] = (uint16_t)start[i];
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      // place rows 64 at a time, ascending: lanes with one length take the
      // next positions of that length in lane order, and the first of them
      // advances that length's cursor
      for (int r0w = 0; r0w < R; r0w += FSC_WAVE) {
        const int r = r0w + lane;
        const bool ok = r < R;
        const int L = ok ? (int)cp[r] : 0;
        const uint64_t m = same_length(L, ok);
        const int32_t base = ok ? h[L] : 0;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        if (ok) {
          const int i = base + __popcll(m & lower);
          sperm[(int64_t)r0 * nslab + (int64_t)p * R + i] = (uint16_t)r;
          spos[p * RS + r] = (uint16_t)i;
          if ((m & lower) == 0) h[L] = (uint16_t)(base + __popcll(m));
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      }
    }
  }
  __syncthreads();
  // regions of the slabs, one after another
  if (threadIdx.x == 0) {
    int64_t region = toff[T];
    for (int p = 0; p < nslab; ++p) {
      regL[p] = region;
      sreg[(int64_t)T * nslab + p] = region;
      region += totL[p];
    }
    regL[nslab] = region;  // end of the tile's last region
  }
  __syncthreads();
  // Scatter the short rows' nonzeros into slab order (CSR order within a
  // row's segment), each straight to its place: a tile's regions span a few
  // tens of KB, so the partial lines meet in L2 before they go to memory.
  // Weights are copied only for a tile that loads them.
  const bool copy_w = !std::is_void<W>::value && !tile_unit;
  for (int i = threadIdx.x; i < nslab * RS; i += NT) cnt[i] = 0;
  __syncthreads();
  if constexpr (GROUP) {
    using WS = typename std::conditional<std::is_void<W>::value, char, W>::type;
    for (int i = 0; i < FSC_WAVE / 8; ++i) {
      const int32_t rg = wave * FSC_WAVE + i * 8 + lane / 8;
      const GroupRow gr = group_row(a, b, i, rg, R);
      for (int u0 = 0; u0 < gr.mlen; u0 += 8 * kGroupQ) {
        int32_t c[kGroupQ];
        WS wv[kGroupQ];
#pragma unroll
        for (int q = 0; q < kGroupQ; ++q) {
          const int e = u0 + 8 * q + g;
          c[q] = e < gr.len ? col[gr.a + e] : 0;
          if constexpr (!std::is_void<W>::value) {
            if (copy_w && e < gr.len) wv[q] = val[gr.a + e];
          }
        }
#pragma unroll
        for (int q = 0; q < kGroupQ; ++q) {
          const int e = u0 + 8 * q + g;
          const bool ok = e < gr.len;
          const int p = slab_of(c[q], S, last);
          const uint64_t m = group_match(ok, p, sbits, gmask);
          const int base = ok ? (int)cnt[p * RS + rg] : 0;
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          if (ok) {
            const int kk = base + __popcll(m & lower);
            const int64_t off = regL[p] + baseL[p * LS + kk] + spos[p * RS + rg];
            scol[off] = (CI)(sizeof(CI) == 2 ? c[q] - p * S : c[q]);  // slab-local in 16 bits
            if constexpr (!std::is_void<W>::value) {
              if (copy_w) sval[off] = wv[q];
            }
            if ((m & lower) == 0) cnt[p * RS + rg] = (uint16_t)(base + __popcll(m));
          }
          __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        }
      }
    }
  } else if (shortrow) {
    for (int64_t q0 = a & ~(int64_t)3; q0 < b; q0 += 4 * kBuildQ) {
      int32_t cq[kBuildQ][4];
#pragma unroll
      for (int q = 0; q < kBuildQ; ++q) {
        const int64_t j0 = q0 + 4 * q;
        quad_cols(col, j0, a, b, aligned && j0 + 4 <= nnz, cq[q]);
      }
#pragma unroll
      for (int e = 0; e < 4 * kBuildQ; ++e) {
        const int64_t j = q0 + e;
        if (j < a || j >= b) continue;
        const int32_t c = cq[e / 4][e % 4];
        const int p = slab_of(c, S, last);
        const int kk = cnt[p * RS + rl]++;
        const int64_t off = regL[p] + baseL[p * LS + kk] + spos[p * RS + rl];
        scol[off] = (CI)(sizeof(CI) == 2 ? c - p * S : c);  // slab-local in 16 bits
        if constexpr (!std::is_void<W>::value) {
          if (copy_w) sval[off] = val[j];
        }
      }
    }
  }
  // long rows: chunks of kSlabChunk nonzeros of the original CSR
  {
    const int32_t isl = rl < R && !shortrow ? 1 : 0;
    const int32_t nc = isl ? (int32_t)((b - a + kSlabChunk - 1) / kSlabChunk) : 0;
    int32_t tl, tc;
    const int32_t il = block_scan_inclusive<NT, int32_t>(isl, scan32, &tl);
    const int32_t ic = block_scan_inclusive<NT, int32_t>(nc, scan32, &tc);
    if (isl) {
      const int32_t lid = loff[T] + il - 1;
      const int32_t first = coff[T] + ic - nc;
      for (int32_t c = 0; c < nc; ++c) {
        LongChunk ch;
        ch.start = a + (int64_t)c * kSlabChunk;
        ch.end = min<int64_t>(ch.start + kSlabChunk, b);
        ch.row = r0 + rl;
        ch.lid = lid;
        ch.index = c;
        ch.count = nc;
        ch.first = first;
        ch.pad = 0;
        chunks[first + c] = ch;
      }
    }
  }
}

// Wave form: per tile, one thread per row.  Each 64-row group (one wave)
// lays out its nonzeros slab by slab; within a slab, row by row in row order,
// each row's segment in CSR order.  Stored per row and slab: the segment
// length (a byte); per group: the start of its nonzeros and a unit-weight
// flag.  The positions within a group come from wave scans, so no sort is
// needed.
template <typename W, typename CI>
__global__ __launch_bounds__(kBuild) void slab_wave_build_kernel(
    const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, const W* __restrict__ val, int32_t n,
    int32_t rows, int32_t S, int32_t nslab, const int64_t* __restrict__ toff, const int32_t* __restrict__ loff,
    const int32_t* __restrict__ coff, CI* __restrict__ scol, W* __restrict__ sval, uint8_t* __restrict__ wlen,
    int64_t* __restrict__ gbase, uint8_t* __restrict__ gunit, LongChunk* __restrict__ chunks, DegreeOut dout) {
  __shared__ uint16_t cnt[kSlabMax * kSlabRows];   // segment length, later the scatter cursor
  __shared__ uint16_t spos[kSlabMax * kSlabRows];  // start of each (row, slab) segment within its group
  __shared__ int32_t scan32[kBuild / FSC_WAVE];
  __shared__ int64_t scan64[kBuild / FSC_WAVE];
  const int32_t T = blockIdx.x;
  const int32_t r0 = T * rows;  // rows is a multiple of 64: groups do not straddle tiles
  const int32_t R = min(rows, n - r0);
  const int last = nslab - 1;
  const int rl = threadIdx.x;
  const int lane = rl % FSC_WAVE;
  int64_t a = 0, b = 0;
  if (rl < R) {
    a = row_ptr[r0 + rl];
    b = row_ptr[r0 + rl + 1];
  }
  const bool shortrow = rl < R && b - a <= kSlabLong;
  for (int i = threadIdx.x; i < nslab * R; i += kBuild) cnt[i] = 0;
  __syncthreads();
  if (shortrow) {
    double dsum = 0.0;
    for (int64_t j0 = a; j0 < b; j0 += kBuildU) {
      int32_t c[kBuildU];
#pragma unroll
      for (int u = 0; u < kBuildU; ++u) c[u] = j0 + u < b ? col[j0 + u] : 0;
#pragma unroll
      for (int u = 0; u < kBuildU; ++u) {
        if (j0 + u >= b) continue;
        dsum += weight<W, double>::get(val, j0 + u);
        cnt[slab_of(c[u], S, last) * R + rl] += 1;
      }
    }
    write_degree(dout, r0 + rl, dsum);
  }
  // start of this row's group: the short-row nonzeros before the group
  int64_t gb;
  {
    int64_t tot;
    const int64_t len = shortrow ? b - a : 0;
    const int64_t excl = block_scan_inclusive<kBuild, int64_t>(len, scan64, &tot) - len;
    gb = toff[T] + __shfl(excl, 0, FSC_WAVE);
    if (lane == 0 && rl < R) gbase[(r0 + rl) / FSC_WAVE] = gb;
  }
  __syncthreads();  // the counts above are complete
  // per slab, the group's rows in row order: segment starts by a wave scan
  int32_t phoff = 0;
  for (int p = 0; p < nslab; ++p) {
    const int len = rl < R ? (int)cnt[p * R + rl] : 0;
    int incl = len;
#pragma unroll
    for (int o = 1; o < FSC_WAVE; o <<= 1) {
      const int x = __shfl_up(incl, o, FSC_WAVE);
      if (lane >= o) incl += x;
    }
    if (rl < R) {
      spos[p * R + rl] = (uint16_t)(phoff + incl - len);
      wlen[(int64_t)p * n + r0 + rl] = (uint8_t)len;
    }
    phoff += __shfl(incl, FSC_WAVE - 1, FSC_WAVE);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nslab * R; i += kBuild) cnt[i] = 0;
  __syncthreads();
  int unit = 1;  // every weight of this thread's row is exactly 1
  if (shortrow) {
    for (int64_t j0 = a; j0 < b; j0 += kBuildU) {
      int32_t c[kBuildU];
#pragma unroll
      for (int u = 0; u < kBuildU; ++u) c[u] = j0 + u < b ? col[j0 + u] : 0;
#pragma unroll
      for (int u = 0; u < kBuildU; ++u) {
        if (j0 + u >= b) continue;
        const int p = slab_of(c[u], S, last);
        const int kk = cnt[p * R + rl]++;
        const int64_t dst = gb + spos[p * R + rl] + kk;
        scol[dst] = (CI)(sizeof(CI) == 2 ? c[u] - p * S : c[u]);
        if constexpr (!std::is_void<W>::value) {
          const W w = val[j0 + u];
          sval[dst] = w;
          if (weight<W, float>::get(&w, 0) != 1.0f) unit = 0;
        }
      }
    }
  }
  {
    const bool all_unit = __all(unit);
    if (lane == 0 && rl < R) gunit[(r0 + rl) / FSC_WAVE] = all_unit ? 1 : 0;
  }
  // long rows: chunks of kSlabChunk nonzeros of the original CSR
  {
    const int32_t isl = rl < R && !shortrow ? 1 : 0;
    const int32_t nc = isl ? (int32_t)((b - a + kSlabChunk - 1) / kSlabChunk) : 0;
    int32_t tl, tc;
    const int32_t il = block_scan_inclusive<kBuild, int32_t>(isl, scan32, &tl);
    const int32_t ic = block_scan_inclusive<kBuild, int32_t>(nc, scan32, &tc);
    if (isl) {
      const int32_t lid = loff[T] + il - 1;
      const int32_t first = coff[T] + ic - nc;
      for (int32_t c = 0; c < nc; ++c) {
        LongChunk ch;
        ch.start = a + (int64_t)c * kSlabChunk;
        ch.end = min<int64_t>(ch.start + kSlabChunk, b);
        ch.row = r0 + rl;
        ch.lid = lid;
        ch.index = c;
        ch.count = nc;
        ch.first = first;
        ch.pad = 0;
        chunks[first + c] = ch;
      }
    }
  }
}

__global__ void slab_fill_i32(int32_t* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// ===========================================================================
// Host side
// ===========================================================================
// Which slab form a block of n rows x LH columns takes (slab_kb of the
// context's tuning, slab_mode 0 automatic, 1 phases, 2 per-XCD, 4 waves; the
// wave form has the phase form's slabs):
//   - none when the block fits one slab (FP64 blocks never take one);
//   - phases (automatic): slabs of a power of two rows of at most slab_kb
//     KiB, no more than kSlabMax of them (larger slabs if needed);
//   - per-XCD (on request): 8 slabs of ceil(n/8) rows, one per XCD.  Its
//     gathers are faster (90% L2 hits against 80% on the 1M-vertex SBM),
//     but the reduce pass reads the partial sums back at a high latency and
//     loses the gain (370 us per step against 335 us).
bool slab_shape(const Context* ctx, int64_t n, int LH, int vec_dtype, int32_t* S_out, int32_t* nslab, int* xcd) {
  if (ctx->tune.slab_kb <= 0 || vec_dtype == FSC_F64 || n <= 0) return false;
  const int64_t row = (int64_t)LH * (vec_dtype == FSC_F32 ? 4 : 2);
  int64_t S = 1;
  while (S * 2 * row <= (int64_t)ctx->tune.slab_kb * 1024) S *= 2;
  if (n <= S) return false;  // the block is one slab: the plain tiles do
  const int64_t sx = (n + 7) / 8;
  if (ctx->tune.slab_mode == 2) {  // kernels assume at most 8 slabs in this form
    *S_out = (int32_t)sx;
    *nslab = (int32_t)((n + sx - 1) / sx);
    *xcd = 1;
    return true;
  }
  while ((n + S - 1) / S > kSlabMax) S *= 2;
  *S_out = (int32_t)S;
  *nslab = (int32_t)((n + S - 1) / S);
  *xcd = 0;
  return true;
}

static size_t weight_bytes(const fsc_csr* g) {
  if (!g->val) return 0;
  return g->val_dtype == FSC_F64 ? 8 : g->val_dtype == FSC_F32 ? 4 : 2;
}

// Rows per tile.  Phase form: about one tile per resident block, a multiple
// of 64 in [256, kSlabRows], so blocks move through the slabs together.
// Per-XCD form: kSlabRows (each (tile, slab) region is a work item).  Wave
// form: kSlabRows (tiles only group the build).
int32_t slab_rows(const Context* ctx, int64_t n, int xcd) {
  if (xcd || ctx->tune.slab_mode == 4) return kSlabRows;
  const int64_t blocks = (int64_t)ctx->num_cu * ctx->tune.slab_bpc;
  int64_t r = (n + blocks - 1) / std::max<int64_t>(blocks, 1);
  r = (r + 63) / 64 * 64;
  return (int32_t)std::min<int64_t>(kSlabRows, std::max<int64_t>(256, r));
}

size_t slab_workspace_bytes(const Context* ctx, const fsc_csr* g, int LH, int vec_dtype) {
  int32_t S, nslab;
  int xcd;
  if (!slab_shape(ctx, g->n, LH, vec_dtype, &S, &nslab, &xcd)) return 0;
  const int64_t n = g->n, nnz = g->nnz;
  const int32_t rows = slab_rows(ctx, n, xcd);
  const int64_t nt = (n + rows - 1) / rows;
  const int64_t ml = nnz / (kSlabLong + 1) + 1;
  const int64_t mc = nnz / kSlabChunk + ml + 1;
  size_t b = 0;
  b += align_up(nnz * 4) + align_up(nnz * weight_bytes(g));
  if (ctx->tune.slab_mode == 4) {
    b += align_up(n * nslab) + align_up((n + 63) / 64 * 8) + align_up((n + 63) / 64);
  } else {
    b += align_up(n * nslab * 2);
    b += align_up(nt * nslab * (kSlabLong + 1) * 4) + align_up(nt * nslab * 4) + align_up(nt * nslab * 8);
  }
  b += align_up(nt * 8) + align_up((nt + 1) * 8) + 4 * align_up((nt + 1) * 4);
  b += align_up(mc * sizeof(LongChunk)) + align_up(16);
  b += align_up(2 * ml * 2 * LH * 8) + align_up(mc * LH * 4) + align_up(ml * 4);  // lnorm: two steps'
  if (xcd) b += align_up((size_t)nslab * ((n + 63) / 64 * 64) * LH * 4);  // partial sums (float)
  b += align_up(nt);                                     // unit-weight flags
  b += 24 * 256;  // alignment slack
  return b;
}

int slab_bind(Context* ctx, Arena* a, EmbedIO* io) {
  SlabPlan& sp = io->slab;
  sp = SlabPlan();
  const fsc_csr* g = io->g;
  if (!slab_shape(ctx, g->n, io->LH, io->vec_dtype, &sp.S, &sp.nslab, &sp.xcd)) return FSC_OK;
  const int64_t n = g->n, nnz = g->nnz;
  sp.rows = slab_rows(ctx, n, sp.xcd);
  const int64_t nt = (n + sp.rows - 1) / sp.rows;
  sp.enabled = 1;
  sp.ntiles = (int32_t)nt;
  sp.max_long = nnz / (kSlabLong + 1) + 1;
  sp.max_chunks = nnz / kSlabChunk + sp.max_long + 1;
  sp.c16 = sp.S <= 65536 ? 1 : 0;
  sp.scol = sp.c16 ? (void*)a->take<uint16_t>(nnz) : (void*)a->take<int32_t>(nnz);
  sp.sval = g->val ? (void*)a->take<char>(nnz * weight_bytes(g)) : nullptr;
  sp.wave = !sp.xcd && ctx->tune.slab_mode == 4;
  if (sp.wave) {
    sp.wlen = a->take<uint8_t>(n * sp.nslab);
    sp.gbase = a->take<int64_t>((n + 63) / 64);
    sp.gunit = a->take<uint8_t>((n + 63) / 64);
  } else {
    sp.sperm = a->take<uint16_t>(n * sp.nslab);
    sp.sbase = a->take<int32_t>(nt * sp.nslab * (kSlabLong + 1));
    sp.smax = a->take<int32_t>(nt * sp.nslab);
    sp.sreg = a->take<int64_t>(nt * sp.nslab);
  }
  sp.tshort = a->take<int64_t>(nt);
  sp.toff = a->take<int64_t>(nt + 1);
  sp.tlong = a->take<int32_t>(nt + 1);
  sp.tchunks = a->take<int32_t>(nt + 1);
  sp.loff = a->take<int32_t>(nt + 1);
  sp.coff = a->take<int32_t>(nt + 1);
  sp.chunks = a->take<LongChunk>(sp.max_chunks);
  sp.meta = a->take<int32_t>(4);
  sp.lnorm = a->take<double>(2 * sp.max_long * 2 * io->LH);  // two steps' (the finish may lag a step)
  sp.lpart = a->take<float>(sp.max_chunks * io->LH);
  sp.lcount = a->take<int32_t>(sp.max_long);
  sp.tunit = a->take<uint8_t>(nt);
  sp.part = sp.xcd ? a->take<float>((size_t)sp.nslab * ((n + 63) / 64 * 64) * io->LH) : nullptr;
  if (a->used > a->size) return fail(FSC_E_NOMEM, "workspace arena too small for the slab plan");
  return FSC_OK;
}

template <typename W, typename CI>
static void launch_build_ci(const fsc_csr* g, SlabPlan& sp, const DegreeOut& dout, hipStream_t s) {
  CI* scol = static_cast<CI*>(sp.scol);
  if (sp.wave) {
    hipLaunchKernelGGL((slab_wave_build_kernel<W, CI>), dim3(sp.ntiles), dim3(kBuild), 0, s, g->row_ptr,
                       g->col_idx, reinterpret_cast<const W*>(g->val), (int32_t)g->n, sp.rows, sp.S, sp.nslab,
                       sp.toff, sp.loff, sp.coff, scol, reinterpret_cast<W*>(sp.sval), sp.wlen, sp.gbase, sp.gunit,
                       sp.chunks, dout);
  } else {
    // quads of indices and weights load as one access when both arrays are
    // 16-byte aligned
    const int aligned = reinterpret_cast<uintptr_t>(g->col_idx) % 16 == 0 &&
                        reinterpret_cast<uintptr_t>(g->val) % 16 == 0;
    if (sp.rows <= 512)
      hipLaunchKernelGGL((slab_build_kernel<W, CI, 512, true>), dim3(sp.ntiles), dim3(512), 0, s, g->row_ptr, g->col_idx,
                         reinterpret_cast<const W*>(g->val), (int32_t)g->n, sp.rows, sp.S, sp.nslab, sp.toff,
                         sp.loff, sp.coff, scol, reinterpret_cast<W*>(sp.sval), sp.sperm, sp.sbase, sp.smax,
                         sp.sreg, sp.chunks, sp.tunit, dout, (int64_t)g->nnz, aligned);
    else
      hipLaunchKernelGGL((slab_build_kernel<W, CI, kBuild, false>), dim3(sp.ntiles), dim3(kBuild), 0, s, g->row_ptr,
                         g->col_idx, reinterpret_cast<const W*>(g->val), (int32_t)g->n, sp.rows, sp.S, sp.nslab,
                         sp.toff, sp.loff, sp.coff, scol, reinterpret_cast<W*>(sp.sval), sp.sperm, sp.sbase,
                         sp.smax, sp.sreg, sp.chunks, sp.tunit, dout, (int64_t)g->nnz, aligned);
  }
}

template <typename W>
static void launch_build(const fsc_csr* g, SlabPlan& sp, const DegreeOut& dout, hipStream_t s) {
  if (sp.c16) launch_build_ci<W, uint16_t>(g, sp, dout, s);
  else launch_build_ci<W, int32_t>(g, sp, dout, s);
  hipLaunchKernelGGL((slab_long_degree_kernel<W>), dim3(256), dim3(256), 0, s, g->row_ptr,
                     reinterpret_cast<const W*>(g->val), sp.chunks, sp.meta, dout);
}

int slab_build(Context*, EmbedIO* io, hipStream_t s) {
  SlabPlan& sp = io->slab;
  const fsc_csr* g = io->g;
  DegreeOut dout;
  dout.deg = io->deg;
  dout.hinv = reinterpret_cast<float*>(io->hinv);
  dout.isq = io->isq;
  dout.elig = io->elig;
  const int32_t n = (int32_t)g->n;
  hipLaunchKernelGGL(slab_count_kernel, dim3(sp.ntiles), dim3(256), 0, s, g->row_ptr, n, sp.rows, sp.tshort,
                     sp.tlong, sp.tchunks);
  hipLaunchKernelGGL(slab_scan_kernel, dim3(1), dim3(1024), 0, s, sp.tshort, sp.tlong, sp.tchunks, sp.ntiles,
                     sp.toff, sp.loff, sp.coff, sp.meta);
  if (!g->val) {
    launch_build<void>(g, sp, dout, s);
  } else if (g->val_dtype == FSC_F32) {
    launch_build<float>(g, sp, dout, s);
  } else if (g->val_dtype == FSC_BF16) {
    launch_build<bf16_t>(g, sp, dout, s);
  } else {
    return fail(FSC_E_UNSUPPORTED, "the slab form takes f32 or bf16 weights");
  }
  hipLaunchKernelGGL(slab_fill_i32, dim3((int)std::min<int64_t>((sp.max_long + 255) / 256, 1024)), dim3(256), 0,
                     s, sp.lcount, sp.max_long);
  return check_hip(hipGetLastError(), "slab plan kernels");
}

}  // namespace fsc
