// Column-slab form of the sparse product of one PowerMethod step, for blocks
// Z too large for one XCD's L2.
//
// The gathers of Z rows dominate a step on a large sparse graph: one random
// 8..32-byte row per nonzero.  They run at the L2's request rate only while
// the rows an XCD touches fit its 4 MB L2; spread over a 16 MB block they
// miss to the Infinity Cache and run almost 3x slower.  So the columns are
// cut into nslab slabs of about 2 MB of Z each, and a step makes nslab phases:
// in phase p every block gathers only from slab p, so each XCD's L2 holds one
// slab at a time.
//
// Column indices are stored relative to their slab's first column in 16 bits
// when a slab has at most 65536 columns (half the index stream), else as
// 32-bit columns.
//
// Layout (built once per graph, fsc_slab.hip): the rows are cut into tiles of
// at most kSlabRows consecutive rows (about one tile per resident block).  In each (tile, phase) the rows' nonzeros in
// the phase's slab are stored in jagged-diagonal order: rows sorted by their
// segment length (longest first), and diagonal k holds the k-th nonzero of
// every row longer than k, in sorted order.  A wave takes 64 sorted rows, one
// per lane, so the loads of diagonal k by a wave are contiguous, and no
// padding is stored.  Per-row sums of a phase are added to an LDS accumulator
// in a fixed order (phase by phase, diagonal by diagonal), so results are
// deterministic.  Rows longer than kSlabLong are left out of the tiles and
// summed by the long-row chunks of the plain tile kernel (original CSR).
#pragma once

#include "fsc_tiles.hpp"

namespace fsc {

struct SlabArgs {
  int32_t ntiles, rows, nslab;        // tiles of `rows` consecutive rows (<= kSlabRows)
  int32_t xcd;                        // 1: per-XCD slabs with partial sums (slab_xcd_kernel)
  int32_t rgrid;                      // per-XCD form: grid of slab_reduce_kernel
  void* part;                         // per-XCD form: A[n/64][nslab][64][LH] partial sums
  const uint8_t* tunit;               // [ntiles] 1: the tile's weights are all 1 (skip them)
  const void* scol;       // column indices in slab order: uint16_t slab-local (c16) or int32_t columns
  int32_t c16;            // 1: 16-bit indices relative to the slab's first column p * S
  int32_t S;              // columns per slab
  const uint16_t* sperm;  // tile T, phase p, sorted position i -> local row, at r0*nslab + p*R + i
  const int32_t* sbase;   // [ntiles*nslab][kSlabLong+1]: start of diagonal k within the region
  const int32_t* smax;    // [ntiles*nslab]: longest segment of the (tile, phase)
  const int64_t* sreg;    // [ntiles*nslab]: start of the (tile, phase) region
  int32_t wave;           // 1: wave form (slab_wave_kernel), with the three arrays below
  const uint8_t* wlen;
  const int64_t* gbase;
  const uint8_t* gunit;
};


// Start of diagonal kk of the current (tile, phase): from the lane-resident
// copy of the first 64 starts, else from memory.
__device__ __forceinline__ int32_t diag_start(const int32_t* base, int32_t lane_copy, int32_t kk) {
  return kk < FSC_WAVE ? __builtin_amdgcn_readlane(lane_copy, kk) : base[kk];
}

// Adds the (tile T, slab p) region's per-row sums to acc (LDS, R x LH): one
// lane per sorted row, kU nonzeros in flight per row.  With J = 2 a lane takes
// two rows at once, positions s0 + lane and s0 + kBlock + lane, whose loads
// are all issued together (rows are sorted by length, so the first is never
// shorter); each row's sum is built in the same order either way.
template <int kU, int J, bool UNIT, typename CI, class Op>
__device__ __forceinline__ void slab_region_as(const Op& op, const SlabArgs& sb, int32_t T, int p, int32_t r0,
                                               int32_t R, typename Op::A* acc) {
  constexpr int LH = Op::LH;
  using A = typename Op::A;
  const CI* scol = static_cast<const CI*>(sb.scol);
  const int32_t cbase = sizeof(CI) == 2 ? p * sb.S : 0;
  const int wave = threadIdx.x / FSC_WAVE, lane = threadIdx.x % FSC_WAVE;
  const int64_t tp = (int64_t)T * sb.nslab + p;
  const int32_t maxlen = sb.smax[tp];
  if (maxlen <= 0) return;
  const int64_t reg = sb.sreg[tp];
  const int32_t* base = sb.sbase + tp * (kSlabLong + 1);
  const uint16_t* perm = sb.sperm + (int64_t)r0 * sb.nslab + (int64_t)p * R;
  // diagonal starts 0..63 live in the lanes of every wave
  const int32_t bl = lane <= maxlen ? base[lane] : 0;
  const int32_t active = diag_start(base, bl, 1);  // rows with a nonempty segment
  for (int32_t s0 = wave * FSC_WAVE; s0 < active; s0 += J * kBlock) {
    const int32_t i0 = s0 + lane;
    const int32_t i1 = i0 + kBlock;
    const int rl0 = i0 < active ? (int)perm[i0] : 0;
    const int rl1 = J == 2 && i1 < active ? (int)perm[i1] : 0;
    A a0[LH], a1[LH];
#pragma unroll
    for (int q = 0; q < LH; ++q) a0[q] = a1[q] = A(0);
    int32_t b0 = 0;
    for (int32_t k = 0; k < maxlen; k += kU) {
      int32_t off0[kU], off1[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int32_t kk = k + u;
        off0[u] = off1[u] = -1;
        if (kk < maxlen) {
          const int32_t b1 = diag_start(base, bl, kk + 1);  // diagonal kk holds positions [0, b1 - b0)
          if (i0 < b1 - b0) off0[u] = b0 + i0;
          if (J == 2 && i1 < b1 - b0) off1[u] = b0 + i1;
          b0 = b1;
        }
      }
      if constexpr (J == 2) op.template accumulate_at2<kU, UNIT>(scol, reg, off0, off1, cbase, a0, a1);
      else op.template accumulate_at<kU, UNIT>(scol, reg, off0, cbase, a0);
      // rows are sorted by length: once diagonal k+kU is no longer than s0
      // rows, the whole slice is done
      const int32_t kn = k + kU;
      if (kn < maxlen && s0 >= diag_start(base, bl, kn + 1) - b0) break;
    }
    if (i0 < active) {
#pragma unroll
      for (int q = 0; q < LH; ++q) acc[rl0 * LH + q] += a0[q];
    }
    if (J == 2 && i1 < active) {
#pragma unroll
      for (int q = 0; q < LH; ++q) acc[rl1 * LH + q] += a1[q];
    }
  }
}

// A tile whose weights are all 1 takes the code path without weight loads.
template <int kU, int J, typename CI, class Op>
__device__ __forceinline__ void slab_region(const Op& op, const SlabArgs& sb, int32_t T, int p, int32_t r0,
                                            int32_t R, typename Op::A* acc) {
  if (sb.tunit[T]) slab_region_as<kU, J, true, CI>(op, sb, T, p, r0, R, acc);
  else slab_region_as<kU, J, false, CI>(op, sb, T, p, r0, R, acc);
}

// Phase form: each block takes whole tiles and walks the slabs in order, so
// at any time the blocks gather from about one slab.
template <int kU, int J, typename CI, class Op>
__global__ __launch_bounds__(kBlock, 8) void slab_kernel(Op op_in, TileArgs ta, SlabArgs sb, StatsArgs sa,
                                                      PendingFinish pf) {
  constexpr int LH = Op::LH;
  using A = typename Op::A;
  __shared__ A acc[kSlabRows * LH];
  __shared__ double red[kBlock / FSC_WAVE];
  __shared__ double blk[2 * LH];  // this block's statistics so far (thread 0 adds)
  Op op = op_in;
  op.init();
  // the previous step's statistics, finished by the last block (the host
  // adds a block to the grid when every block has a tile)
  if constexpr (Op::STATS) {
    if (pf.grid > 0 && blockIdx.x == gridDim.x - 1) stats_finish_lean<LH>(pf.sa, pf.grid);
  }
  if (threadIdx.x < 2 * LH) blk[threadIdx.x] = 0.0;
  const int32_t n = ta.n;
  for (int32_t T = blockIdx.x; T < sb.ntiles; T += gridDim.x) {
    const int32_t r0 = T * sb.rows;
    const int32_t R = min(sb.rows, n - r0);
    for (int i = threadIdx.x; i < R * LH; i += kBlock) acc[i] = A(0);
    __syncthreads();
    for (int p = 0; p < sb.nslab; ++p) {
      slab_region<kU, J, CI>(op, sb, T, p, r0, R, acc);
      __syncthreads();  // the next phase may give a row to another wave
    }
    // statistics stay out of registers during the phases: each tile's are
    // reduced over the block and added to blk in tile order
    double st[2 * LH];
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) st[q] = 0.0;
    for (int32_t rl = threadIdx.x; rl < R; rl += kBlock) {
      const int32_t r = r0 + rl;
      if (ta.row_ptr[r + 1] - ta.row_ptr[r] > kSlabLong) continue;  // finished by its chunks
      typename Op::Pre pre;
      op.prefetch(r, pre);
      op.finish(r, &acc[rl * LH], pre, st);
    }
    if constexpr (Op::STATS) {
#pragma unroll
      for (int q = 0; q < 2 * LH; ++q) {
        const double v = block_sum<kBlock>(st[q], red);
        if (threadIdx.x == 0) blk[q] += v;
      }
    }
    __syncthreads();
  }
  const int32_t nch = ta.meta[0];
  for (int32_t c = blockIdx.x; c < nch; c += gridDim.x) long_chunk<kU>(op, ta, c);
  if constexpr (Op::STATS) {
    __syncthreads();
    double st[2 * LH];
#pragma unroll
    for (int q = 0; q < 2 * LH; ++q) st[q] = threadIdx.x == 0 ? blk[q] : 0.0;
    op.epilogue(sa, st);
  }
}

// Per-XCD form: blocks reach the 8 XCDs round-robin by index, and block b
// takes only the regions of slabs b % 8, b % 8 + 8, ...: each XCD gathers
// from its own slab the whole time, whatever the pace of other blocks.  The
// rows' sums of each slab go to part[slab]; slab_reduce_kernel adds them in
// slab order and applies the row operator.  Long rows are summed and finished
// by their chunks here.
template <int kU, typename CI, class Op>
__global__ __launch_bounds__(kBlock) void slab_xcd_kernel(Op op_in, TileArgs ta, SlabArgs sb) {
  constexpr int LH = Op::LH;
  using A = typename Op::A;
  __shared__ A acc[kSlabRows * LH];
  Op op = op_in;
  op.init();
  const int32_t n = ta.n;
  const int x = blockIdx.x & 7, slot = blockIdx.x >> 3, per = gridDim.x >> 3;
  A* part = reinterpret_cast<A*>(sb.part);
  for (int p = x; p < sb.nslab; p += 8)
    for (int32_t T = slot; T < sb.ntiles; T += per) {
      const int32_t r0 = T * sb.rows;
      const int32_t R = min(sb.rows, n - r0);
      for (int i = threadIdx.x; i < R * LH; i += kBlock) acc[i] = A(0);
      __syncthreads();
      slab_region<kU, 1, CI>(op, sb, T, p, r0, R, acc);
      __syncthreads();
      // part: groups of 64 rows, each holding its nslab slabs' 64 x LH sums
      // in a row, so every write here and every read of the reduce is
      // contiguous
      for (int i = threadIdx.x; i < R * LH; i += kBlock) {
        const int32_t r = r0 + i / LH;
        part[(((int64_t)(r >> 6) * sb.nslab + p) * 64 + (r & 63)) * LH + i % LH] = acc[i];
      }
      __syncthreads();
    }
  const int32_t nch = ta.meta[0];
  for (int32_t c = blockIdx.x; c < nch; c += gridDim.x) long_chunk<kU>(op, ta, c);
}

template <class Op>
__global__ __launch_bounds__(kBlock) void slab_reduce_kernel(Op op_in, TileArgs ta, SlabArgs sb, StatsArgs sa) {
  constexpr int LH = Op::LH;
  using A = typename Op::A;
  Op op = op_in;
  op.init();
  const int32_t n = ta.n;
  const A* part = reinterpret_cast<const A*>(sb.part);
  double st[2 * LH];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) st[q] = 0.0;
  for (int32_t r = blockIdx.x * kBlock + threadIdx.x; r < n; r += gridDim.x * kBlock) {
    if (ta.row_ptr[r + 1] - ta.row_ptr[r] > kSlabLong) continue;  // finished by its chunks
    // the per-XCD form has at most 8 slabs: all loads in flight at once
    A v[8][LH];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      if (p < sb.nslab) {
        rowio<A, LH>::load(part + (((int64_t)(r >> 6) * sb.nslab + p) * 64 + (r & 63)) * LH, v[p]);
      } else {
#pragma unroll
        for (int q = 0; q < LH; ++q) v[p][q] = A(0);
      }
    }
    A sum[LH];
#pragma unroll
    for (int q = 0; q < LH; ++q) sum[q] = A(0);
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int q = 0; q < LH; ++q) sum[q] += v[p][q];
    typename Op::Pre pre;
    op.prefetch(r, pre);
    op.finish(r, sum, pre, st);
  }
  if constexpr (Op::STATS) op.epilogue(sa, st);
}

// ---------------------------------------------------------------------------
// Wave form: each wave owns a group of 64 consecutive rows, one per lane, and
// takes them through the slabs in order with the row sums in registers, so
// no wave waits for another.  Waves start together and run at about the same
// pace, so the XCDs still gather from about one slab at a time.  Layout
// (slab_wave_build_kernel): the group's nonzeros slab by slab, within a slab
// row by row, each row's segment in CSR order; per row and slab the segment
// length (a byte).  A row's sum is built in the phase form's order (per slab
// a partial sum over the segment, added to the row's total slab by slab), so
// the two forms give the same bits.
// ---------------------------------------------------------------------------
struct SlabWaveArgs {
  int32_t nslab;
  const uint8_t* wlen;    // [nslab][n] segment length of row r in slab p (0 for long rows)
  const int64_t* gbase;   // [ceil(n/64)] start of group g's nonzeros in scol
  const uint8_t* gunit;   // [ceil(n/64)] 1: the group's weights are all 1
  const void* scol;       // as SlabArgs::scol
  int32_t S;
};

template <int kU, bool UNIT, typename CI, class Op>
__device__ __forceinline__ void wave_group(const Op& op, const TileArgs& ta, const SlabWaveArgs& sw, int32_t g,
                                           double* st) {
  constexpr int LH = Op::LH;
  using A = typename Op::A;
  const CI* scol = static_cast<const CI*>(sw.scol);
  const int lane = threadIdx.x % FSC_WAVE;
  const int32_t n = ta.n;
  const int32_t r = g * FSC_WAVE + lane;
  const bool in = r < n;
  const uint8_t* lp = sw.wlen + (in ? r : 0);
  A acc[LH];
#pragma unroll
  for (int q = 0; q < LH; ++q) acc[q] = A(0);
  int64_t base = sw.gbase[g];
  int len_next = in ? (int)lp[0] : 0;
  for (int p = 0; p < sw.nslab; ++p) {
    const int len = len_next;
    len_next = in && p + 1 < sw.nslab ? (int)lp[(int64_t)(p + 1) * n] : 0;  // in flight during this slab
    int incl = len;
#pragma unroll
    for (int o = 1; o < FSC_WAVE; o <<= 1) {
      const int x = __shfl_up(incl, o, FSC_WAVE);
      if (lane >= o) incl += x;
    }
    const int total = __shfl(incl, FSC_WAVE - 1, FSC_WAVE);
    int mx = len;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) mx = max(mx, __shfl_xor(mx, o, FSC_WAVE));
    const int start = incl - len;
    A a[LH];
#pragma unroll
    for (int q = 0; q < LH; ++q) a[q] = A(0);
    for (int k = 0; k < mx; k += kU) {
      int32_t off[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) off[u] = k + u < len ? start + k + u : -1;
      op.template accumulate_at<kU, UNIT>(scol, base, off, sizeof(CI) == 2 ? p * sw.S : 0, a);
    }
#pragma unroll
    for (int q = 0; q < LH; ++q) acc[q] += a[q];
    base += total;
  }
  if (in && ta.row_ptr[r + 1] - ta.row_ptr[r] <= kSlabLong) {  // long rows: finished by their chunks
    typename Op::Pre pre;
    op.prefetch(r, pre);
    op.finish(r, acc, pre, st);
  }
}

template <int kU, typename CI, class Op>
__global__ __launch_bounds__(kBlock) void slab_wave_kernel(Op op_in, TileArgs ta, SlabWaveArgs sw, StatsArgs sa) {
  constexpr int LH = Op::LH;
  constexpr int WPB = kBlock / FSC_WAVE;
  Op op = op_in;
  op.init();
  double st[2 * LH];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) st[q] = 0.0;
  const int wave = threadIdx.x / FSC_WAVE;
  const int32_t ng = (ta.n + FSC_WAVE - 1) / FSC_WAVE;
  for (int32_t g = blockIdx.x * WPB + wave; g < ng; g += gridDim.x * WPB) {
    if (sw.gunit[g]) wave_group<kU, true, CI>(op, ta, sw, g, st);
    else wave_group<kU, false, CI>(op, ta, sw, g, st);
  }
  const int32_t nch = ta.meta[0];
  for (int32_t c = blockIdx.x; c < nch; c += gridDim.x) long_chunk<kU>(op, ta, c);
  if constexpr (Op::STATS) op.epilogue(sa, st);
}

}  // namespace fsc
