// The embedding D^{-1/2} Y of FastSpectralCluster (Algorithm 2) on gfx950.
//
// Everything runs in z-space, Z = D^{-1/2} Y: one PowerMethod step
// (Algorithm 1) with the halved signless Laplacian M = (I + D^{-1/2} A
// D^{-1/2}) / 2 (Sec. 2) becomes
//     Z' = Z / 2 + (1 / (2 d)) (.) (A Z),
// so the degree scaling is one multiply per row and Z_t is the embedding
// itself.  The sparse product is the only pass over the graph per step.
//
// Tiles of the sparse product: the nonzeros are cut into buckets of tile_nnz;
// bucket b owns the rows whose first nonzero lies in [b*tile_nnz,
// (b+1)*tile_nnz).  Its rows are no longer than tile_nnz except possibly the
// last one; such a long row is cut into chunks of tile_nnz, each a tile of its
// own whose partial sums are combined, in chunk order, by the chunk that
// finishes last.  A short tile gives each of its rows a group of G lanes
// (G a power of two chosen per bucket from its row count and mean length);
// the lanes of a group stream the row's column indices and weights with
// coalesced non-temporal loads, gather the l-wide rows of Z (which stay in
// cache), accumulate in registers and combine with wave shuffles.  The grid is
// persistent with a static tile order, so per-block statistics -- and so the
// FP64 column norms -- are deterministic.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"
#include "fsc_slab.hpp"
#include "fsc_tiles.hpp"

#include <algorithm>
#include <type_traits>

namespace fsc {


// ---------------------------------------------------------------------------
// Tile plan
// ---------------------------------------------------------------------------
__global__ void plan_buckets(const int64_t* __restrict__ row_ptr, int32_t n, int32_t nb, int32_t NB,
                             TileDesc* __restrict__ desc, int32_t* __restrict__ nch) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t r0 = min<int64_t>(lower_bound_i64(row_ptr, (int64_t)n + 1, (int64_t)b * NB), n);
  int64_t r1 = min<int64_t>(lower_bound_i64(row_ptr, (int64_t)n + 1, (int64_t)(b + 1) * NB), n);
  if (b == nb - 1) r1 = n;
  int32_t c = 0;
  if (r1 > r0) {
    const int64_t len = row_ptr[r1] - row_ptr[r1 - 1];
    if (len > NB) {
      c = (int32_t)((len + NB - 1) / NB);
      r1 -= 1;  // the long last row goes to chunk tiles
    }
  }
  TileDesc d;
  d.r0 = (int32_t)r0;
  d.r1 = (int32_t)r1;
  d.G = lanes_per_row(r1 - r0, row_ptr[r1] - row_ptr[r0]);
  d.pad = 0;
  desc[b] = d;
  nch[b] = c;
}

// Exclusive scans of nch and of (nch > 0), one block.
__global__ __launch_bounds__(1024) void plan_scan(const int32_t* __restrict__ nch, int32_t nb,
                                                  int32_t* __restrict__ choff, int32_t* __restrict__ lid,
                                                  int32_t* __restrict__ meta) {
  __shared__ int32_t lds_a[1024 / FSC_WAVE + 1], lds_b[1024 / FSC_WAVE + 1];
  int32_t carry_a = 0, carry_b = 0;
  for (int32_t base = 0; base < nb; base += 1024) {
    const int32_t i = base + threadIdx.x;
    const int32_t va = i < nb ? nch[i] : 0;
    const int32_t vb = va > 0 ? 1 : 0;
    int32_t ta, tb;
    const int32_t ia = block_scan_inclusive<1024>(va, lds_a, &ta);
    const int32_t ib = block_scan_inclusive<1024>(vb, lds_b, &tb);
    if (i < nb) {
      choff[i] = carry_a + ia - va;
      lid[i] = carry_b + ib - vb;
    }
    carry_a += ta;
    carry_b += tb;
  }
  if (threadIdx.x == 0) {
    choff[nb] = carry_a;
    lid[nb] = carry_b;
    meta[0] = carry_a;
    meta[1] = carry_b;
  }
}

__global__ void plan_chunks(const int64_t* __restrict__ row_ptr, int32_t nb, int32_t NB,
                            const TileDesc* __restrict__ desc, const int32_t* __restrict__ nch,
                            const int32_t* __restrict__ choff, const int32_t* __restrict__ lid,
                            LongChunk* __restrict__ chunks) {
  const int32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb || nch[b] == 0) return;
  const int32_t r = desc[b].r1;  // the long row follows the bucket's short rows
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
// Start block: Z0 = D^{-1/2} X0, X0 Gaussian (Algorithm 2) or given.
// ---------------------------------------------------------------------------
// Entry (i, q) of X0: the caller's, or Philox4x32-10 with counter
// (i, 0, q, 0) and Box-Muller on its two 53-bit uniforms.
__device__ __forceinline__ double start_value(int32_t i, int q, int32_t l, uint32_t k0, uint32_t k1,
                                              const double* __restrict__ x0) {
  if (x0) return x0[(int64_t)i * l + q];
  const u32x4 r = philox4x32_10(u32x4{(uint32_t)i, 0u, (uint32_t)q, 0u}, k0, k1);
  const double u1 = uniform53(r.x, r.y), u2 = uniform53(r.z, r.w);
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

template <typename S, int LH>
__global__ __launch_bounds__(kBlock) void start_block(int32_t n, int32_t l, uint32_t k0, uint32_t k1,
                                                      const double* __restrict__ x0,
                                                      const double* __restrict__ isq,
                                                      const double* __restrict__ deg, S* __restrict__ z,
                                                      StatsArgs sa, int stats) {
  using A = typename elem<S>::acc;
  double st[2 * LH];
#pragma unroll
  for (int q = 0; q < 2 * LH; ++q) st[q] = 0.0;
  for (int32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const double s = isq[i];
    const double d = deg[i];
    A row[LH];
#pragma unroll
    for (int q = 0; q < LH; ++q) {
      const double x = q < l ? start_value(i, q, l, k0, k1, x0) : 0.0;
      row[q] = elem<S>::to_acc(elem<S>::from_acc(static_cast<A>(s * x)));
      st[q] += d * (double)row[q] * (double)row[q];
    }
    rowio<S, LH>::store(z + (int64_t)i * LH, row);
  }
  if (stats) stats_epilogue<LH>(sa, st);
}

// ---------------------------------------------------------------------------
// Output conversions
// ---------------------------------------------------------------------------
// Y = D^{1/2} Z_t, the PowerMethod iterates themselves (n x l, unpadded):
// sqrt(d_v) z_v where d_v > 0; an isolated vertex's row of M is e_v / 2, so
// its row of Y is 2^-t times its row of X0.
template <typename S, int LH>
__global__ void rows_to_y(const S* __restrict__ z, const double* __restrict__ deg, int32_t n, int32_t l, int32_t t,
                          uint32_t k0, uint32_t k1, const double* __restrict__ x0, S* __restrict__ out) {
  using A = typename elem<S>::acc;
  const int64_t total = (int64_t)n * l;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t r = (int32_t)(i / l);
    const int q = (int)(i - (int64_t)r * l);
    const double d = deg[r];
    double y;
    if (d > 0.0) {
      y = sqrt(d) * (double)elem<S>::to_acc(z[(int64_t)r * LH + q]);
    } else {
      y = ldexp(start_value(r, q, l, k0, k1, x0), -t);
    }
    out[i] = elem<S>::from_acc(static_cast<A>(y));
  }
}

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
int fill_zero_i32(int32_t* p, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32, dim3((int)std::min<int64_t>((count + 255) / 256, 1024)), dim3(256), 0, s, p, count, 0);
  return check_hip(hipGetLastError(), "fill launch");
}

int effective_tile_nnz(const Context* ctx, int tile_nnz) { return tile_nnz > 0 ? tile_nnz : ctx->tune.tile_nnz; }

int max_tile_nnz(int, int) { return 1 << 20; }

static int64_t num_buckets(int64_t nnz, int NB) { return nnz / NB + 1; }

size_t embed_workspace_bytes(const Context* ctx, const fsc_csr* g, int l, int vec_dtype, int tile_nnz) {
  const int LH = padded_width(l);
  const int NB = effective_tile_nnz(ctx, tile_nnz);
  const int64_t n = g->n;
  const int64_t nb = num_buckets(g->nnz, NB);
  const size_t se = vec_dtype == FSC_F64 ? 8 : vec_dtype == FSC_F32 ? 4 : 2;
  const size_t ae = vec_dtype == FSC_F64 ? 8 : 4;
  size_t b = 0;
  b += align_up(n * 8) * 2 + align_up(n * ae) + align_up(n);        // deg, isq, hinv, elig
  b += 2 * align_up(n * LH * se);                                   // z ping-pong
  b += align_up((size_t)2 * kMaxGrid * 2 * LH * 8);                 // partials (two steps')
  b += align_up((5 * LH + 8) * 8);                                  // state
  b += align_up(nb * 2 * LH * 8);                                   // lnorm
  b += align_up((2 * nb + 1) * std::max<size_t>(LH * ae, 8));       // lpart (FP64 for degrees)
  b += align_up(nb * 4);                                            // lcount
  b += align_up(nb * sizeof(TileDesc)) + align_up((nb + 1) * 4) * 3;  // plan
  b += align_up((2 * nb + 1) * sizeof(LongChunk)) + align_up(16);
  b += 16 * 256;                                                    // alignment slack
  b += slab_workspace_bytes(ctx, g, LH, vec_dtype);
  return b;
}

int embed_bind_workspace(Context* ctx, Arena* a, EmbedIO* io) {
  const fsc_csr* g = io->g;
  const int LH = io->LH;
  const int NB = effective_tile_nnz(ctx, io->tile_nnz);
  io->tile_nnz = NB;
  const int64_t n = g->n;
  const int64_t nb = num_buckets(g->nnz, NB);
  const size_t se = io->vec_dtype == FSC_F64 ? 8 : io->vec_dtype == FSC_F32 ? 4 : 2;
  const size_t ae = io->vec_dtype == FSC_F64 ? 8 : 4;
  io->deg = a->take<double>(n);
  io->isq = a->take<double>(n);
  io->hinv = a->take<char>(n * ae);
  io->elig = a->take<uint8_t>(n);
  io->z[0] = a->take<char>(n * LH * se);
  io->z[1] = a->take<char>(n * LH * se);
  io->partials = a->take<double>((size_t)2 * kMaxGrid * 2 * LH);
  io->state = a->take<double>(5 * LH + 8);
  io->lnorm = a->take<double>(nb * 2 * LH);
  io->lpart = a->take<char>((2 * nb + 1) * std::max<size_t>(LH * ae, 8));
  io->lcount = a->take<int32_t>(nb);
  io->plan.nb = (int32_t)nb;
  io->plan.tile_nnz = NB;
  io->plan.desc = a->take<TileDesc>(nb);
  io->plan.nch = a->take<int32_t>(nb + 1);
  io->plan.choff = a->take<int32_t>(nb + 1);
  io->plan.lid = a->take<int32_t>(nb + 1);
  io->plan.max_chunks = (int32_t)(2 * nb + 1);
  io->plan.chunks = a->take<LongChunk>(2 * nb + 1);
  io->plan.meta = a->take<int32_t>(4);
  if (a->used > a->size) return fail(FSC_E_NOMEM, "workspace arena too small");
  return slab_bind(ctx, a, io);
}

template <class Op>
static int launch_tiles(const Op& op, const TileArgs& ta, const StatsArgs& sa, int grid, int unroll, hipStream_t s) {
  if (unroll == 4)
    hipLaunchKernelGGL((tile_kernel<4, Op>), dim3(grid), dim3(kBlock), 0, s, op, ta, sa);
  else
    hipLaunchKernelGGL((tile_kernel<8, Op>), dim3(grid), dim3(kBlock), 0, s, op, ta, sa);
  return check_hip(hipGetLastError(), "tile_kernel launch");
}

// Phase-form kernel shape: nonzeros in flight per row, rows per lane.
constexpr int kSlabU = 4;
constexpr int kSlabJ = 1;

template <typename CI, class Op>
static int launch_slab_ci(const Op& op, const TileArgs& ta, const SlabArgs& sb, const StatsArgs& sa, int grid,
                          int rgrid, const PendingFinish& pf, hipStream_t s) {
  if (sb.wave) {
    SlabWaveArgs sw;
    sw.nslab = sb.nslab;
    sw.wlen = sb.wlen;
    sw.gbase = sb.gbase;
    sw.gunit = sb.gunit;
    sw.scol = sb.scol;
    sw.S = sb.S;
    hipLaunchKernelGGL((slab_wave_kernel<8, CI, Op>), dim3(grid), dim3(kBlock), 0, s, op, ta, sw, sa);
  } else if (sb.xcd) {
    hipLaunchKernelGGL((slab_xcd_kernel<8, CI, Op>), dim3(grid), dim3(kBlock), 0, s, op, ta, sb);
    hipLaunchKernelGGL((slab_reduce_kernel<Op>), dim3(rgrid), dim3(kBlock), 0, s, op, ta, sb, sa);
  } else {
    hipLaunchKernelGGL((slab_kernel<kSlabU, kSlabJ, CI, Op>), dim3(grid), dim3(kBlock), 0, s, op, ta, sb, sa, pf);
  }
  return check_hip(hipGetLastError(), "slab_kernel launch");
}

template <class Op>
static int launch_slab(const Op& op, const TileArgs& ta, const SlabArgs& sb, const StatsArgs& sa, int grid,
                       int rgrid, const PendingFinish& pf, hipStream_t s) {
  return sb.c16 ? launch_slab_ci<uint16_t>(op, ta, sb, sa, grid, rgrid, pf, s)
                : launch_slab_ci<int32_t>(op, ta, sb, sa, grid, rgrid, pf, s);
}

// One step's launch: the column-slab kernel when the plan has slabs (only
// its phase form takes a pending finish).
template <class Op>
static int launch_step(const Op& op, const TileArgs& ta, const SlabArgs* sb, const StatsArgs& sa, int grid,
                       int unroll, const PendingFinish& pf, hipStream_t s) {
  if constexpr (!std::is_same<typename Op::A, double>::value) {
    if (sb) return launch_slab(op, ta, *sb, sa, grid, sb->rgrid, pf, s);
  }
  return launch_tiles(op, ta, sa, grid, unroll, s);
}

// Persistent grid: a few resident blocks per CU, a multiple of 8 so the XCD
// round-robin is even, never many more blocks than tiles.
static int persistent_grid(const Context* ctx, int64_t tiles, int blocks_per_cu) {
  int64_t g = (int64_t)ctx->num_cu * blocks_per_cu;
  if (g > kMaxGrid) g = kMaxGrid;
  const int64_t cap = std::max<int64_t>(8, (tiles + 7) / 8 * 8);
  if (g > cap) g = cap;
  g = std::max<int64_t>(8, g / 8 * 8);
  return (int)g;
}

// Whether a step's statistics are finished inside the next step kernel: the
// phase form of the column-slab kernel, with the statistics on and no scale
// to apply (without re-normalisation every scale is 1, so the next step does
// not wait for them).  The partials (and the long rows' statistics) then
// alternate between two buffers by step parity, so that a step writes its
// own while the previous step's are being finished.
static bool fold_finish(const EmbedIO* io, bool stats) {
  return stats && !io->renorm && !io->ortho && io->slab.enabled && !io->slab.wave && !io->slab.xcd &&
         io->vec_dtype != FSC_F64;
}

template <typename S, typename W, int LH>
static int run_steps(Context* ctx, EmbedIO* io, const TileArgs& ta_in, const SlabArgs* sb_in, StatsArgs sa,
                     hipStream_t s, bool stats, PendingFinish pending) {
  const SlabArgs* sb = sb_in;
  using A = typename elem<S>::acc;
  const fsc_csr* g = io->g;
  const W* sval = reinterpret_cast<const W*>(io->slab.sval);
  const A* scale = reinterpret_cast<const A*>(io->state + 3 * LH);
  const bool fold = sb && fold_finish(io, stats);
  TileArgs ta = ta_in;
  int rc;
  for (int step = 1; step <= io->t; ++step) {
    const S* zin = reinterpret_cast<const S*>(io->z[(step - 1) & 1]);
    S* zout = reinterpret_cast<S*>(io->z[step & 1]);
    sa.step = step;
    int grid = io->grid;
    PendingFinish pf;
    pf.grid = 0;
    if (fold) {
      sa.partials = io->partials + (size_t)(step & 1) * kMaxGrid * 2 * LH;
      ta.lnorm = io->slab.lnorm + (size_t)(step & 1) * io->slab.max_long * 2 * LH;
      sa.lnorm = ta.lnorm;
      if (grid <= sb->ntiles) ++grid;  // a block for the finish
      pf = pending;
    }
    auto* ev = timing_start(ctx, s);
    if (stats) {
      StepOp<S, W, LH, true> op;
      op.val = reinterpret_cast<const W*>(g->val);
      op.sval = sval;
      op.zin = zin;
      op.zout = zout;
      op.hinv = reinterpret_cast<const A*>(io->hinv);
      op.deg = io->deg;
      op.scale = fold ? nullptr : scale;  // folded: every scale is 1
      rc = launch_step(op, ta, sb, sa, grid, ctx->tune.unroll, pf, s);
    } else {
      StepOp<S, W, LH, false> op;
      op.val = reinterpret_cast<const W*>(g->val);
      op.sval = sval;
      op.zin = zin;
      op.zout = zout;
      op.hinv = reinterpret_cast<const A*>(io->hinv);
      op.deg = io->deg;
      op.scale = nullptr;
      rc = launch_step(op, ta, sb, sa, grid, ctx->tune.unroll, pf, s);
    }
    timing_stop(ev, s);
    if (rc) return rc;
    if (fold) {
      pending.sa = sa;
      pending.grid = grid;
    } else if (stats) {
      // the partials come from the per-XCD form's reduce kernel, else from the step kernel
      const bool reduce = sb && sb->xcd && !std::is_same<A, double>::value;
      hipLaunchKernelGGL((stats_finish_kernel<LH>), dim3(1), dim3(kFinish), 0, s, sa, reduce ? sb->rgrid : io->grid);
      if ((rc = check_hip(hipGetLastError(), "stats_finish launch"))) return rc;
    }
    if (io->ortho && (rc = ortho_run(io, zout, step == io->t, s))) return rc;
  }
  if (pending.grid > 0) {  // the last step's statistics (or the start block's when t = 0)
    hipLaunchKernelGGL((stats_finish_kernel<LH>), dim3(1), dim3(kFinish), 0, s, pending.sa, pending.grid);
    if ((rc = check_hip(hipGetLastError(), "stats_finish launch"))) return rc;
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
  // Graphs whose steps take the slab form get their degrees from the slab
  // builder (it reads every weight anyway) and need no tile plan unless a
  // later tile kernel asks for one.
  const bool slab_steps = io->slab.enabled && !std::is_same<A, double>::value;
  // tile plan
  if (!slab_steps || io->need_tiles) {
    const int blocks = (nb + 255) / 256;
    hipLaunchKernelGGL(plan_buckets, dim3(blocks), dim3(256), 0, s, g->row_ptr, n, nb, NB, io->plan.desc,
                       io->plan.nch);
    hipLaunchKernelGGL(plan_scan, dim3(1), dim3(1024), 0, s, io->plan.nch, nb, io->plan.choff, io->plan.lid,
                       io->plan.meta);
    hipLaunchKernelGGL(plan_chunks, dim3(blocks), dim3(256), 0, s, g->row_ptr, nb, NB, io->plan.desc,
                       io->plan.nch, io->plan.choff, io->plan.lid, io->plan.chunks);
    hipLaunchKernelGGL(fill_i32, dim3((nb + 255) / 256), dim3(256), 0, s, io->lcount, (int64_t)nb, 0);
    if ((rc = check_hip(hipGetLastError(), "plan kernels"))) return rc;
  }
  io->grid = persistent_grid(ctx, nb, ctx->tune.blocks_per_cu);
  TileArgs ta;
  ta.row_ptr = g->row_ptr;
  ta.col = g->col_idx;
  ta.n = n;
  ta.nb = nb;
  ta.desc = io->plan.desc;
  ta.chunks = io->plan.chunks;
  ta.meta = io->plan.meta;
  ta.lcount = io->lcount;
  ta.lnorm = io->lnorm;
  ta.lpart = io->lpart;
  ta.xcd_order = ctx->tune.xcd_order;
  const bool stats = io->renorm || io->sqnorm_trace || io->rayleigh_trace;
  StatsArgs sa;
  sa.partials = io->partials;
  sa.lnorm = io->lnorm;
  sa.meta = io->plan.meta;
  sa.state = io->state;
  sa.sqnorm = io->sqnorm_trace;
  sa.rayleigh = io->rayleigh_trace;
  sa.step = 0;
  sa.t = io->t;
  sa.l = io->l;
  sa.renorm = io->renorm;
  sa.acc_is_double = std::is_same<A, double>::value ? 1 : 0;
  // degrees (FP64), 1/(2d), d^{-1/2}, eligibility
  if (slab_steps) {
    // column-slab plan: its own tiles and long-row chunks for the steps
    if ((rc = slab_build(ctx, io, s))) return rc;
  } else {
    DegreeOp<W, A> op;
    op.val = reinterpret_cast<const W*>(g->val);
    op.deg = io->deg;
    op.hinv = reinterpret_cast<A*>(io->hinv);
    op.isq = io->isq;
    op.elig = io->elig;
    if ((rc = launch_tiles(op, ta, sa, io->grid, 8, s))) return rc;
  }
  // start block (and the statistics of X0)
  PendingFinish pending;
  pending.grid = 0;
  {
    const uint64_t seed = io->seed;
    const int grid = persistent_grid(ctx, ((int64_t)n + 255) / 256, 8);
    hipLaunchKernelGGL((start_block<S, LH>), dim3(grid), dim3(kBlock), 0, s, n, io->l,
                       (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32), io->x0, io->isq, io->deg,
                       reinterpret_cast<S*>(io->z[0]), sa, stats ? 1 : 0);
    if ((rc = check_hip(hipGetLastError(), "start_block launch"))) return rc;
    if (slab_steps && fold_finish(io, stats)) {
      pending.sa = sa;  // finished inside the first step kernel
      pending.grid = grid;
    } else if (stats) {
      hipLaunchKernelGGL((stats_finish_kernel<LH>), dim3(1), dim3(kFinish), 0, s, sa, grid);
      if ((rc = check_hip(hipGetLastError(), "stats_finish launch"))) return rc;
    }
    if (io->ortho && (rc = ortho_run(io, io->z[0], io->t == 0, s))) return rc;
  }
  if (!slab_steps) return run_steps<S, W, LH>(ctx, io, ta, nullptr, sa, s, stats, pending);
  const SlabPlan& sp = io->slab;
  TileArgs ts = ta;
  ts.nb = 0;
  ts.chunks = sp.chunks;
  ts.meta = sp.meta;
  ts.lcount = sp.lcount;
  ts.lnorm = sp.lnorm;
  ts.lpart = sp.lpart;
  StatsArgs ss = sa;
  ss.lnorm = sp.lnorm;
  ss.meta = sp.meta;
  SlabArgs sb;
  sb.ntiles = sp.ntiles;
  sb.rows = sp.rows;
  sb.nslab = sp.nslab;
  sb.xcd = sp.xcd;
  sb.part = sp.part;
  sb.tunit = sp.tunit;
  sb.rgrid = persistent_grid(ctx, ((int64_t)n + kBlock - 1) / kBlock, 8);
  sb.scol = sp.scol;
  sb.c16 = sp.c16;
  sb.S = sp.S;
  sb.sperm = sp.sperm;
  sb.sbase = sp.sbase;
  sb.smax = sp.smax;
  sb.sreg = sp.sreg;
  sb.wave = sp.wave;
  sb.wlen = sp.wlen;
  sb.gbase = sp.gbase;
  sb.gunit = sp.gunit;
  io->grid = sp.wave  ? persistent_grid(ctx, ((int64_t)n + 4 * FSC_WAVE - 1) / (4 * FSC_WAVE), ctx->tune.slab_wave_bpc)
             : sp.xcd ? persistent_grid(ctx, (int64_t)sp.ntiles * sp.nslab, ctx->tune.slab_xcd_bpc)
                      : persistent_grid(ctx, sp.ntiles, ctx->tune.slab_bpc);
  return run_steps<S, W, LH>(ctx, io, ts, &sb, ss, s, stats, pending);
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
      if constexpr (std::is_same<S, double>::value) return run_embed_lh<S, double>(ctx, io, s);
      break;
    case FSC_F32: return run_embed_lh<S, float>(ctx, io, s);
    case FSC_BF16:
      if constexpr (!std::is_same<S, double>::value) return run_embed_lh<S, bf16_t>(ctx, io, s);
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

template <typename S>
static int y_typed(const EmbedIO* io, void* out, hipStream_t s) {
  const int32_t n = (int32_t)io->g->n;
  const int64_t total = (int64_t)n * io->l;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
  const S* z = reinterpret_cast<const S*>(io->zt);
  S* o = reinterpret_cast<S*>(out);
  const uint32_t k0 = (uint32_t)(io->seed & 0xffffffffu), k1 = (uint32_t)(io->seed >> 32);
  switch (io->LH) {
    case 1: hipLaunchKernelGGL((rows_to_y<S, 1>), dim3(blocks), dim3(256), 0, s, z, io->deg, n, io->l, io->t, k0, k1, io->x0, o); break;
    case 2: hipLaunchKernelGGL((rows_to_y<S, 2>), dim3(blocks), dim3(256), 0, s, z, io->deg, n, io->l, io->t, k0, k1, io->x0, o); break;
    case 4: hipLaunchKernelGGL((rows_to_y<S, 4>), dim3(blocks), dim3(256), 0, s, z, io->deg, n, io->l, io->t, k0, k1, io->x0, o); break;
    case 8: hipLaunchKernelGGL((rows_to_y<S, 8>), dim3(blocks), dim3(256), 0, s, z, io->deg, n, io->l, io->t, k0, k1, io->x0, o); break;
  }
  return check_hip(hipGetLastError(), "rows_to_y launch");
}

int embed_y(Context*, const EmbedIO* io, void* out, hipStream_t s) {
  if (io->g->n == 0) return FSC_OK;
  switch (io->vec_dtype) {
    case FSC_F64: return y_typed<double>(io, out, s);
    case FSC_F32: return y_typed<float>(io, out, s);
    case FSC_BF16: return y_typed<bf16_t>(io, out, s);
  }
  return fail(FSC_E_ARG, "bad vec_dtype");
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

int validate_csr(Context* ctx, const fsc_csr* g, int level, const Arena& scratch, hipStream_t s) {
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
  if (level >= 2) return validate_symmetry(ctx, g, scratch, s);
  return FSC_OK;
}

}  // namespace fsc
