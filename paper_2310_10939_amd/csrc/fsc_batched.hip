// The batched form: FastSpectralCluster (Algorithm 2) on many independent
// graphs of uneven size in one call.
//
// Every stage runs once for the whole batch: the tile plans, the degree pass
// and the start blocks are single grids over all graphs; the power iterations
// run level by level -- level i is one persistent grid (per block width) over
// the tiles of every graph that still has a step i to do; k-means++ rounds and
// Lloyd steps are segmented grids over all graphs.  Levels are separate
// launches because step i of a graph reads what step i-1 wrote on any XCD; the
// kernel boundary is the cross-XCD hand-off.  The whole sequence is captured
// once as a hipGraph and replayed while the batch is unchanged.
//
// The level grids are XCD-affine: every graph is given to one XCD (balanced
// by its work, nonzeros times steps), and the blocks of the grid that the
// dispatcher places on XCD x (block index mod 8) take only the tiles of XCD
// x's graphs, in one sequence (graphs by decreasing t, so the graphs still
// iterating at a level are a prefix).  A graph's n x l block (at most a few
// MB for the batch's sizes) is then gathered by one XCD only and stays in its
// L2, where the single-graph path would need the column-slab layout.
//
// A bucket's long last row (longer than its graph's tile size) is summed by
// the same block right after the bucket's short rows, so each level is a flat
// list of tiles whose count the host knows.  Vectors are FP32; weights FP32 or
// unit.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"
#include "fsc_tiles.hpp"

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

namespace fsc {

struct BGraph {
  const int64_t* row_ptr;
  const int32_t* col;
  const float* val;  // null: unit weights
  int32_t n, l, LH, KD, t, nb, NB, pad;
  TileDesc* desc;
  int32_t* nch;
  double* deg;
  double* isq;
  float* hinv;
  uint8_t* elig;
  float* z[2];
  float* pts;   // k-means points when LH != KD
  float* emb;   // optional n x l output
  uint32_t k0, k1;
};

// Index p with off[p] <= x < off[p+1] (off non-decreasing, off[0] = 0).
__device__ __forceinline__ int seg_find(const int64_t* off, int cnt, int64_t x) {
  int lo = 0, hi = cnt;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// Plan: per-graph buckets (as in the single-graph plan)
// ---------------------------------------------------------------------------
__global__ void bplan_kernel(const BGraph* __restrict__ gs, const int64_t* __restrict__ boff, int ng) {
  const int64_t total = boff[ng];
  for (int64_t B = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; B < total; B += (int64_t)gridDim.x * blockDim.x) {
    const int gi = seg_find(boff, ng, B);
    const BGraph& g = gs[gi];
    const int32_t b = (int32_t)(B - boff[gi]);
    const int64_t NB = g.NB;
    const int64_t r0 = min<int64_t>(lower_bound_i64(g.row_ptr, (int64_t)g.n + 1, (int64_t)b * NB), g.n);
    int64_t r1 = min<int64_t>(lower_bound_i64(g.row_ptr, (int64_t)g.n + 1, (int64_t)(b + 1) * NB), g.n);
    if (b == g.nb - 1) r1 = g.n;
    int32_t c = 0;
    if (r1 > r0 && g.row_ptr[r1] - g.row_ptr[r1 - 1] > NB) {
      c = 1;
      r1 -= 1;
    }
    TileDesc d;
    d.r0 = (int32_t)r0;
    d.r1 = (int32_t)r1;
    d.G = lanes_per_row(r1 - r0, g.row_ptr[r1] - g.row_ptr[r0]);
    d.pad = 0;
    g.desc[b] = d;
    g.nch[b] = c;
  }
}

// A whole long row summed by one block, then finished by thread 0.
template <int kU, class Op>
__device__ __forceinline__ void long_row_block(const Op& op, const TileArgs& ta, int32_t r,
                                               typename Op::A (*wred)[8]) {
  constexpr int LH = Op::LH;
  using A = typename Op::A;
  A acc[LH];
#pragma unroll
  for (int q = 0; q < LH; ++q) acc[q] = A(0);
  const int64_t a = ta.row_ptr[r], e = ta.row_ptr[r + 1];
  for (int64_t j0 = a + threadIdx.x; j0 < e; j0 += (int64_t)kBlock * kU)
    op.template accumulate<kU>(ta.col, j0, kBlock, e, acc);
  group_reduce<LH, A>(acc, FSC_WAVE);
  const int w = threadIdx.x / FSC_WAVE;
  if ((threadIdx.x & (FSC_WAVE - 1)) == 0)
#pragma unroll
    for (int q = 0; q < LH; ++q) wred[w][q] = acc[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    A tot[LH];
#pragma unroll
    for (int q = 0; q < LH; ++q) {
      tot[q] = A(0);
      for (int i = 0; i < kBlock / FSC_WAVE; ++i) tot[q] += wred[i][q];
    }
    typename Op::Pre pre;
    double st[2 * LH];
    op.prefetch(r, pre);
    op.finish(r, tot, pre, st);
  }
  __syncthreads();
}

template <int kU, class Op>
__device__ __forceinline__ void run_tile(const Op& op, const BGraph& g, int32_t b, typename Op::A (*wred)[8]) {
  TileArgs ta;
  ta.row_ptr = g.row_ptr;
  ta.col = g.col;
  double st[2 * Op::LH];
  const TileDesc d = g.desc[b];
  short_tile<kU>(op, ta, d, st);
  if (g.nch[b] > 0) long_row_block<kU>(op, ta, d.r1, wred);
}

// ---------------------------------------------------------------------------
// Degree pass over all graphs' rows: one thread per row sums its weights in
// CSR order in FP64 (a unit-weight graph counts its entries), and writes d,
// 1/(2d), d^{-1/2} and the k-means eligibility d > 0.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void bdegree_kernel(const BGraph* __restrict__ gs,
                                                         const int64_t* __restrict__ noff, int ng) {
  const int64_t total = noff[ng];
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  int p = seg_find(noff, ng, i);
  for (; i < total; i += (int64_t)gridDim.x * kBlock) {
    while (noff[p + 1] <= i) ++p;
    const BGraph& g = gs[p];
    const int32_t r = (int32_t)(i - noff[p]);
    const int64_t a = g.row_ptr[r], e = g.row_ptr[r + 1];
    double d = 0.0;
    if (g.val == nullptr) {
      d = (double)(e - a);
    } else {
      for (int64_t j = a; j < e; ++j) d += (double)g.val[j];
    }
    g.deg[r] = d;
    g.hinv[r] = d > 0.0 ? (float)(0.5 / d) : 0.f;
    g.isq[r] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    g.elig[r] = d > 0.0 ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Start blocks of all graphs: Z0 = D^{-1/2} X0 (Philox + Box-Muller)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void bstart_kernel(const BGraph* __restrict__ gs,
                                                        const int64_t* __restrict__ noff, int ng) {
  const int64_t total = noff[ng];
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  int p = seg_find(noff, ng, i);
  for (; i < total; i += (int64_t)gridDim.x * kBlock) {
    while (noff[p + 1] <= i) ++p;
    const BGraph& g = gs[p];
    const int32_t r = (int32_t)(i - noff[p]);
    const double s = g.isq[r];
    float* z = g.z[0] + (int64_t)r * g.LH;
    for (int q = 0; q < g.LH; ++q) {
      double x = 0.0;
      if (q < g.l) {
        const u32x4 rr = philox4x32_10(u32x4{(uint32_t)r, 0u, (uint32_t)q, 0u}, g.k0, g.k1);
        x = sqrt(-2.0 * log(uniform53(rr.x, rr.y))) * cos(2.0 * M_PI * uniform53(rr.z, rr.w));
      }
      z[q] = (float)(s * x);
    }
  }
}

// ---------------------------------------------------------------------------
// One power-iteration level over all graphs with t > level
// ---------------------------------------------------------------------------
template <int kU, int LH, typename W>
__device__ __forceinline__ void step_tile(const BGraph& g, int32_t b, int level, float (*wred)[8]) {
  StepOp<float, W, LH, false> op;
  op.val = reinterpret_cast<const W*>(g.val);
  op.zin = g.z[level & 1];
  op.zout = g.z[(level + 1) & 1];
  op.hinv = g.hinv;
  op.deg = g.deg;
  op.scale = nullptr;
  op.init();
  run_tile<kU>(op, g, b, wred);
}

// The graphs of one XCD at one level: per XCD x, its sequence starts at
// order[first[x]] with the tile prefix toffs[tfirst[x] ..]; act[x] graphs
// (a prefix) still iterate, with tiles[x] tiles between them.
struct XcdLevel {
  int32_t first[8];
  int32_t tfirst[8];
  int32_t act[8];
  int64_t tiles[8];
};

template <int kU, int LH>
__global__ __launch_bounds__(kBlock) void blevel_kernel(const BGraph* __restrict__ gs,
                                                        const int32_t* __restrict__ order,
                                                        const int64_t* __restrict__ toffs, XcdLevel lv, int level) {
  __shared__ float wred[kBlock / FSC_WAVE][8];
  const int x = blockIdx.x & 7;             // the XCD the dispatcher puts this block on
  const int64_t per = gridDim.x >> 3;       // blocks per XCD (the grid is a multiple of 8)
  const int act = lv.act[x];
  const int64_t total = lv.tiles[x];
  int64_t T = blockIdx.x >> 3;
  if (act == 0 || T >= total) return;
  const int64_t* tf = toffs + lv.tfirst[x];
  const int32_t* od = order + lv.first[x];
  int p = seg_find(tf, act, T);
  for (; T < total; T += per) {
    while (tf[p + 1] <= T) ++p;
    const BGraph& g = gs[od[p]];
    const int32_t b = (int32_t)(T - tf[p]);
    if (g.val == nullptr) step_tile<kU, LH, void>(g, b, level, wred);
    else step_tile<kU, LH, float>(g, b, level, wred);
  }
}

// ---------------------------------------------------------------------------
// Final iterate -> k-means points (when the widths differ) and the optional
// unpadded embedding output
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void bpoints_kernel(const BGraph* __restrict__ gs,
                                                         const int64_t* __restrict__ noff, int ng) {
  const int64_t total = noff[ng];
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= total) return;
  int p = seg_find(noff, ng, i);
  for (; i < total; i += (int64_t)gridDim.x * kBlock) {
    while (noff[p + 1] <= i) ++p;
    const BGraph& g = gs[p];
    const int32_t r = (int32_t)(i - noff[p]);
    const float* z = g.z[g.t & 1] + (int64_t)r * g.LH;
    if (g.pts)
      for (int q = 0; q < g.KD; ++q) g.pts[(int64_t)r * g.KD + q] = q < g.LH ? z[q] : 0.f;
    if (g.emb)
      for (int q = 0; q < g.l; ++q) g.emb[(int64_t)r * g.l + q] = z[q];
  }
}

// ===========================================================================
// Host side
// ===========================================================================
static int grid_for(int64_t work_items, int cap) {
  int64_t g = std::min<int64_t>(work_items, cap);
  return (int)std::max<int64_t>(1, g);
}

static uint64_t mix(uint64_t h, uint64_t v) {
  h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
  return h;
}

// Tile size for a graph of the given mean degree: the autotuned entry of its
// degree class, else the context default.
int tile_for_degree(const Context* ctx, double mean_degree) {
  const int cls = degree_class(mean_degree);
  const int v = ctx->tile_by_class[cls];
  return v > 0 ? v : ctx->tune.tile_nnz;
}

int batched_run(Context* ctx, int G, const fsc_csr* graphs, const int32_t* ks, const int32_t* ls,
                const int32_t* ts, uint64_t seed, const fsc_opts& o, int32_t* labels, float* emb, hipStream_t s) {
  const int iters = o.kmeans_iters > 0 ? o.kmeans_iters : 30;
  // ---- per-graph shapes; the replay key
  struct Host {
    int64_t n, nnz, nb;
    int l, LH, KD, t, k, NB;
  };
  std::vector<Host> h(G);
  uint64_t key = mix(0, (uint64_t)G);
  key = mix(key, seed);
  key = mix(key, (uint64_t)iters);
  key = mix(key, (uint64_t)(uintptr_t)labels);
  key = mix(key, (uint64_t)(uintptr_t)emb);
  key = mix(key, (uint64_t)ctx->tune.unroll);
  key = mix(key, (uint64_t)ctx->tune.blocks_per_cu);
  for (int g = 0; g < G; ++g) {
    const fsc_csr& c = graphs[g];
    Host& x = h[g];
    x.n = c.n;
    x.nnz = c.nnz;
    x.l = ls[g];
    x.LH = padded_width(x.l);
    x.KD = kmeans_width(x.l);
    x.t = ts[g];
    x.k = ks[g];
    x.NB = tile_for_degree(ctx, c.n > 0 ? (double)c.nnz / (double)c.n : 0.0);
    x.nb = c.nnz / x.NB + 1;
    for (uint64_t v : {(uint64_t)(uintptr_t)c.row_ptr, (uint64_t)(uintptr_t)c.col_idx, (uint64_t)(uintptr_t)c.val,
                       (uint64_t)c.n, (uint64_t)c.nnz, (uint64_t)x.l, (uint64_t)x.t, (uint64_t)x.k, (uint64_t)x.NB})
      key = mix(key, v);
  }
  int rc;
  if (G > 0 && ctx->bexec && ctx->bkey == key && !o.no_graph)
    return check_hip(hipGraphLaunch(ctx->bexec, s), "hipGraphLaunch");

  // ---- sizes of the batch arena
  size_t bytes = 0;
  auto add = [&](size_t b) { bytes += align_up(b); };
  add(sizeof(BGraph) * (G + 1));
  add(sizeof(KmJob) * (G + 1));
  add(8 * (G + 1) * 2);              // boff, noff
  add(8 * (G + 33) * 4);             // toffs: per width class and XCD, a list with a leading 0
  add(4 * (G + 1) * 4);              // order per class
  add(4 * (G + 1) * 2);              // pp_off, ll_off
  for (int g = 0; g < G; ++g) {
    const Host& x = h[g];
    add(sizeof(TileDesc) * x.nb);
    add(4 * x.nb);
    add(8 * x.n * 2 + 4 * x.n + x.n);   // deg, isq, hinv, elig
    add(4 * x.n * x.LH * 2);            // z ping-pong
    if (x.LH != x.KD) add(4 * x.n * x.KD);
    int pp, ll, tpw;
    kmeans_shape(x.n, ctx->num_cu, &pp, &ll, &tpw);
    // d2, bsum, cand, cand_row, centres, cpart, chosen, conv: 8 takes, each
    // padded to 256 bytes
    add(4 * x.n + 8 * 6 * pp + 4 * 6 * x.KD + 4 * 6 + 4 * 64 * x.KD + 8 * (size_t)ll * 64 * (x.KD + 1) + 4 * 64 +
        4 * 4 + 9 * 256);
  }
  bytes += 64 * 1024;
  if (bytes > ctx->barena_size) {
    if (ctx->bexec) {
      hipGraphExecDestroy(ctx->bexec);
      ctx->bexec = nullptr;
    }
    if (ctx->barena) {
      if ((rc = check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize"))) return rc;
      hipFree(ctx->barena);
      ctx->barena = nullptr;
      ctx->barena_size = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FSC_E_NOMEM, "cannot allocate " + std::to_string(bytes) + " bytes for the batch workspace");
    }
    ctx->barena = static_cast<char*>(p);
    ctx->barena_size = bytes;
  }
  Arena a;
  a.base = ctx->barena;
  a.size = ctx->barena_size;
  a.used = 0;
  BGraph* d_graphs = a.take<BGraph>(G + 1);
  KmJob* d_jobs = a.take<KmJob>(G + 1);
  int64_t* d_boff = a.take<int64_t>(G + 1);
  int64_t* d_noff = a.take<int64_t>(G + 1);
  int64_t* d_toffs = a.take<int64_t>((size_t)G + 33);
  int32_t* d_order = a.take<int32_t>(G + 1);
  int32_t* d_ppoff = a.take<int32_t>(G + 1);
  int32_t* d_lloff = a.take<int32_t>(G + 1);

  std::vector<BGraph> bg(G);
  std::vector<KmJob> jobs(G);
  std::vector<int64_t> boff(G + 1, 0), noff(G + 1, 0);
  std::vector<int32_t> ppoff(G + 1, 0), lloff(G + 1, 0);
  std::vector<int64_t> eoff(G + 1, 0);
  int tmax = 0, kmax = 0;
  for (int g = 0; g < G; ++g) eoff[g + 1] = eoff[g] + h[g].n * h[g].l;
  for (int g = 0; g < G; ++g) {
    const Host& x = h[g];
    BGraph& b = bg[g];
    std::memset(&b, 0, sizeof(b));
    b.row_ptr = graphs[g].row_ptr;
    b.col = graphs[g].col_idx;
    b.val = reinterpret_cast<const float*>(graphs[g].val);
    b.n = (int32_t)x.n;
    b.l = x.l;
    b.LH = x.LH;
    b.KD = x.KD;
    b.t = x.t;
    b.nb = (int32_t)x.nb;
    b.NB = x.NB;
    b.desc = a.take<TileDesc>(x.nb);
    b.nch = a.take<int32_t>(x.nb);
    b.deg = a.take<double>(x.n);
    b.isq = a.take<double>(x.n);
    b.hinv = a.take<float>(x.n);
    b.elig = a.take<uint8_t>(x.n);
    b.z[0] = a.take<float>(x.n * x.LH);
    b.z[1] = a.take<float>(x.n * x.LH);
    b.pts = x.LH != x.KD ? a.take<float>(x.n * x.KD) : nullptr;
    b.emb = emb ? emb + eoff[g] : nullptr;
    const uint64_t sg = seed + (uint64_t)g;
    b.k0 = (uint32_t)(sg & 0xffffffffu);
    b.k1 = (uint32_t)(sg >> 32);
    KmJob& J = jobs[g];
    J.n = x.n;
    J.pts = b.pts ? b.pts : b.z[x.t & 1];
    J.elig = b.elig;
    J.KD = x.KD;
    J.k = x.k;
    kmeans_shape(x.n, ctx->num_cu, &J.nblk_pp, &J.nblk_ll, &J.tpw);
    J.d2 = a.take<float>(x.n);
    J.bsum = a.take<double>((size_t)J.nblk_pp * 6);
    J.cand = a.take<float>(6 * x.KD);
    J.cand_row = a.take<int32_t>(6);
    J.trials = kpp_trials(x.k);
    J.centres = a.take<float>(64 * x.KD);
    J.cpart = a.take<double>((size_t)J.nblk_ll * 64 * (x.KD + 1));
    J.chosen = a.take<int32_t>(64);
    J.conv = a.take<int32_t>(4);
    J.labels = labels + noff[g];
    J.k0 = b.k0;
    J.k1 = b.k1;
    boff[g + 1] = boff[g] + x.nb;
    noff[g + 1] = noff[g] + x.n;
    ppoff[g + 1] = ppoff[g] + J.nblk_pp;
    lloff[g + 1] = lloff[g] + J.nblk_ll;
    tmax = std::max(tmax, x.t);
    kmax = std::max(kmax, x.k);
  }
  if (a.used > a.size) return fail(FSC_E_NOMEM, "batch workspace layout overflow");
  // Per width class: the graphs go to the 8 XCDs, largest work (nonzeros
  // times steps) first, each to the least loaded; each XCD's list is sorted
  // by decreasing t, so the graphs still iterating at a level are a prefix.
  const int widths[4] = {1, 2, 4, 8};
  std::vector<int32_t> order;
  std::vector<int64_t> toffs;
  int first[4][8], tfirst[4][8], count[4][8];
  std::vector<std::vector<std::vector<int>>> act(4, std::vector<std::vector<int>>(8, std::vector<int>(std::max(tmax, 1), 0)));
  std::vector<std::vector<std::vector<int64_t>>> tiles(
      4, std::vector<std::vector<int64_t>>(8, std::vector<int64_t>(std::max(tmax, 1), 0)));
  for (int c = 0; c < 4; ++c) {
    std::vector<int> og;
    for (int g = 0; g < G; ++g)
      if (h[g].LH == widths[c] && h[g].t > 0) og.push_back(g);
    std::stable_sort(og.begin(), og.end(), [&](int x, int y) {
      return (double)h[x].nnz * h[x].t > (double)h[y].nnz * h[y].t;
    });
    std::vector<std::vector<int>> lists(8);
    double load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int g : og) {
      const int x = (int)(std::min_element(load, load + 8) - load);
      lists[x].push_back(g);
      load[x] += (double)(h[g].nnz + h[g].n) * h[g].t;
    }
    for (int x = 0; x < 8; ++x) {
      std::stable_sort(lists[x].begin(), lists[x].end(), [&](int p, int q) { return h[p].t > h[q].t; });
      first[c][x] = (int)order.size();
      tfirst[c][x] = (int)toffs.size();
      count[c][x] = (int)lists[x].size();
      toffs.push_back(0);
      for (size_t i = 0; i < lists[x].size(); ++i) {
        const int g = lists[x][i];
        order.push_back(g);
        toffs.push_back(toffs.back() + h[g].nb);
        for (int lv = 0; lv < h[g].t; ++lv) {
          act[c][x][lv] = (int)i + 1;
          tiles[c][x][lv] = toffs.back();
        }
      }
    }
  }
  // ---- upload the tables (once per batch; the graph replays reuse them)
  if ((rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
  if (G > 0) {
    struct Up {
      void* dst;
      const void* src;
      size_t n;
    };
    const size_t G1 = (size_t)G + 1;
    const Up ups[] = {{d_graphs, bg.data(), sizeof(BGraph) * G},    {d_jobs, jobs.data(), sizeof(KmJob) * G},
                      {d_boff, boff.data(), 8 * G1},                {d_noff, noff.data(), 8 * G1},
                      {d_toffs, toffs.data(), 8 * toffs.size()},
                      {d_order, order.data(), 4 * order.size()},    {d_ppoff, ppoff.data(), 4 * G1},
                      {d_lloff, lloff.data(), 4 * G1}};
    for (const Up& u : ups)
      if (u.n > 0 && (rc = check_hip(hipMemcpy(u.dst, u.src, u.n, hipMemcpyHostToDevice), "batch table upload")))
        return rc;
  }

  // ---- the launch sequence
  const int cap = ctx->num_cu * ctx->tune.blocks_per_cu;
  const int lgrid = std::max(8, cap / 8 * 8);  // XCD-affine level grids: a multiple of 8
  auto launches = [&](hipStream_t s) -> int {
    hipLaunchKernelGGL(bplan_kernel, dim3(grid_for((boff[G] + 255) / 256, 8192)), dim3(256), 0, s, d_graphs, d_boff,
                       G);
    hipLaunchKernelGGL(bdegree_kernel, dim3(grid_for((noff[G] + kBlock - 1) / kBlock, 8192)), dim3(kBlock), 0, s,
                       d_graphs, d_noff, G);
    hipLaunchKernelGGL(bstart_kernel, dim3(grid_for((noff[G] + kBlock - 1) / kBlock, 8192)), dim3(kBlock), 0, s,
                       d_graphs, d_noff, G);
    for (int i = 0; i < tmax; ++i) {
      for (int c = 0; c < 4; ++c) {
        XcdLevel lv;
        int64_t most = 0;
        for (int x = 0; x < 8; ++x) {
          lv.first[x] = first[c][x];
          lv.tfirst[x] = tfirst[c][x];
          lv.act[x] = act[c][x][i];
          lv.tiles[x] = lv.act[x] > 0 ? tiles[c][x][i] : 0;
          most = std::max(most, lv.tiles[x]);
        }
        if (most == 0) continue;
        const dim3 grid((unsigned)std::min<int64_t>(lgrid, std::max<int64_t>(8, most * 8)));
        switch (widths[c]) {
          case 1: hipLaunchKernelGGL((blevel_kernel<4, 1>), grid, dim3(kBlock), 0, s, d_graphs, d_order, d_toffs, lv, i); break;
          case 2: hipLaunchKernelGGL((blevel_kernel<4, 2>), grid, dim3(kBlock), 0, s, d_graphs, d_order, d_toffs, lv, i); break;
          case 4: hipLaunchKernelGGL((blevel_kernel<4, 4>), grid, dim3(kBlock), 0, s, d_graphs, d_order, d_toffs, lv, i); break;
          default: hipLaunchKernelGGL((blevel_kernel<4, 8>), grid, dim3(kBlock), 0, s, d_graphs, d_order, d_toffs, lv, i); break;
        }
      }
    }
    hipLaunchKernelGGL(bpoints_kernel, dim3(grid_for((noff[G] + kBlock - 1) / kBlock, 8192)), dim3(kBlock), 0, s,
                       d_graphs, d_noff, G);
    int r2 = check_hip(hipGetLastError(), "batched launches");
    if (r2) return r2;
    return kmeans_run_batched(ctx, d_jobs, d_ppoff, ppoff[G], d_lloff, lloff[G], G, kmax, iters, s);
  };
  if (o.no_graph) return launches(s);
  if (ctx->bexec) {
    hipGraphExecDestroy(ctx->bexec);
    ctx->bexec = nullptr;
  }
  // capture the launches on a private stream (the caller's may be the null
  // stream, which cannot be captured); the instantiated graph is launched on
  // the caller's and replayed while the batch stays the same
  if (!ctx->cap_stream &&
      (rc = check_hip(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking), "hipStreamCreate")))
    return rc;
  if ((rc = check_hip(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal),
                      "hipStreamBeginCapture")))
    return rc;
  const int erc = launches(ctx->cap_stream);
  hipGraph_t graph = nullptr;
  rc = check_hip(hipStreamEndCapture(ctx->cap_stream, &graph), "hipStreamEndCapture");
  if (erc) {
    if (graph) hipGraphDestroy(graph);
    return erc;
  }
  if (rc) return rc;
  hipGraphExec_t exec = nullptr;
  rc = check_hip(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
  hipGraphDestroy(graph);
  if (rc) return rc;
  ctx->bexec = exec;
  ctx->bkey = key;
  return check_hip(hipGraphLaunch(exec, s), "hipGraphLaunch");
}

}  // namespace fsc
