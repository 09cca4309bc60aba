// The C ABI of libfsc (include/fsc.h): argument checks, the context and its
// device workspace, and the order in which the kernels of a call are queued.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "fsc_internal.hpp"

namespace fsc {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return FSC_OK;
  return fail(FSC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int reserve_arena(Context* ctx, size_t bytes, Arena* out) {
  if (bytes > ctx->arena_size) {
    if (ctx->arena) {
      // the old arena may still be read by queued work: wait for it
      hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return check_hip(e, "hipDeviceSynchronize");
      hipFree(ctx->arena);
      ctx->arena = nullptr;
      ctx->arena_size = 0;
    }
    size_t want = std::max(bytes, ctx->arena_size + ctx->arena_size / 4);
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
      (void)hipGetLastError();
      return fail(FSC_E_NOMEM, "cannot allocate " + std::to_string(want) + " bytes of device workspace");
    }
    ctx->arena = static_cast<char*>(p);
    ctx->arena_size = want;
  }
  out->base = ctx->arena;
  out->size = ctx->arena_size;
  out->used = 0;
  return FSC_OK;
}

std::pair<hipEvent_t, hipEvent_t>* timing_start(Context* ctx, hipStream_t s) {
  if (!ctx->timing) return nullptr;
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (!ctx->ev_free.empty()) {
    ev = ctx->ev_free.back();
    ctx->ev_free.pop_back();
  } else {
    if (hipEventCreate(&ev.first) != hipSuccess || hipEventCreate(&ev.second) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
  }
  ctx->ev_used.push_back(ev);
  hipEventRecord(ev.first, s);
  return &ctx->ev_used.back();
}

void timing_stop(std::pair<hipEvent_t, hipEvent_t>* ev, hipStream_t s) {
  if (ev) hipEventRecord(ev->second, s);
}

static int check_csr(const fsc_csr* g) {
  if (!g) return fail(FSC_E_ARG, "graph is NULL");
  if (g->n < 1) return fail(FSC_E_ARG, "graph must have n >= 1 vertices");
  if (g->n > INT32_MAX - 1) return fail(FSC_E_ARG, "n must fit a 32-bit column index");
  if (g->nnz < 0) return fail(FSC_E_ARG, "nnz must be >= 0");
  if (!g->row_ptr) return fail(FSC_E_ARG, "row_ptr is NULL");
  if (g->nnz > 0 && !g->col_idx) return fail(FSC_E_ARG, "col_idx is NULL");
  if (g->val && (g->val_dtype < FSC_F64 || g->val_dtype > FSC_BF16))
    return fail(FSC_E_ARG, "val_dtype must be FSC_F64, FSC_F32 or FSC_BF16");
  return FSC_OK;
}

static fsc_opts default_opts() {
  fsc_opts o;
  std::memset(&o, 0, sizeof(o));
  o.vec_dtype = FSC_F32;
  return o;
}

// Embedding setup shared by fsc_embed and fsc_cluster.  `extra` bytes of the
// arena are left for the caller after the embedding workspace.
static int prepare_embed(Context* ctx, const fsc_csr* g, int l, int t, uint64_t seed, const fsc_opts& o,
                         size_t extra, EmbedIO* io, Arena* arena, const Arena* given = nullptr) {
  int rc;
  if ((rc = check_csr(g))) return rc;
  if (l < 1 || l > 8) return fail(FSC_E_ARG, "l must be in [1, 8]");
  if (t < 0) return fail(FSC_E_ARG, "t must be >= 0");
  if (o.vec_dtype < FSC_F64 || o.vec_dtype > FSC_BF16) return fail(FSC_E_ARG, "bad vec_dtype");
  if (o.tile_nnz < 0 || (o.tile_nnz > 0 && o.tile_nnz < 64)) return fail(FSC_E_ARG, "tile_nnz must be 0 or >= 64");
  std::memset(io, 0, sizeof(*io));
  io->g = g;
  io->l = l;
  io->t = t;
  io->LH = padded_width(l);
  io->seed = seed;
  io->vec_dtype = o.vec_dtype;
  io->renorm = o.renorm;
  io->tile_nnz = o.tile_nnz;
  io->x0 = o.x0;
  io->sqnorm_trace = o.sqnorm_trace;
  io->rayleigh_trace = o.rayleigh_trace;
  if (o.validate < 0 || o.validate > 2) return fail(FSC_E_ARG, "validate must be 0, 1 or 2");
  const size_t bytes = std::max(embed_workspace_bytes(ctx, g, l, o.vec_dtype, o.tile_nnz) + extra,
                                o.validate >= 2 ? symmetry_workspace_bytes(g) : size_t(0));
  if (given) {
    if (given->size < bytes) return fail(FSC_E_NOMEM, "given workspace too small");
    *arena = *given;
    arena->used = 0;
  } else if ((rc = reserve_arena(ctx, bytes, arena))) {
    return rc;
  }
  return embed_bind_workspace(ctx, arena, io);
}

// Workspace of the learned form on top of the embedding's: the 8 further
// Chebyshev basis blocks, a spare block Y (M^8 X0 for the fallback check),
// the filtered block S, statistics, features, coefficients and the small MLP
// scratch.
struct FilterWS {
  float* basis[9];
  float* Y;
  float* S;
  double* ray;       // [16][LH]
  double* part;      // [2 * num_cu][55]
  int32_t* counter;  // [4]
  double* gram;      // [91]: the basis Gram matrix, or the k-means cost
  float* feat;       // [9]
  float* coef;       // [8]
  int32_t* used;     // [1]
  char* mlp;         // mlp workspace for one row
};

static size_t filter_extra_bytes(const Context* ctx, const fsc_csr* g, int l) {
  const int LH = padded_width(l);
  const size_t blk = align_up((size_t)g->n * LH * 4);
  return blk * 10 + align_up(16 * 8 * 8) + align_up((size_t)2 * ctx->num_cu * 55 * 8) + 256 * 6 +
         align_up(91 * 8) + mlp_workspace_bytes(1) + 4096;
}

static void filter_bind(Context* ctx, Arena* a, EmbedIO* io, FilterWS* w) {
  const size_t cnt = (size_t)io->g->n * io->LH;
  w->basis[0] = reinterpret_cast<float*>(io->z[0]);
  for (int j = 1; j < 9; ++j) w->basis[j] = a->take<float>(cnt);
  w->Y = a->take<float>(cnt);
  w->S = a->take<float>(cnt);
  w->ray = a->take<double>(16 * 8);
  w->part = a->take<double>((size_t)2 * ctx->num_cu * 55);
  w->counter = a->take<int32_t>(4);
  w->gram = a->take<double>(91);
  w->feat = a->take<float>(9);
  w->coef = a->take<float>(8);
  w->used = a->take<int32_t>(4);
  w->mlp = a->take<char>(mlp_workspace_bytes(1));
}

static int zero_counter(int32_t* p, hipStream_t s) { return fill_zero_i32(p, 4, s); }

// Largest normalised k-means cost (within-cluster over total variance of the
// embedding rows) accepted from the filtered embedding before falling back.
constexpr double kFilterMaxCost = 0.1;

size_t cluster_workspace_bytes(const Context* ctx, const fsc_csr* g, int l, const fsc_opts& o) {
  const int KD = kmeans_width(l);
  const int LH = padded_width(l);
  const bool direct = o.vec_dtype == FSC_F32 && LH == KD;
  const size_t extra = kmeans_workspace_bytes(g->n, KD) + (direct ? 0 : align_up(g->n * KD * 4)) + 1024;
  return std::max(embed_workspace_bytes(ctx, g, l, o.vec_dtype, o.tile_nnz) + extra,
                  o.validate >= 2 ? symmetry_workspace_bytes(g) : size_t(0));
}

int cluster_run(Context* c, const fsc_csr* g, int k, int l, int t, uint64_t seed, const fsc_opts& o,
                int32_t* labels, void* emb, float* centres, hipStream_t s, const Arena* ws) {
  int rc;
  const int iters = o.kmeans_iters > 0 ? o.kmeans_iters : 30;
  const int KD = kmeans_width(l);
  const int LH = padded_width(l);
  const bool direct = o.vec_dtype == FSC_F32 && LH == KD;
  const size_t extra = kmeans_workspace_bytes(g->n, KD) + (direct ? 0 : align_up(g->n * KD * 4)) + 1024;
  EmbedIO io;
  Arena arena;
  if ((rc = prepare_embed(c, g, l, t, seed, o, extra, &io, &arena, ws))) return rc;
  KmeansIO km;
  std::memset(&km, 0, sizeof(km));
  km.n = g->n;
  km.l = l;
  km.KD = KD;
  km.k = k;
  km.iters = iters;
  km.seed = seed;
  km.labels = labels;
  km.centres_out = centres;
  float* pts = direct ? nullptr : arena.take<float>(g->n * KD);
  if ((rc = kmeans_bind_workspace(&arena, &km))) return rc;
  if (o.validate && (rc = validate_csr(c, g, o.validate, arena, s))) return rc;
  if ((rc = embed_run(c, &io, s))) return rc;
  if (emb && (rc = embed_unpad(c, &io, emb, s))) return rc;
  if (direct) {
    km.pts = reinterpret_cast<const float*>(io.zt);
  } else {
    if ((rc = embed_to_points(c, &io, pts, s))) return rc;
    km.pts = pts;
  }
  km.elig = io.elig;
  return kmeans_run(c, &km, s);
}

// Orthogonal iteration on m columns for t steps (fsc_pmk.hip): the plain
// path's start block and power steps with the block orthonormalised after
// each, then the same k-means (k clusters) on the rows of D^{-1/2} U.  PM
// with k vectors has m = k; the eigenvector baselines run it long enough for
// U to reach the m leading eigenvectors, and the last step's singular values
// (sigma_out) then estimate their eigenvalues.
static int ortho_cluster_run(Context* c, const fsc_csr* g, int k, int m, int t, uint64_t seed, const fsc_opts& o,
                             int32_t* labels, float* emb, double* sigma_out, hipStream_t s) {
  int rc;
  if (o.vec_dtype != FSC_F32 && o.vec_dtype != FSC_F64)
    return fail(FSC_E_UNSUPPORTED, "orthogonal iteration takes FP32 or FP64 vectors");
  const int iters = o.kmeans_iters > 0 ? o.kmeans_iters : 30;
  const int KD = kmeans_width(m);
  const int LH = padded_width(m);
  const size_t extra =
      kmeans_workspace_bytes(g->n, KD) + align_up(g->n * KD * 4) + ortho_workspace_bytes(g->n, LH) + 2048;
  fsc_opts oc = o;
  oc.renorm = 0;
  oc.sqnorm_trace = nullptr;
  oc.rayleigh_trace = nullptr;
  EmbedIO io;
  Arena arena;
  if ((rc = prepare_embed(c, g, m, t, seed, oc, extra, &io, &arena))) return rc;
  KmeansIO km;
  std::memset(&km, 0, sizeof(km));
  km.n = g->n;
  km.l = m;
  km.KD = KD;
  km.k = k;
  km.iters = iters;
  km.seed = seed;
  km.labels = labels;
  float* pts = arena.take<float>(g->n * KD);
  OrthoArgs oa;
  ortho_bind(&arena, g->n, LH, m, &oa);
  oa.sigma_out = sigma_out;
  io.ortho = &oa;
  if ((rc = kmeans_bind_workspace(&arena, &km))) return rc;
  if (arena.used > arena.size) return fail(FSC_E_NOMEM, "orthogonal iteration workspace too small");
  if (o.validate && (rc = validate_csr(c, g, o.validate, arena, s))) return rc;
  if ((rc = embed_run(c, &io, s))) return rc;
  if ((rc = embed_to_points(c, &io, pts, s))) return rc;
  if (emb && (rc = points_cols_run(pts, g->n, KD, m, emb, s))) return rc;
  km.pts = pts;
  km.elig = io.elig;
  return kmeans_run(c, &km, s);
}

}  // namespace fsc

using namespace fsc;

struct fsc_context {
  Context c;
};

extern "C" {

int fsc_version(void) { return (1 << 16) | 0; }

const char* fsc_last_error(void) { return g_last_error.c_str(); }

int fsc_create(int device, fsc_context** out) {
  if (!out) return fail(FSC_E_ARG, "out is NULL");
  *out = nullptr;
  int rc;
  if ((rc = check_hip(hipSetDevice(device), "hipSetDevice"))) return rc;
  fsc_context* ctx = new fsc_context();
  ctx->c.device = device;
  if ((rc = check_hip(hipGetDeviceProperties(&ctx->c.prop, device), "hipGetDeviceProperties"))) {
    delete ctx;
    return rc;
  }
  ctx->c.num_cu = ctx->c.prop.multiProcessorCount;
  if ((rc = check_hip(hipMalloc(&ctx->c.error_flag, 16), "hipMalloc(flag)"))) {
    delete ctx;
    return rc;
  }
  if ((rc = check_hip(hipHostMalloc(&ctx->c.host_flag, 16, hipHostMallocDefault), "hipHostMalloc(flag)"))) {
    hipFree(ctx->c.error_flag);
    delete ctx;
    return rc;
  }
  // the no-allocation entry point's scratch address on this device; a
  // failure here is reported by that entry point, which tries again
  if (noalloc_setup(device) != FSC_OK) g_last_error.clear();
  *out = ctx;
  return FSC_OK;
}

void fsc_destroy(fsc_context* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->c.device);
  hipDeviceSynchronize();
  for (auto& e : ctx->c.ev_used) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  for (auto& e : ctx->c.ev_free) {
    hipEventDestroy(e.first);
    hipEventDestroy(e.second);
  }
  if (ctx->c.bexec) hipGraphExecDestroy(ctx->c.bexec);
  if (ctx->c.cap_stream) hipStreamDestroy(ctx->c.cap_stream);
  if (ctx->c.barena) hipFree(ctx->c.barena);
  if (ctx->c.arena) hipFree(ctx->c.arena);
  if (ctx->c.error_flag) hipFree(ctx->c.error_flag);
  if (ctx->c.host_flag) hipHostFree(ctx->c.host_flag);
  delete ctx;
}

int fsc_embed(fsc_context* ctx, const fsc_csr* g, int32_t l, int32_t t, uint64_t seed, const fsc_opts* opts,
              void* emb, void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!emb) return fail(FSC_E_ARG, "emb is NULL");
  const fsc_opts o = opts ? *opts : default_opts();
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  EmbedIO io;
  Arena arena;
  if ((rc = prepare_embed(&ctx->c, g, l, t, seed, o, 0, &io, &arena))) return rc;
  if (o.validate && (rc = validate_csr(&ctx->c, g, o.validate, arena, s))) return rc;
  if ((rc = embed_run(&ctx->c, &io, s))) return rc;
  return o.return_y ? embed_y(&ctx->c, &io, emb, s) : embed_unpad(&ctx->c, &io, emb, s);
}

int fsc_cluster(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t l, int32_t t, uint64_t seed,
                const fsc_opts* opts, int32_t* labels, void* emb, float* centres, void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!labels) return fail(FSC_E_ARG, "labels is NULL");
  int rc;
  if ((rc = check_csr(g))) return rc;
  if (k < 1 || k > 64 || k > g->n) return fail(FSC_E_ARG, "k must be in [1, min(n, 64)]");
  const fsc_opts o = opts ? *opts : default_opts();
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  return cluster_run(&ctx->c, g, k, l, t, seed, o, labels, emb, centres, static_cast<hipStream_t>(stream), nullptr);
}

int fsc_cluster_noalloc(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t l, int32_t t, uint64_t seed,
                        const fsc_opts* opts, int32_t* labels, void* emb, float* centres, void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!labels) return fail(FSC_E_ARG, "labels is NULL");
  int rc;
  if ((rc = check_csr(g))) return rc;
  if (k < 1 || k > 64 || k > g->n) return fail(FSC_E_ARG, "k must be in [1, min(n, 64)]");
  if (l < 1 || l > 8) return fail(FSC_E_ARG, "l must be in [1, 8]");
  if (t < 0) return fail(FSC_E_ARG, "t must be >= 0");
  const fsc_opts o = opts ? *opts : default_opts();
  if (o.vec_dtype < FSC_F64 || o.vec_dtype > FSC_BF16) return fail(FSC_E_ARG, "bad vec_dtype");
  if (o.tile_nnz < 0 || (o.tile_nnz > 0 && o.tile_nnz < 64)) return fail(FSC_E_ARG, "tile_nnz must be 0 or >= 64");
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  return cluster_noalloc_run(&ctx->c, g, k, l, t, seed, o, labels, emb, centres, static_cast<hipStream_t>(stream));
}

int fsc_cluster_pmk(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t t, uint64_t seed, const fsc_opts* opts,
                    int32_t* labels, float* emb, double* sigma, void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!labels) return fail(FSC_E_ARG, "labels is NULL");
  int rc;
  if ((rc = check_csr(g))) return rc;
  if (k < 1 || k > 8 || k > g->n) return fail(FSC_E_ARG, "k must be in [1, min(n, 8)]");
  const fsc_opts o = opts ? *opts : default_opts();
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  return ortho_cluster_run(&ctx->c, g, k, k, t, seed, o, labels, emb, sigma, static_cast<hipStream_t>(stream));
}

int fsc_knn(fsc_context* ctx, const float* X, int64_t n, int32_t dim, int32_t knn, int32_t* nbr, float* dist,
            void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!X || !nbr || !dist) return fail(FSC_E_ARG, "null pointer");
  if (n < 2 || n > (1 << 30)) return fail(FSC_E_ARG, "n must be in [2, 2^30]");
  if (dim < 4 || dim > 1024 || dim % 4 != 0) return fail(FSC_E_ARG, "dim must be a multiple of 4 in [4, 1024]");
  if (knn < 1 || knn > 16 || knn > n - 1) return fail(FSC_E_ARG, "knn must be in [1, min(16, n - 1)]");
  if (reinterpret_cast<uintptr_t>(X) % 16 != 0) return fail(FSC_E_ARG, "X must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  Arena arena;
  if ((rc = reserve_arena(&ctx->c, knn_workspace_bytes(n, ctx->c.num_cu), &arena))) return rc;
  return knn_run(&arena, X, n, dim, knn, ctx->c.num_cu, nbr, dist, s);
}

int fsc_knn_graph(fsc_context* ctx, const float* X, int64_t n, int32_t dim, int32_t knn, int64_t* indptr,
                  int32_t* indices, float* weights, void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!X || !indptr || !indices || !weights) return fail(FSC_E_ARG, "null pointer");
  if (n < 2 || n > (1 << 30)) return fail(FSC_E_ARG, "n must be in [2, 2^30]");
  if (dim < 4 || dim > 1024 || dim % 4 != 0) return fail(FSC_E_ARG, "dim must be a multiple of 4 in [4, 1024]");
  if (knn < 1 || knn > 16 || knn > n - 1) return fail(FSC_E_ARG, "knn must be in [1, min(16, n - 1)]");
  if (2 * n * (int64_t)knn > INT32_MAX) return fail(FSC_E_ARG, "2 n knn must be below 2^31");
  if (reinterpret_cast<uintptr_t>(X) % 16 != 0) return fail(FSC_E_ARG, "X must be 16-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  Arena arena;
  if ((rc = reserve_arena(&ctx->c, knn_graph_workspace_bytes(n, knn, ctx->c.num_cu), &arena))) return rc;
  return knn_graph_run(&arena, X, n, dim, knn, ctx->c.num_cu, indptr, indices, weights, s);
}

int fsc_cluster_eigs(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t m, int32_t cycles, int32_t steps,
                     uint64_t seed, const fsc_opts* opts, int32_t* labels, float* emb, double* gamma, void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!labels) return fail(FSC_E_ARG, "labels is NULL");
  int rc;
  if ((rc = check_csr(g))) return rc;
  if (k < 1 || k > 64 || k > g->n) return fail(FSC_E_ARG, "k must be in [1, min(n, 64)]");
  if (m < 1 || m > 8 || m > g->n) return fail(FSC_E_ARG, "m must be in [1, min(n, 8)]");
  if (cycles < 1 || steps < 1) return fail(FSC_E_ARG, "cycles and steps must be >= 1");
  const fsc_opts o = opts ? *opts : default_opts();
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  if ((int64_t)cycles * steps > INT32_MAX) return fail(FSC_E_ARG, "cycles * steps must fit 32 bits");
  fsc_opts oc = o;
  oc.x0 = nullptr;
  return ortho_cluster_run(&ctx->c, g, k, m, cycles * steps, seed, oc, labels, emb, gamma,
                           static_cast<hipStream_t>(stream));
}

int fsc_kmeans(fsc_context* ctx, const void* points, int32_t dtype, int64_t n, int32_t l, int32_t k, int32_t iters,
               uint64_t seed, const uint8_t* eligible, int32_t* labels, float* centres, void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!points || !labels) return fail(FSC_E_ARG, "points and labels must not be NULL");
  if (n < 1 || n > INT32_MAX) return fail(FSC_E_ARG, "n must be in [1, 2^31)");
  if (l < 1 || l > 8) return fail(FSC_E_ARG, "l must be in [1, 8]");
  if (k < 1 || k > 64 || k > n) return fail(FSC_E_ARG, "k must be in [1, min(n, 64)]");
  if (iters < 0) return fail(FSC_E_ARG, "iters must be >= 0");
  if (dtype != FSC_F32 && dtype != FSC_F64) return fail(FSC_E_UNSUPPORTED, "points must be FSC_F32 or FSC_F64");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  const int KD = kmeans_width(l);
  Arena arena;
  if ((rc = reserve_arena(&ctx->c, kmeans_workspace_bytes(n, KD) + align_up(n * KD * 4) + 1024, &arena))) return rc;
  float* pts = arena.take<float>(n * KD);
  KmeansIO km;
  std::memset(&km, 0, sizeof(km));
  km.n = n;
  km.l = l;
  km.KD = KD;
  km.k = k;
  km.iters = iters;
  km.seed = seed;
  km.labels = labels;
  km.centres_out = centres;
  km.elig = eligible;
  if ((rc = kmeans_bind_workspace(&arena, &km))) return rc;
  if ((rc = points_from_user(&ctx->c, points, dtype, n, l, KD, pts, s))) return rc;
  km.pts = pts;
  return kmeans_run(&ctx->c, &km, s);
}

int fsc_ari(fsc_context* ctx, const int32_t* a, const int32_t* b, int64_t n, int32_t ka, int32_t kb, double* out,
            void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!out || (n > 0 && (!a || !b))) return fail(FSC_E_ARG, "null pointer");
  if (n < 0) return fail(FSC_E_ARG, "n must be >= 0");
  if (ka < 1 || kb < 1 || (int64_t)ka * kb > (1 << 22)) return fail(FSC_E_ARG, "need ka, kb >= 1 and ka*kb <= 2^22");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  Arena arena;
  if ((rc = reserve_arena(&ctx->c, align_up((size_t)ka * kb * 8) + 256, &arena))) return rc;
  unsigned long long* table = arena.take<unsigned long long>((size_t)ka * kb);
  return ari_run(&ctx->c, a, b, n, ka, kb, out, table, s);
}

int fsc_nmi(fsc_context* ctx, const int32_t* a, const int32_t* b, int64_t n, int32_t ka, int32_t kb, double* out,
            void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (!out || (n > 0 && (!a || !b))) return fail(FSC_E_ARG, "null pointer");
  if (n < 0) return fail(FSC_E_ARG, "n must be >= 0");
  if (ka < 1 || kb < 1 || (int64_t)ka * kb > (1 << 22)) return fail(FSC_E_ARG, "need ka, kb >= 1 and ka*kb <= 2^22");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  Arena arena;
  if ((rc = reserve_arena(&ctx->c, align_up((size_t)ka * kb * 8) + align_up(((size_t)ka + kb) * 8) + 512, &arena)))
    return rc;
  unsigned long long* table = arena.take<unsigned long long>((size_t)ka * kb);
  double* margin = arena.take<double>((size_t)ka + kb);
  return nmi_run(&ctx->c, a, b, n, ka, kb, out, table, margin, s);
}

int fsc_cluster_batched(fsc_context* ctx, int32_t count, const fsc_csr* graphs, const int32_t* k,
                        const int32_t* l, const int32_t* t, uint64_t seed, const fsc_opts* opts,
                        int32_t* labels, float* emb, void* stream) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  if (count < 1) return fail(FSC_E_ARG, "count must be >= 1");
  if (!graphs || !k || !l || !t || !labels) return fail(FSC_E_ARG, "null pointer");
  const fsc_opts o = opts ? *opts : default_opts();
  if (o.vec_dtype != FSC_F32) return fail(FSC_E_UNSUPPORTED, "the batched form computes in FP32 vectors");
  if (o.renorm || o.sqnorm_trace || o.rayleigh_trace || o.x0 || o.validate)
    return fail(FSC_E_UNSUPPORTED, "the batched form takes no traces, renorm, x0 or validation");
  int rc;
  for (int g = 0; g < count; ++g) {
    if ((rc = check_csr(&graphs[g]))) return fail(rc, "graph " + std::to_string(g) + ": " + fsc_last_error());
    if (graphs[g].val && graphs[g].val_dtype != FSC_F32)
      return fail(FSC_E_UNSUPPORTED, "the batched form takes FP32 or unit weights");
    if (l[g] < 1 || l[g] > 8) return fail(FSC_E_ARG, "l must be in [1, 8]");
    if (t[g] < 0) return fail(FSC_E_ARG, "t must be >= 0");
    if (k[g] < 1 || k[g] > 64 || k[g] > graphs[g].n) return fail(FSC_E_ARG, "k must be in [1, min(n, 64)]");
  }
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  return batched_run(&ctx->c, count, graphs, k, l, t, seed, o, labels, emb, static_cast<hipStream_t>(stream));
}

int fsc_autotune(fsc_context* ctx, const fsc_csr* g, int32_t l, int32_t steps, fsc_tuning* best, void* stream) {
  if (!ctx || !best) return fail(FSC_E_ARG, "null pointer");
  if (steps < 1) return fail(FSC_E_ARG, "steps must be >= 1");
  int rc;
  if ((rc = check_csr(g))) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  const Tune saved = ctx->c.tune;
  const bool saved_timing = ctx->c.timing;
  fsc_opts o = default_opts();
  if (g->val && g->val_dtype != FSC_F32) o.vec_dtype = FSC_BF16;
  Tune bestt = saved;
  double best_ms = 1e30;
  // the trials time the tile kernel (the kernel whose shape is tuned; the
  // batched form runs every graph on it): the column-slab form is off
  const int tiles[] = {256, 512, 1024, 2048, 4096};
  for (int tile : tiles)
    for (int un : {4, 8})
      for (int bpc : {4, 8})
        for (int xo : {1, 0}) {
          Tune tu;
          tu.slab_kb = -1;
          tu.slab_mode = saved.slab_mode;
          tu.tile_nnz = tile;
          tu.unroll = un;
          tu.blocks_per_cu = bpc;
          tu.xcd_order = xo;
          ctx->c.tune = tu;
          EmbedIO io;
          Arena arena;
          if ((rc = prepare_embed(&ctx->c, g, l, steps, 0, o, 0, &io, &arena))) break;
          // discard earlier records, time this shape
          for (auto& e : ctx->c.ev_used) ctx->c.ev_free.push_back(e);
          ctx->c.ev_used.clear();
          ctx->c.timing = true;
          rc = embed_run(&ctx->c, &io, s);
          ctx->c.timing = false;
          if (rc) break;
          double sum = 0.0;
          for (auto& e : ctx->c.ev_used) {
            if ((rc = check_hip(hipEventSynchronize(e.second), "hipEventSynchronize"))) break;
            float ms = 0.f;
            hipEventElapsedTime(&ms, e.first, e.second);
            sum += ms;
          }
          const double avg = ctx->c.ev_used.empty() ? 1e30 : sum / ctx->c.ev_used.size();
          for (auto& e : ctx->c.ev_used) ctx->c.ev_free.push_back(e);
          ctx->c.ev_used.clear();
          if (rc) break;
          if (avg < best_ms) {
            best_ms = avg;
            bestt = tu;
          }
        }
  ctx->c.timing = saved_timing;
  if (rc) {
    ctx->c.tune = saved;
    return rc;
  }
  bestt.slab_kb = saved.slab_kb;
  ctx->c.tune = bestt;
  ctx->c.tile_by_class[degree_class(g->n > 0 ? (double)g->nnz / (double)g->n : 0.0)] = bestt.tile_nnz;
  best->tile_nnz = bestt.tile_nnz;
  best->blocks_per_cu = bestt.blocks_per_cu;
  best->xcd_order = bestt.xcd_order ? 1 : 2;
  best->unroll = bestt.unroll;
  best->slab_kb = bestt.slab_kb > 0 ? bestt.slab_kb : -1;
  best->slab_mode = bestt.slab_mode == 0 ? 3 : bestt.slab_mode;
  return FSC_OK;
}

int fsc_mlp_param_count(void) { return mlp_param_count(); }

static int filter_front(Context* ctx, const fsc_csr* g, int k, int l, uint64_t seed, const fsc_opts& o,
                        size_t extra, EmbedIO* io, Arena* arena, FilterWS* w, hipStream_t s);

int fsc_filter_stats(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t l, int32_t t, uint64_t seed,
                     const fsc_opts* opts, float* features, double* within, double* total, int32_t* labels,
                     void* stream) {
  if (!ctx || !features || !within || !total || !labels) return fail(FSC_E_ARG, "null pointer");
  int rc;
  if ((rc = check_csr(g))) return rc;
  if (l < 1 || l > 8) return fail(FSC_E_ARG, "l must be in [1, 8]");
  if (k < 1 || k > 64 || k > g->n) return fail(FSC_E_ARG, "k must be in [1, min(n, 64)]");
  if (t < 0) return fail(FSC_E_ARG, "t must be >= 0");
  if (g->val && g->val_dtype != FSC_F32) return fail(FSC_E_UNSUPPORTED, "the learned form takes FP32 or unit weights");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  fsc_opts o = opts ? *opts : default_opts();
  o.vec_dtype = FSC_F32;
  o.sqnorm_trace = nullptr;
  o.rayleigh_trace = nullptr;
  o.renorm = 0;
  o.x0 = nullptr;
  // the plain method's labels (Algorithm 2)
  if ((rc = cluster_run(&ctx->c, g, k, l, t, seed, o, labels, nullptr, nullptr, s, nullptr))) return rc;
  // the basis blocks, features, and the scatter statistics under those labels
  EmbedIO io;
  Arena arena;
  FilterWS w;
  const size_t sums_bytes = scatter_workspace_bytes(g->n, l, k);
  if ((rc = filter_front(&ctx->c, g, k, l, seed, o, sums_bytes + 256, &io, &arena, &w, s))) return rc;
  double* sums = arena.take<double>(sums_bytes / 8);
  if (arena.used > arena.size) return fail(FSC_E_NOMEM, "workspace layout overflow");
  if ((rc = gram_run(&ctx->c, &io, w.basis, w.part, w.counter, w.gram, s))) return rc;
  if ((rc = scatter_run(&io, w.basis, labels, k, w.gram, sums, within, total, s))) return rc;
  return check_hip(hipMemcpyAsync(features, w.feat, 9 * 4, hipMemcpyDeviceToDevice, s), "copy features");
}

int fsc_mlp_forward(fsc_context* ctx, const float* params, int32_t count, const float* features, float* coeffs,
                    void* stream) {
  if (!ctx || !params || !features || !coeffs) return fail(FSC_E_ARG, "null pointer");
  if (count < 1) return fail(FSC_E_ARG, "count must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  Arena arena;
  if ((rc = reserve_arena(&ctx->c, mlp_workspace_bytes(count), &arena))) return rc;
  return mlp_coefficients_run(params, count, features, arena.base, coeffs, s);
}

int fsc_mlp_loss_grad(fsc_context* ctx, const float* params, int32_t count, const float* features,
                      const double* within, const double* total, float* grad, double* loss, void* stream) {
  if (!ctx || !params || !features || !within || !total || !grad || !loss) return fail(FSC_E_ARG, "null pointer");
  if (count < 1) return fail(FSC_E_ARG, "count must be >= 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  Arena arena;
  if ((rc = reserve_arena(&ctx->c, mlp_workspace_bytes(count), &arena))) return rc;
  return mlp_loss_grad_run(params, count, features, within, total, grad, loss, arena.base, s);
}

int fsc_mlp_adam(fsc_context* ctx, float* params, float* m, float* v, const float* grad, float lr, int32_t step,
                 void* stream) {
  if (!ctx || !params || !m || !v || !grad) return fail(FSC_E_ARG, "null pointer");
  if (step < 1) return fail(FSC_E_ARG, "step counts from 1");
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  return mlp_adam_run(params, m, v, grad, lr, step, static_cast<hipStream_t>(stream));
}

int fsc_mlp_train(fsc_context* ctx, float* params, float* m, float* v, int32_t count, const float* features,
                  const double* within, const double* total, int32_t steps, float lr, int32_t first_step,
                  double* loss_trace, void* stream) {
  if (!ctx || !params || !m || !v || !features || !within || !total) return fail(FSC_E_ARG, "null pointer");
  if (count < 1 || steps < 0 || first_step < 1) return fail(FSC_E_ARG, "bad count, steps or first_step");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc;
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  const size_t np = mlp_param_count();
  Arena arena;
  if ((rc = reserve_arena(&ctx->c, mlp_workspace_bytes(count) + align_up(np * 4) + align_up(8) + 512, &arena)))
    return rc;
  char* ws = arena.take<char>(mlp_workspace_bytes(count));
  float* grad = arena.take<float>(np);
  double* lbuf = arena.take<double>(1);
  for (int i = 0; i < steps; ++i) {
    double* lo = loss_trace ? loss_trace + i : lbuf;
    if ((rc = mlp_loss_grad_run(params, count, features, within, total, grad, lo, ws, s))) return rc;
    if ((rc = mlp_adam_run(params, m, v, grad, lr, first_step + i, s))) return rc;
  }
  return FSC_OK;
}

// Shared front half of the filtered paths: degrees, start block, basis,
// Rayleigh rows 0..7 and the features.
static int filter_front(Context* ctx, const fsc_csr* g, int k, int l, uint64_t seed, const fsc_opts& o,
                        size_t extra, EmbedIO* io, Arena* arena, FilterWS* w, hipStream_t s) {
  int rc;
  if ((rc = prepare_embed(ctx, g, l, 0, seed, o, filter_extra_bytes(ctx, g, l) + extra, io, arena))) return rc;
  io->need_tiles = 1;  // the Chebyshev steps run the tile kernel
  filter_bind(ctx, arena, io, w);
  if (arena->used > arena->size) return fail(FSC_E_NOMEM, "workspace layout overflow");
  if ((rc = embed_run(ctx, io, s))) return rc;
  if ((rc = zero_counter(w->counter, s))) return rc;
  if ((rc = cheb_basis_run(ctx, io, w->basis, w->ray, s))) return rc;
  return features_run(ctx, io, k, w->ray, w->part, w->counter + 1, w->feat, s);
}

int fsc_filter_embed(fsc_context* ctx, const fsc_csr* g, int32_t l, uint64_t seed, const float* coeffs, float* emb,
                     void* stream) {
  if (!ctx || !coeffs || !emb) return fail(FSC_E_ARG, "null pointer");
  int rc;
  if ((rc = check_csr(g))) return rc;
  if (l < 1 || l > 8) return fail(FSC_E_ARG, "l must be in [1, 8]");
  if (g->val && g->val_dtype != FSC_F32) return fail(FSC_E_UNSUPPORTED, "the learned form takes FP32 or unit weights");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  EmbedIO io;
  Arena arena;
  FilterWS w;
  if ((rc = filter_front(&ctx->c, g, 1, l, seed, default_opts(), 0, &io, &arena, &w, s))) return rc;
  if ((rc = combine_run(&io, w.basis, coeffs, w.S, s))) return rc;
  io.zt = w.S;
  return embed_unpad(&ctx->c, &io, emb, s);
}

int fsc_cluster_filtered(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t l, uint64_t seed,
                         const float* params, const float* coeffs, int32_t fallback_t, const fsc_opts* opts,
                         int32_t* labels, float* coeffs_out, double* diagnostics, int32_t* used_fallback,
                         void* stream) {
  if (!ctx || !labels || (!params && !coeffs)) return fail(FSC_E_ARG, "null pointer");
  int rc;
  if ((rc = check_csr(g))) return rc;
  if (l < 1 || l > 8) return fail(FSC_E_ARG, "l must be in [1, 8]");
  if (k < 1 || k > 64 || k > g->n) return fail(FSC_E_ARG, "k must be in [1, min(n, 64)]");
  if (g->val && g->val_dtype != FSC_F32) return fail(FSC_E_UNSUPPORTED, "the learned form takes FP32 or unit weights");
  fsc_opts o = opts ? *opts : default_opts();
  o.vec_dtype = FSC_F32;
  o.sqnorm_trace = nullptr;
  o.rayleigh_trace = nullptr;
  o.renorm = 0;
  o.x0 = nullptr;
  const int iters = o.kmeans_iters > 0 ? o.kmeans_iters : 30;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = check_hip(hipSetDevice(ctx->c.device), "hipSetDevice"))) return rc;
  const int KD = kmeans_width(l);
  const int LH = padded_width(l);
  const bool direct = LH == KD;
  const size_t extra = kmeans_workspace_bytes(g->n, KD) + (direct ? 0 : align_up(g->n * KD * 4)) + 1024;
  EmbedIO io;
  Arena arena;
  FilterWS w;
  if ((rc = filter_front(&ctx->c, g, k, l, seed, o, extra, &io, &arena, &w, s))) return rc;
  float* pts = direct ? nullptr : arena.take<float>(g->n * KD);
  KmeansIO km;
  std::memset(&km, 0, sizeof(km));
  km.n = g->n;
  km.l = l;
  km.KD = KD;
  km.k = k;
  km.iters = iters;
  km.seed = seed;
  km.labels = labels;
  if ((rc = kmeans_bind_workspace(&arena, &km))) return rc;
  const float* c_rest = coeffs;
  if (!c_rest) {
    if ((rc = mlp_coefficients_run(params, 1, w.feat, w.mlp, w.coef, s))) return rc;
    c_rest = w.coef;
  }
  if ((rc = combine_run(&io, w.basis, c_rest, w.S, s))) return rc;
  if ((rc = rayleigh_run(&ctx->c, &io, w.S, w.ray, 8, s))) return rc;
  // reference: M^8 X0 (the same budget of plain steps), in the free Y buffer
  if ((rc = combine_run(&io, w.basis, nullptr, w.Y, s))) return rc;
  if ((rc = rayleigh_run(&ctx->c, &io, w.Y, w.ray, 9, s))) return rc;
  if (coeffs_out &&
      (rc = check_hip(hipMemcpyAsync(coeffs_out, c_rest, 32, hipMemcpyDeviceToDevice, s), "copy coefficients")))
    return rc;
  io.zt = w.S;
  if (direct) {
    km.pts = w.S;
  } else {
    if ((rc = embed_to_points(&ctx->c, &io, pts, s))) return rc;
    km.pts = pts;
  }
  km.elig = io.elig;
  if ((rc = kmeans_run(&ctx->c, &km, s))) return rc;
  if ((rc = kmeans_cost_run(&ctx->c, &km, w.part, w.counter + 2, w.gram, s))) return rc;
  if ((rc = fallback_run(&io, w.ray, 8, 9, w.gram, kFilterMaxCost, c_rest, w.used, diagnostics, s))) return rc;
  int32_t used = 0;
  if (fallback_t > 0 || used_fallback) {
    if ((rc = check_hip(hipMemcpyAsync(ctx->c.host_flag, w.used, 4, hipMemcpyDeviceToHost, s), "copy flag")))
      return rc;
    if ((rc = check_hip(hipStreamSynchronize(s), "hipStreamSynchronize"))) return rc;
    used = ctx->c.host_flag[0];
  }
  if (used_fallback) *used_fallback = used;
  if (used && fallback_t > 0) {
    fsc_opts po = o;
    return fsc_cluster(ctx, g, k, l, fallback_t, seed, &po, labels, nullptr, nullptr, stream);
  }
  return FSC_OK;
}

int fsc_tuning_set(fsc_context* ctx, fsc_tuning* t) {
  if (!ctx || !t) return fail(FSC_E_ARG, "null pointer");
  Tune nt = ctx->c.tune;
  if (t->tile_nnz > 0) {
    if (t->tile_nnz < 64) return fail(FSC_E_ARG, "tile_nnz must be >= 64");
    nt.tile_nnz = t->tile_nnz;
  }
  if (t->blocks_per_cu > 0) {
    if (t->blocks_per_cu > 16) return fail(FSC_E_ARG, "blocks_per_cu must be in [1, 16]");
    nt.blocks_per_cu = t->blocks_per_cu;
  }
  if (t->xcd_order > 0) nt.xcd_order = t->xcd_order == 1 ? 1 : 0;
  if (t->unroll > 0) {
    if (t->unroll != 4 && t->unroll != 8) return fail(FSC_E_ARG, "unroll must be 4 or 8");
    nt.unroll = t->unroll;
  }
  if (t->slab_kb > 65536) return fail(FSC_E_ARG, "slab_kb must be <= 65536");
  if (t->slab_kb != 0) nt.slab_kb = t->slab_kb > 0 ? t->slab_kb : -1;
  if (t->slab_mode < 0 || t->slab_mode > 4) return fail(FSC_E_ARG, "slab_mode must be in [0, 4]");
  if (t->slab_mode != 0) nt.slab_mode = t->slab_mode == 3 ? 0 : t->slab_mode;
  ctx->c.tune = nt;
  t->tile_nnz = nt.tile_nnz;
  t->blocks_per_cu = nt.blocks_per_cu;
  t->xcd_order = nt.xcd_order ? 1 : 2;
  t->unroll = nt.unroll;
  t->slab_kb = nt.slab_kb > 0 ? nt.slab_kb : -1;
  t->slab_mode = nt.slab_mode == 0 ? 3 : nt.slab_mode;
  return FSC_OK;
}

int fsc_timing_enable(fsc_context* ctx, int on) {
  if (!ctx) return fail(FSC_E_ARG, "context is NULL");
  ctx->c.timing = on != 0;
  if (!on) {
    for (auto& e : ctx->c.ev_used) ctx->c.ev_free.push_back(e);
    ctx->c.ev_used.clear();
  }
  return FSC_OK;
}

int fsc_timing_read(fsc_context* ctx, int64_t* launches, double* total_ms) {
  if (!ctx || !launches || !total_ms) return fail(FSC_E_ARG, "null pointer");
  double sum = 0.0;
  int rc = FSC_OK;
  for (auto& e : ctx->c.ev_used) {
    if (!rc) rc = check_hip(hipEventSynchronize(e.second), "hipEventSynchronize");
    float ms = 0.f;
    if (!rc) rc = check_hip(hipEventElapsedTime(&ms, e.first, e.second), "hipEventElapsedTime");
    sum += ms;
  }
  *launches = (int64_t)ctx->c.ev_used.size();
  *total_ms = sum;
  for (auto& e : ctx->c.ev_used) ctx->c.ev_free.push_back(e);
  ctx->c.ev_used.clear();
  return rc;
}

}  // extern "C"
