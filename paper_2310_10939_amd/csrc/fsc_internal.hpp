// Host-side declarations shared by the libfsc translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/fsc.h"

namespace fsc {

// Sets the calling thread's last-error text and returns `code`.
int fail(int code, const std::string& msg);
// Checks a HIP result; on failure records `what` and returns FSC_E_HIP.
int check_hip(hipError_t e, const char* what);

// Padded row width used for an l-column block.
inline int padded_width(int l) { return l <= 1 ? 1 : l <= 2 ? 2 : l <= 4 ? 4 : 8; }
// Width of the FP32 k-means point rows (the MFMA contraction depth is 4).
inline int kmeans_width(int l) { return l <= 4 ? 4 : 8; }

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// A bump allocator over one device arena owned by the context.
struct Arena {
  char* base = nullptr;
  size_t size = 0;
  size_t used = 0;
  template <typename T>
  T* take(size_t count) {
    size_t off = align_up(used);
    used = off + align_up(count * sizeof(T));
    return reinterpret_cast<T*>(base + off);
  }
};

// One chunk of a long row: the nonzeros [start, end) of `row`; the row has
// `count` chunks, this is number `index`, its partial sums go to slot
// (first + index); `lid` indexes the per-long-row counters.
struct LongChunk {
  int64_t start, end;
  int32_t row, lid, index, count, first, pad;
};

// A short tile: rows [r0, r1), G lanes per row.
struct TileDesc {
  int32_t r0, r1, G, pad;
};

constexpr int kMaxGrid = 4096;

// Column-slab form of the sparse product (fsc_slab.hpp, fsc_slab.hip).
constexpr int kSlabRows = 1024;   // rows per slab tile
constexpr int kSlabLong = 255;    // longer rows are summed by long-row chunks (a length fits a byte)
constexpr int kSlabMax = 16;      // most slabs per graph
constexpr int kSlabChunk = 2048;  // nonzeros per long-row chunk

// Tuning knobs of the sparse product (per context).
struct Tune {
  // defaults: the best shape of a sweep on the 1M-vertex SBM (tile 512..4096,
  // 4 or 8 blocks per CU, both tile orders, 4 or 8 nonzeros in flight)
  int tile_nnz = 512;      // nonzeros per short tile
  int blocks_per_cu = 4;   // persistent blocks per CU
  int xcd_order = 1;       // contiguous short-tile range per XCD
  int unroll = 4;          // nonzeros in flight per lane
  int slab_kb = 1024;      // column-slab size (KiB of the start block); <= 0: off
  int slab_bpc = 8;        // resident blocks per CU of the column-slab kernel (phases)
  int slab_xcd_bpc = 7;    // the same for the per-XCD form
  int slab_mode = 0;       // 0 automatic, 1 phases, 2 per-XCD slabs, 4 waves
  int slab_wave_bpc = 8;   // resident blocks per CU of the wave form
};

// Tile plan of one graph for the sparse product (built on the device).
struct Plan {
  int32_t nb = 0;          // short tiles: buckets of tile_nnz nonzeros
  int32_t tile_nnz = 0;
  TileDesc* desc = nullptr;  // [nb]
  int32_t* nch = nullptr;  // int32[nb]: chunks of the bucket's long last row
  int32_t* choff = nullptr;  // int32[nb+1]: exclusive scan of nch
  int32_t* lid = nullptr;    // int32[nb+1]: exclusive scan of (nch > 0)
  LongChunk* chunks = nullptr;  // up to max_chunks entries
  int32_t max_chunks = 0;
  int32_t* meta = nullptr;      // int32[4]: {total chunks, long rows, -, -}
};

// Column-slab plan of one graph (built on the device by slab_build).
struct SlabPlan {
  int enabled = 0;
  int32_t S = 0, nslab = 0, ntiles = 0, rows = 0;  // slabs of S columns
  int xcd = 0;                 // 1: per-XCD slabs with partial sums
  int wave = 0;                // 1: wave form (each wave owns 64 rows through all slabs)
  uint8_t* wlen = nullptr;     // wave form: [nslab][n] segment length of each row in each slab
  int64_t* gbase = nullptr;    // wave form: [ceil(n/64)] start of each 64-row group's nonzeros
  uint8_t* gunit = nullptr;    // wave form: [ceil(n/64)] 1: the group's weights are all 1
  float* part = nullptr;       // per-XCD form: [n/64][nslab][64][LH] partial sums
  uint8_t* tunit = nullptr;    // [ntiles] 1: every weight of the tile's short rows is 1
  int64_t max_long = 0, max_chunks = 0;
  void* scol = nullptr;        // [nnz] column indices in slab order (uint16_t slab-local when c16, else int32_t)
  int c16 = 0;                 // 1: S <= 65536, indices relative to the slab's first column
  void* sval = nullptr;        // [nnz] weights in slab order (null: unit weights)
  uint16_t* sperm = nullptr;   // [n * nslab]
  int32_t* sbase = nullptr;    // [ntiles * nslab][kSlabLong + 1]
  int32_t* smax = nullptr;     // [ntiles * nslab]
  int64_t* sreg = nullptr;     // [ntiles * nslab]
  int64_t* tshort = nullptr;   // [ntiles] short-row nonzeros per tile
  int64_t* toff = nullptr;     // [ntiles + 1] exclusive scan of tshort
  int32_t* tlong = nullptr;    // [ntiles] long rows per tile
  int32_t* tchunks = nullptr;  // [ntiles] long-row chunks per tile
  int32_t* loff = nullptr;     // [ntiles + 1]
  int32_t* coff = nullptr;     // [ntiles + 1]
  LongChunk* chunks = nullptr; // [max_chunks]
  int32_t* meta = nullptr;     // {chunks, long rows, -, -}
  double* lnorm = nullptr;     // [max_long][2 * LH]
  void* lpart = nullptr;       // float[max_chunks][LH]
  int32_t* lcount = nullptr;   // [max_long]
};

struct Context {
  int device = 0;
  int num_cu = 0;
  hipDeviceProp_t prop{};
  char* arena = nullptr;
  size_t arena_size = 0;
  Tune tune;
  int32_t* error_flag = nullptr;   // device int32[4]
  int32_t* host_flag = nullptr;    // pinned host int32[4]
  // tile size per degree class, filled by the autotuner (0 = use tune)
  int tile_by_class[4] = {0, 0, 0, 0};
  // batched form: its own workspace and the captured launch graph
  char* barena = nullptr;
  size_t barena_size = 0;
  hipGraphExec_t bexec = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only to capture
  uint64_t bkey = 0;
  // event timing of the sparse-product launches
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
};

// Records a (start) event pair slot; returns the pair to close with
// timing_stop, or nullptr when timing is off.
std::pair<hipEvent_t, hipEvent_t>* timing_start(Context* ctx, hipStream_t s);
void timing_stop(std::pair<hipEvent_t, hipEvent_t>* ev, hipStream_t s);

// Grows the context arena to at least `bytes` (synchronises the device when
// it has to reallocate).
int reserve_arena(Context* ctx, size_t bytes, Arena* out);

// ---- embedding pipeline (fsc_embed.hip) ----
// Orthogonal iteration (fsc_pmk.hip): the block is orthonormalised after the
// start block and after every power step.
struct OrthoArgs {
  int k;               // live columns
  int grid;            // blocks of the Gram and sign passes
  double* partials;    // [grid][LH*(LH+1)/2]
  double* W;           // [LH*LH] the current transform
  double* pmax;        // [grid][LH] sign pass: largest |D^{1/2} z| per column
  int64_t* prow;       // [grid][LH] and its row
  double* sigma_out;   // FP64[k]: the last step's singular values (optional)
};

struct EmbedIO {
  // inputs
  const fsc_csr* g;
  int l, t, LH;
  uint64_t seed;
  int vec_dtype;
  int renorm;
  int tile_nnz;
  const double* x0;
  double* sqnorm_trace;
  double* rayleigh_trace;
  int need_tiles;   // 1: build the tile plan even when the steps take the slab form (later tile kernels use it)
  OrthoArgs* ortho; // non-null: orthogonal iteration (fsc_pmk.hip)
  // workspace (filled by embed_workspace)
  double* deg;
  void* hinv;       // float[n] or double[n]
  double* isq;
  uint8_t* elig;
  void* z[2];       // S[n*LH] ping-pong
  double* partials; // [grid][2*LH]
  double* state;    // [5][LH]: prev_sq, cum, scale, scale as A, spare
  double* lnorm;    // [max long rows][2*LH]
  void* lpart;      // A[max chunks][LH]
  int32_t* lcount;  // [max long rows]
  Plan plan;
  SlabPlan slab;    // column-slab plan (slab.enabled = 0: plain tiles)
  int grid;         // persistent grid of the sparse product
  // result: pointer to Z_t (S[n*LH]) inside the workspace
  const void* zt;
};

// Largest tile size whose LDS staging fits a block's budget.
int max_tile_nnz(int l, int vec_dtype);
size_t embed_workspace_bytes(const Context* ctx, const fsc_csr* g, int l, int vec_dtype, int tile_nnz);
// Zeroes count int32 values with a kernel (capturable, unlike a memset node).
int fill_zero_i32(int32_t* p, int64_t count, hipStream_t s);
// Tile size used when fsc_opts.tile_nnz is 0.
int effective_tile_nnz(const Context* ctx, int tile_nnz);
int embed_bind_workspace(Context* ctx, Arena* a, EmbedIO* io);
// Enqueues validation (optional), degrees, start block, t steps and stats.
int embed_run(Context* ctx, EmbedIO* io, hipStream_t s);
// Writes Z_t (n x LH, vec dtype) to an unpadded n x l array of the same dtype.
int embed_unpad(Context* ctx, const EmbedIO* io, void* out, hipStream_t s);
// Writes Z_t as FP32 n x KD k-means points (KD = kmeans_width(l)).
int embed_to_points(Context* ctx, const EmbedIO* io, float* pts, hipStream_t s);
// Writes Y = D^{1/2} Z_t (the PowerMethod iterates, n x l, vec dtype).
int embed_y(Context* ctx, const EmbedIO* io, void* out, hipStream_t s);
// Device-side validation of a CSR; synchronises `s`.  Returns FSC_OK or
// FSC_E_GRAPH.  Level 2 also checks symmetry (fsc_validate.hip) in
// `scratch`, which must hold symmetry_workspace_bytes(g) and must not hold
// live data (validation runs before the call's other kernels).
int validate_csr(Context* ctx, const fsc_csr* g, int level, const Arena& scratch, hipStream_t s);
size_t symmetry_workspace_bytes(const fsc_csr* g);
int validate_symmetry(Context* ctx, const fsc_csr* g, Arena scratch, hipStream_t s);

// ---- column-slab plan (fsc_slab.hip) ----
// Slab shape for an n-row block of LH columns: true (and the slab width S,
// nslab, and the form) when the block is larger than one slab of
// ctx->tune.slab_kb KiB.
bool slab_shape(const Context* ctx, int64_t n, int LH, int vec_dtype, int32_t* S, int32_t* nslab, int* xcd);
size_t slab_workspace_bytes(const Context* ctx, const fsc_csr* g, int LH, int vec_dtype);
// Takes the slab arrays from the arena (sets io->slab.enabled when used).
int slab_bind(Context* ctx, Arena* a, EmbedIO* io);
// Enqueues the kernels that build io->slab from the CSR.
int slab_build(Context* ctx, EmbedIO* io, hipStream_t s);

// ---- k-means (fsc_kmeans.hip) ----
struct KmeansIO {
  int64_t n;
  int l, KD, k, iters;
  uint64_t seed;
  const float* pts;        // n x KD FP32
  const uint8_t* elig;     // optional
  int32_t* labels;         // n
  float* centres_out;      // optional k x l
  // workspace
  float* d2;               // n
  double* bsum;            // blocks x 6
  float* cand;             // 6 x KD: the seeding round's candidates
  int32_t* cand_row;       // 6
  float* centres;          // 64 x KD (padded)
  double* cpart;           // blocks x 64 x (KD+1)
  int32_t* chosen;         // 64
  int32_t* conv;           // 4: labels changed by the current Lloyd step; 1 once a step changed none
  int nblk_pp, nblk_ll;
};
// One k-means problem as the kernels see it.
struct KmJob {
  int64_t n;
  const float* pts;        // n x KD
  const uint8_t* elig;     // optional
  int KD, k;
  float* d2;
  double* bsum;
  float* cand;
  int32_t* cand_row;
  int trials;              // candidates per seeding round
  float* centres;          // 64 x KD
  int32_t* chosen;
  int32_t* labels;
  double* cpart;
  uint32_t k0, k1;         // Philox key (seed)
  int nblk_pp, nblk_ll, tpw;
  int32_t* conv;           // Lloyd convergence state (KmeansIO::conv)
};
void kmeans_shape(int64_t n, int num_cu, int* nblk_pp, int* nblk_ll, int* tpw);
int kpp_trials(int k);
KmJob make_job(Context* ctx, const KmeansIO* io);
int kmeans_run_batched(Context* ctx, const KmJob* jobs_dev, const int32_t* pp_off_dev, int pp_total,
                       const int32_t* ll_off_dev, int ll_total, int njobs, int kmax, int iters, hipStream_t s);
size_t kmeans_workspace_bytes(int64_t n, int KD);
int kmeans_bind_workspace(Arena* a, KmeansIO* io);
int kmeans_run(Context* ctx, KmeansIO* io, hipStream_t s);
int kmeans_cost_run(Context* ctx, const KmeansIO* io, double* partials, int32_t* counter, double* out,
                    hipStream_t s);
int points_from_user(Context* ctx, const void* pts, int dtype, int64_t n, int l, int KD, float* out,
                     hipStream_t s);

// ---- the plain single-graph path (fsc_api.hip) ----
// Workspace of cluster_run on the context arena, and the run itself (labels,
// optional unpadded embedding and centres); it reserves the arena, which
// allocates only when the arena is too small.
size_t cluster_workspace_bytes(const Context* ctx, const fsc_csr* g, int l, const fsc_opts& o);
// With ws, the run uses that workspace instead of the context arena.
// The no-allocation entry point's scratch (fsc_noalloc.hip).
int noalloc_setup(int device);
int cluster_noalloc_run(Context* ctx, const fsc_csr* g, int k, int l, int t, uint64_t seed, const fsc_opts& o,
                        int32_t* labels, void* emb, float* centres, hipStream_t s);
int cluster_run(Context* c, const fsc_csr* g, int k, int l, int t, uint64_t seed, const fsc_opts& o,
                int32_t* labels, void* emb, float* centres, hipStream_t s, const Arena* ws);

// ---- batched form (fsc_batched.hip) ----
inline int degree_class(double mean_degree) {
  return mean_degree < 12.0 ? 0 : mean_degree < 24.0 ? 1 : mean_degree < 48.0 ? 2 : 3;
}
int tile_for_degree(const Context* ctx, double mean_degree);
int batched_run(Context* ctx, int G, const fsc_csr* graphs, const int32_t* ks, const int32_t* ls,
                const int32_t* ts, uint64_t seed, const fsc_opts& o, int32_t* labels, float* emb, hipStream_t s);

// ---- learned form (fsc_filter.hip, fsc_mlp.hip) ----
int cheb_basis_run(Context* ctx, EmbedIO* io, float* const* basis, double* ray, hipStream_t s);
int rayleigh_run(Context* ctx, EmbedIO* io, const float* x, double* ray, int row, hipStream_t s);
int gram_run(Context* ctx, const EmbedIO* io, float* const* basis, double* partials, int32_t* counter, double* out,
             hipStream_t s);
size_t scatter_workspace_bytes(int64_t n, int l, int k);
int scatter_run(const EmbedIO* io, float* const* basis, const int32_t* labels, int k, const double* gram,
                double* sums, double* within, double* total, hipStream_t s);
int features_run(Context* ctx, const EmbedIO* io, int k, const double* ray, double* partials, int32_t* counter,
                 float* feat, hipStream_t s);
int combine_run(const EmbedIO* io, float* const* basis, const float* c_rest, float* S, hipStream_t s);
int fallback_run(const EmbedIO* io, const double* ray, int row_f, int row_ref, const double* kcost, double kmax,
                 const float* c_rest, int32_t* used, double* diag, hipStream_t s);
int mlp_param_count();
size_t mlp_workspace_bytes(int B);
int mlp_forward_run(const float* params, int B, const float* feats, float* acts, float* raw, hipStream_t s);
int mlp_coefficients_run(const float* params, int B, const float* feats, char* ws, float* c_out, hipStream_t s);
int mlp_loss_grad_run(const float* params, int B, const float* feats, const double* W, const double* T,
                      float* grad, double* loss_out, char* ws, hipStream_t s);
int mlp_adam_run(float* p, float* m, float* v, const float* g, float lr, int step, hipStream_t s);

// ---- PM with k vectors (fsc_pmk.hip) ----
size_t ortho_workspace_bytes(int64_t n, int LH);
void ortho_bind(Arena* a, int64_t n, int LH, int k, OrthoArgs* oa);
// Orthonormalises the block z (n x LH, the io's vector dtype) in place; on
// the last step also fixes the column signs and writes sigma_out.
int ortho_run(const EmbedIO* io, void* z, bool last, hipStream_t s);
// Copies the first k values of each FP32 point row (width KD) to n x k.
int points_cols_run(const float* pts, int64_t n, int KD, int k, float* out, hipStream_t s);

// ---- k-nearest neighbours (fsc_knn.hip) ----
size_t knn_workspace_bytes(int64_t n, int num_cu);
int knn_run(Arena* a, const float* X, int64_t n, int dim, int knn, int num_cu, int32_t* nbr, float* dist,
            hipStream_t s);
size_t knn_graph_workspace_bytes(int64_t n, int knn, int num_cu);
int knn_graph_run(Arena* a, const float* X, int64_t n, int dim, int knn, int num_cu, int64_t* indptr, int32_t* indices,
                  float* weights, hipStream_t s);

// ---- ARI and NMI (fsc_ari.hip) ----
int ari_run(Context* ctx, const int32_t* a, const int32_t* b, int64_t n, int ka, int kb, double* out,
            unsigned long long* table, hipStream_t s);
int nmi_run(Context* ctx, const int32_t* a, const int32_t* b, int64_t n, int ka, int kb, double* out,
            unsigned long long* table, double* margin, hipStream_t s);

}  // namespace fsc
