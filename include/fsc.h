/*
 * fsc.h -- C ABI of libfsc, an MI355X (gfx950) implementation of the hot path
 * of FastSpectralCluster (Macgregor, "Fast and Simple Spectral Clustering in
 * Theory and Practice", NeurIPS 2023).
 *
 * The method (Sec. 3.2, Algorithm 2): with M = I - N/2 = (I + D^{-1/2} A
 * D^{-1/2}) / 2 the halved signless Laplacian of a weighted undirected graph
 * (Sec. 2; eigenvalues in [0, 1]), draw l Gaussian vectors, apply M to each of
 * them t times (Algorithm 1, PowerMethod, no normalisation), stack them into
 * Y and run k-means (k-means++ seeding, then Lloyd; Sec. 2.2) on the rows of
 * D^{-1/2} Y.
 *
 * Conventions shared by every entry point:
 *   - Every array argument is a DEVICE pointer on the context's device, owned
 *     by the caller, unless stated otherwise.  The library never frees or
 *     keeps caller memory past the call's stream work.
 *   - `stream` is a hipStream_t passed as a plain pointer (NULL = the null
 *     stream).  Every call only enqueues work on that stream and returns; the
 *     results are ready when the stream reaches that point.  Argument errors
 *     are reported synchronously by the return value; device-side failures
 *     surface as FSC_E_HIP on this or a later call.
 *   - Arrays of n x l values are row-major: vertex i's l values are adjacent.
 *   - Labels are 0..k-1 and meaningful up to a permutation of the clusters.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by `seed`.
 *     Start-block entry (i, j) uses counter (i_lo, i_hi, j, 0) and the
 *     Box-Muller transform of the two 53-bit uniforms it yields.  k-means++
 *     seeding is greedy: centre 0 is a uniform draw over the eligible rows
 *     (counter (0, 0, 0, 1)); centre r >= 1 is the best of L = 2 + floor(ln k)
 *     candidates drawn with probability proportional to D^2, candidate j
 *     with counter (r L + j, 0, 0, 3), the one that lowers
 *     sum_v min(D^2(v), ||x_v - c||^2) most (ties to the lower j).
 *   - An isolated vertex (degree 0) has no D^{-1/2} (Sec. 2); it is given
 *     D^{-1/2} := 0, so its embedding row is 0.  It takes no part in k-means
 *     seeding or centre updates and is labelled by its nearest final centre.
 *   - A context is used by one host thread at a time; calls on one context
 *     share its workspace and must be issued on one stream (or be ordered).
 */
#ifndef FSC_H
#define FSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes.  Every entry point returns one. */
typedef enum {
  FSC_OK = 0,
  FSC_E_ARG = -1,          /* bad argument: null pointer, size out of range, bad dtype */
  FSC_E_GRAPH = -2,        /* validation found a self-loop, a negative/NaN weight,
                              an index out of range, a bad row pointer or (level
                              2) an asymmetric adjacency */
  FSC_E_HIP = -3,          /* a HIP runtime call or kernel launch failed */
  FSC_E_NOMEM = -4,        /* device workspace allocation failed */
  FSC_E_UNSUPPORTED = -5   /* combination of dtypes or sizes not built */
} fsc_status;

/* Element types. */
typedef enum {
  FSC_F64 = 0,   /* IEEE binary64 */
  FSC_F32 = 1,   /* IEEE binary32 */
  FSC_BF16 = 2   /* bfloat16 (upper half of a binary32), round-to-nearest-even */
} fsc_dtype;

/* A weighted undirected graph G = (V, E, w) (Sec. 2) as CSR storing both
 * directions of every edge, so nnz = 2m.  Device pointers.
 *   row_ptr: int64[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz.
 *   col_idx: int32[nnz], each in [0, n); entries of a row in any order.
 *   val:     nnz weights of type val_dtype (> 0 finite), or NULL for unit
 *            weights.
 * Preconditions (checked only when fsc_opts.validate != 0): no self-loops,
 * symmetric A, non-negative finite weights.  On a graph that breaks them the
 * result is unspecified, but every access stays in bounds as long as row_ptr
 * and col_idx are in range. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const void* val;
  int32_t val_dtype;  /* fsc_dtype; ignored when val == NULL */
} fsc_csr;

/* Options (all fields may be zero for the defaults). */
typedef struct {
  /* Storage and arithmetic type of the iterate block and of the embedding
   * written by fsc_embed: FSC_F64 (FP64 accumulation), FSC_F32 or FSC_BF16
   * (FP32 accumulation).  Degrees and column statistics are always FP64. */
  int32_t vec_dtype;
  /* Lloyd steps after k-means++ seeding (fsc_cluster); 0 means 30. */
  int32_t kmeans_iters;
  /* 0: no checks.  1: check row_ptr, column range, self-loops and weights on
   * the device; this synchronises the stream and returns FSC_E_GRAPH on
   * failure.  2: also check that A is symmetric (Sec. 2: G is undirected):
   * A(r, c) == A(c, r) for every stored entry, duplicate entries of one
   * position adding up (FP64, in ascending order of weight), an absent
   * mirror counting as 0; the entries are radix-sorted on the device in
   * workspace of about 32 bytes per nonzero (needs nnz < 2^31, else
   * FSC_E_UNSUPPORTED).  Other values: FSC_E_ARG. */
  int32_t validate;
  /* Non-zero: after every step rescale each column of the iterate to unit
   * D-norm (y-space), keeping the FP64 product of the scales, and undo the
   * product at the last step, so the result equals the un-normalised
   * PowerMethod output up to rounding.  Algorithm 1 itself has no
   * normalisation; this only guards the range of low-precision storage. */
  int32_t renorm;
  /* Optional FP64 n x l start block X0 (overrides the seeded Gaussian). */
  const double* x0;
  /* Optional FP64 outputs, (t+1) x l and t x l: sqnorm[i][j] = ||y_i^(j)||^2
   * and rayleigh[i][j] = y_i^T M y_i / y_i^T y_i for the j-th PowerMethod
   * iterate (both over non-isolated vertices). */
  double* sqnorm_trace;
  double* rayleigh_trace;
  /* Tile size of the sparse product in nonzeros (0 = tuned default). */
  int32_t tile_nnz;
  /* fsc_cluster_batched only: 1 = queue the launches directly instead of
   * capturing them into a hipGraph (which is replayed while the batch stays
   * the same). */
  int32_t no_graph;
  /* fsc_embed only: non-zero writes Y = D^{1/2} Z_t, the PowerMethod
   * iterates of Algorithm 1 (Algorithm 2's Y), instead of the embedding
   * D^{-1/2} Y; an isolated vertex's row is 2^-t times its row of X0 (its row
   * of M is e_v / 2). */
  int32_t return_y;
} fsc_opts;

typedef struct fsc_context fsc_context;

/* Launch shape of the sparse product (the tile kernel of one PowerMethod
 * step), per context.  Zero fields keep the current value. */
typedef struct {
  int32_t tile_nnz;       /* nonzeros per short tile (default 512) */
  int32_t blocks_per_cu;  /* persistent blocks per compute unit (default 4) */
  int32_t xcd_order;      /* 1: contiguous short-tile range per XCD (default), 2: round robin */
  int32_t unroll;         /* nonzeros in flight per lane: 4 (default) or 8 */
  /* Column-slab size in KiB of the n x l block (default 1024; < 0 turns the
   * slab form off).  When an FP32 or BF16 block is larger than one slab, the
   * columns are cut into slabs of this size (at most 16; larger slabs if
   * needed) and each step gathers from one slab at a time, so that the rows
   * an XCD gathers stay in its L2.  Results do not depend on it beyond
   * summation order. */
  int32_t slab_kb;
  /* Which slab form (0 keeps the current one): 1 phases -- every block walks
   * all slabs, one at a time, its rows' sums in LDS; 2 per-XCD -- 8 slabs,
   * one per XCD, whose per-row partial sums a second kernel adds in slab
   * order; 4 waves -- every wave takes its 64 rows through all slabs with the
   * sums in registers (same results as phases, bit for bit); 3 automatic
   * (default: phases). */
  int32_t slab_mode;
} fsc_tuning;

/* Creates a context on HIP device `device` (makes it current on the calling
 * thread).  *out receives the context.  Returns FSC_E_HIP if the device is not
 * usable. */
int fsc_create(int device, fsc_context** out);

/* Waits for the context's outstanding work and frees its workspace. */
void fsc_destroy(fsc_context* ctx);

/* The embedding D^{-1/2} Y of Algorithm 2: Y's columns are PowerMethod(M,
 * x_i, t) (Algorithm 1) for the l start vectors.  `emb` receives n x l values
 * of type opts->vec_dtype.  1 <= l <= 8, t >= 0 (t = 0 gives D^{-1/2} X0). */
int fsc_embed(fsc_context* ctx, const fsc_csr* g, int32_t l, int32_t t, uint64_t seed,
              const fsc_opts* opts, void* emb, void* stream);

/* FastSpectralCluster (Algorithm 2): the embedding above, then k-means++
 * seeding and opts->kmeans_iters Lloyd steps on its rows, then a final
 * assignment.  `labels` receives int32[n].  Optional outputs (NULL to skip):
 * `emb` (n x l of vec_dtype, as fsc_embed) and `centres` (FP32 k x l).
 * 1 <= k <= min(n, 64). */
int fsc_cluster(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t l, int32_t t,
                uint64_t seed, const fsc_opts* opts, int32_t* labels, void* emb,
                float* centres, void* stream);

/* fsc_cluster without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, results and errors as fsc_cluster, but
 * its workspace is a fixed device array of FSC_NOALLOC_MAX_BYTES that the
 * library holds on every GPU it runs on until the process ends (its address
 * is resolved when a context is created on that device).  A graph whose
 * workspace exceeds that size returns FSC_E_NOMEM with the sizes in
 * fsc_last_error().  Every call on one GPU shares that GPU's array and leaves
 * the last call's contents there: calls that overlap on one GPU (other
 * streams, other contexts, other threads) race.  Event timing is off in it. */
#define FSC_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int fsc_cluster_noalloc(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t l, int32_t t, uint64_t seed,
                        const fsc_opts* opts, int32_t* labels, void* emb, float* centres, void* stream);

/* k-means (Sec. 2.2) alone on n points of dimension l (1 <= l <= 8) stored as
 * n x l values of `dtype` (FSC_F32 or FSC_F64; computed in FP32): k-means++
 * seeding then `iters` Lloyd steps and a final assignment.  `eligible` is an
 * optional uint8[n] mask (0 = the point takes no part in seeding/updates).
 * Outputs labels int32[n] and, if non-NULL, centres FP32 k x l. */
int fsc_kmeans(fsc_context* ctx, const void* points, int32_t dtype, int64_t n, int32_t l,
               int32_t k, int32_t iters, uint64_t seed, const uint8_t* eligible,
               int32_t* labels, float* centres, void* stream);

/* The batched form: FastSpectralCluster on `count` independent graphs of
 * uneven size in one call.  `graphs`, `k`, `l` and `t` are HOST arrays of
 * `count` entries (the CSR fields themselves are device pointers); graph g
 * uses seed + g (so its result equals fsc_cluster on that graph with that
 * seed, up to summation order).  Every stage runs once over the whole batch:
 * the power iterations level by level, each level one grid per block width
 * over the tiles of all graphs still iterating, with every graph's tiles
 * given to one XCD (balanced by nonzeros times steps; the block index mod 8
 * picks the XCD) so that its iterate block stays in that XCD's L2; then the
 * k-means rounds over all graphs.  The whole launch sequence is captured into
 * a hipGraph that is replayed while the batch (pointers, sizes, parameters)
 * is unchanged.  Outputs: `labels`, int32 concatenated per graph (graph g at
 * offset sum_{h<g} n_h); optional `emb`, FP32 concatenated n_g x l_g blocks.
 * Supported: FP32 vectors, FP32 or unit weights, 1 <= l <= 8,
 * 1 <= k <= min(n, 64), no traces or re-normalisation (FSC_E_UNSUPPORTED
 * otherwise).  The tile size of each graph comes from the autotuned entry of
 * its mean-degree class. */
int fsc_cluster_batched(fsc_context* ctx, int32_t count, const fsc_csr* graphs, const int32_t* k,
                        const int32_t* l, const int32_t* t, uint64_t seed, const fsc_opts* opts,
                        int32_t* labels, float* emb, void* stream);

/* Autotuner of the sparse-product launch shape: times `steps` power steps of
 * graph g (l columns, FP32) with the tile kernel (the column-slab form off
 * during the trials) under each candidate shape (tile size 256..4096, 4 or 8
 * nonzeros in flight per lane, 4 or 8 blocks per CU, both tile orders) with
 * HIP events, makes the fastest the context default (the slab setting is
 * kept), records its tile size for the graph's mean-degree class (used by
 * fsc_cluster_batched, whose graphs all run the tile kernel) and writes it to
 * *best (host).  Synchronises the stream. */
int fsc_autotune(fsc_context* ctx, const fsc_csr* g, int32_t l, int32_t steps, fsc_tuning* best,
                 void* stream);

/* ---------------------------------------------------------------------------
 * The learned polynomial-filter form.
 *
 * PowerMethod (Algorithm 1) applies M^t, i.e. gamma^t on each eigenvalue of
 * M (Sec. 3.1).  This form applies p(M) = sum_{j=0..8} c_j T*_j(M) instead,
 * with T*_j the Chebyshev polynomials shifted to [0, 1] and c_0 = 1 -
 * sum_{j>0} c_j so that p(1) = 1 (gamma_1 = 1 keeps its weight): 8 sparse
 * products instead of t.  A small MLP (9 inputs, 3 hidden layers of 128 with
 * ReLU, 2 outputs (alpha, beta), FP32) picks the part of the spectrum to
 * damp, the interval [a, b] with b = 1 - e^beta and a = b - e^alpha, and a
 * fixed head makes the filter the Chebyshev polynomial of that interval,
 * p(gamma) = T_8(u(gamma)) / T_8(u(1)) with u = (2 gamma - a - b) / (b - a),
 * the degree-8 polynomial with p(1) = 1 that is smallest on [a, b]; c_0..c_8
 * are its coefficients in the T*_j basis.  The MLP's inputs, in order: log n,
 * log k, log mean degree, log(1 + the degree's coefficient of variation),
 * log(max degree / mean degree) (over non-isolated vertices), and the
 * column-mean Rayleigh quotients <B_j, M B_j> / <B_j, B_j> of the basis
 * blocks B_j = T*_j(M) X0, j = 0..3; each input is then centred and scaled by
 * fixed constants (12, 2, 3, 1, 5, 0, 0, 0, 0) and (2, 1, 1, 1, 2, 1, 1, 1,
 * 1).  Parameters: one flat FP32 array of fsc_mlp_param_count() values, for
 * each layer W (out x in, row-major) then b.  The paper has no learned part;
 * this is built on top of its method.
 * ------------------------------------------------------------------------- */

/* Number of MLP parameters (34562). */
int fsc_mlp_param_count(void);

/* Training statistics of one graph (FP32 vectors).  The plain method
 * (Algorithm 2: t PowerMethod steps from the start block of `seed`, then
 * k-means with opts->kmeans_iters Lloyd steps; opts may be NULL, its vector
 * type, traces, renorm and x0 are ignored) labels the vertices: labels
 * (device int32[n]).  Over the non-isolated vertices, the filtered embedding
 * E(c) = D^{-1/2} p(M) X0 = sum_j c_j B_j (B_j = D^{-1/2} T*_j(M) X0, the
 * same X0) has within-cluster scatter c^T W c under those labels (the k-means
 * cost of Sec. 2.2) and total scatter c^T T c (its value for one cluster):
 * within and total (device FP64 9 x 9, row-major, symmetric).  features:
 * device float[9].  The MLP's training loss of the graph is the ratio
 * c^T W c / c^T T c for the coefficients c its outputs give, the normalised
 * k-means cost, in [0, 1] and independent of the scale of c.
 * k in [1, min(n, 64)], l in [1, 8], t >= 0. */
int fsc_filter_stats(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t l, int32_t t, uint64_t seed,
                     const fsc_opts* opts, float* features, double* within, double* total, int32_t* labels,
                     void* stream);

/* Filter coefficients c_1..c_8 (device float[count][8]) for `count` feature
 * rows (device float[count][9]): the MLP's outputs through the head. */
int fsc_mlp_forward(fsc_context* ctx, const float* params, int32_t count, const float* features,
                    float* coeffs, void* stream);

/* Mean training loss over `count` graphs (device double[1]) and its gradient
 * in the parameters (device float[param_count]); features (float[count][9]),
 * within and total (double[count][81]) as produced by fsc_filter_stats,
 * stacked.  The gradient runs through the head (FP64) and the MLP (FP32).
 * A graph whose total scatter c^T T c is 0 contributes 0 with a zero
 * gradient. */
int fsc_mlp_loss_grad(fsc_context* ctx, const float* params, int32_t count, const float* features,
                      const double* within, const double* total, float* grad, double* loss, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; `step`
 * counts from 1) on params with moment buffers m, v (device, zeroed before
 * step 1). */
int fsc_mlp_adam(fsc_context* ctx, float* params, float* m, float* v, const float* grad, float lr,
                 int32_t step, void* stream);

/* `steps` full-batch Adam steps of the loss above, all on the device;
 * loss_trace (device double[steps], optional) receives the loss before each
 * step.  m and v must be zero for a fresh start; `first_step` is the Adam step
 * number of the first update (1 for a fresh start). */
int fsc_mlp_train(fsc_context* ctx, float* params, float* m, float* v, int32_t count, const float* features,
                  const double* within, const double* total, int32_t steps, float lr, int32_t first_step,
                  double* loss_trace, void* stream);

/* The filtered embedding D^{-1/2} p(M) X0 with given coefficients c_1..c_8
 * (device float[8]); emb: FP32 n x l. */
int fsc_filter_embed(fsc_context* ctx, const fsc_csr* g, int32_t l, uint64_t seed, const float* coeffs,
                     float* emb, void* stream);

/* The learned form of FastSpectralCluster: features, then the MLP (params,
 * device) or the given coefficients (coeffs, device float[8], overrides the
 * MLP when non-NULL), the filtered embedding, a fallback check, and k-means
 * (opts->kmeans_iters Lloyd steps).  Fallback check: (a) the column-mean
 * Rayleigh quotient <S, M S> / <S, S> of the filtered block S is below that
 * of M^8 X0 (what 8 plain PowerMethod steps give; computed from the same
 * basis with the exact Chebyshev coefficients of gamma^8), or (b) the
 * normalised k-means cost of the filtered embedding (within-cluster over
 * total variance) exceeds 0.1, or (c) a coefficient is not finite.  When it
 * fires and fallback_t > 0, the plain method with t = fallback_t overwrites
 * the labels; reading the check synchronises the stream.  Outputs: labels
 * int32[n]; optional coeffs_out (device float[8]); optional diagnostics
 * (device double[4]: the two Rayleigh quotients, the normalised cost, the
 * flag); optional *used_fallback (host). */
int fsc_cluster_filtered(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t l, uint64_t seed,
                         const float* params, const float* coeffs, int32_t fallback_t, const fsc_opts* opts,
                         int32_t* labels, float* coeffs_out, double* diagnostics, int32_t* used_fallback,
                         void* stream);

/* PM with k vectors, the comparison method of Sec. 4 (k mutually orthogonal
 * vectors computed with the power method, the algorithm of Boutsidis et al.;
 * Sec. 1.1 notes its singular value decomposition), as orthogonal iteration:
 * the start block and power steps of fsc_embed with l = k, the block
 * orthonormalised after the start block and after every step, so that
 * D^{1/2} Z_i holds the left singular vectors of Y_i = M (D^{1/2} Z_{i-1})
 * over the non-isolated rows.  Each orthonormalisation takes the FP64 Gram
 * matrix Y^T Y = sum_v d_v z_v z_v^T and its cyclic Jacobi eigenvectors.  In
 * exact arithmetic the span after t steps is that of M^t X0; every direction
 * stays resolved at any t.  k-means then runs exactly as in fsc_cluster on
 * the rows of D^{-1/2} U, U = D^{1/2} Z_t.  Columns of U come in descending
 * order of singular value; a column whose singular value within one step is
 * at most 1e-6 of the largest is set to 0 (the Gram matrix of the stored rows
 * cannot resolve it; it stays 0); after the last step each column's sign
 * makes its largest-magnitude entry positive (the first such row on a tie).
 * `labels` receives int32[n].  Optional outputs (NULL to skip): `emb` (FP32
 * n x k, the rows k-means sees) and `sigma` (FP64 [k], the singular values of
 * the last step's Y, descending; Y = X0 when t = 0).  1 <= k <= min(n, 8);
 * vec_dtype FSC_F32 or FSC_F64 (else FSC_E_UNSUPPORTED); opts as for
 * fsc_cluster otherwise (x0, when given, is n x k; the traces and renorm are
 * ignored). */
int fsc_cluster_pmk(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t t, uint64_t seed,
                    const fsc_opts* opts, int32_t* labels, float* emb, double* sigma, void* stream);

/* The eigenvector baselines of Sec. 4 ("k Eigenvectors" with m = k,
 * "log(k) Eigenvectors" with m = log k): the m leading eigenvectors of M
 * (the m smallest of the normalised Laplacian), reached by the orthogonal
 * iteration of fsc_cluster_pmk on m columns for cycles * steps steps from the
 * seeded Gaussian block, then k-means exactly as fsc_cluster on the rows of
 * D^{-1/2} U.  The span converges to the leading eigenvectors at the rate
 * (gamma_{m+1} / gamma_m)^(cycles*steps).  `labels` receives int32[n].
 * Optional outputs (NULL to skip): `emb` (FP32 n x m, the rows k-means sees)
 * and `gamma` (FP64 [m], the eigenvalue estimates: the singular values of
 * M U for the orthonormal U of the second-to-last step, which equal the
 * eigenvalues once U has converged).  1 <= k <= min(n, 64),
 * 1 <= m <= min(n, 8), cycles, steps >= 1 with cycles * steps < 2^31;
 * opts as for fsc_cluster_pmk (x0 is ignored). */
int fsc_cluster_eigs(fsc_context* ctx, const fsc_csr* g, int32_t k, int32_t m, int32_t cycles, int32_t steps,
                     uint64_t seed, const fsc_opts* opts, int32_t* labels, float* emb, double* gamma,
                     void* stream);

/* Exact k nearest neighbours of every point, the pre-processing of the
 * real-world data in Sec. 4.2 (each point joined to its 10 nearest).  X is a
 * device FP32 matrix of n rows of dim values (row-major, 16-byte aligned).
 * For each row q, nbr[q*knn + j] (int32, device) receives the index of its
 * j-th nearest other row by squared Euclidean distance, and dist[q*knn + j]
 * (FP32, device) that squared distance, |x_q|^2 + |x_c|^2 - 2 x_q.x_c with
 * the dot product on FP32 matrix cores (clamped at 0).  Self is excluded;
 * ties go to the lower index; the list is in ascending order.  Needs
 * 2 <= n <= 2^30, dim a multiple of 4 in [4, 1024], 1 <= knn <= min(16, n-1).
 * Symmetrisation and edge weights are the caller's. */
int fsc_knn(fsc_context* ctx, const float* X, int64_t n, int32_t dim, int32_t knn, int32_t* nbr,
            float* dist, void* stream);

/* The symmetrised kNN graph of the rows of X (the pre-processing of the
 * real-world data in Sec. 4.2), built on the device: the neighbours of
 * fsc_knn; sigma^2 = the median of the n*knn directed squared distances (the
 * mean of the two middle values when n*knn is even); the union of the
 * directed edges, each undirected pair {a, b} weighted exp(-d / sigma^2)
 * with d the squared distance in the list of min(a, b) if that list holds the
 * pair, else in the other's (all weights 1 when sigma^2 = 0).  Output CSR on
 * the device, both directions stored, rows sorted by column: indptr (int64
 * [n+1]; indptr[n] is the number of stored entries, between n*knn and
 * 2*n*knn), indices (int32) and weights (FP32), each with room for 2*n*knn
 * entries.  Same limits as fsc_knn, and 2*n*knn < 2^31. */
int fsc_knn_graph(fsc_context* ctx, const float* X, int64_t n, int32_t dim, int32_t knn, int64_t* indptr,
                  int32_t* indices, float* weights, void* stream);

/* Adjusted Rand index (Hubert and Arabie; the accuracy score of Sec. 4.2)
 * between labelings a (values in [0, ka)) and b (values in [0, kb)) of n
 * items, written as one FP64 value to device memory `out`.  If both labelings
 * are trivial (the index's denominator is 0) the value is 1.  Labels outside
 * their range are counted in no cell (and so lower the score). */
int fsc_ari(fsc_context* ctx, const int32_t* a, const int32_t* b, int64_t n, int32_t ka,
            int32_t kb, double* out, void* stream);

/* Normalised mutual information (the second accuracy score of Sec. 4.2)
 * between labelings a (values in [0, ka)) and b (values in [0, kb)) of n
 * items, written as one FP64 value to device memory `out`:
 * I(A; B) / ((H(A) + H(B)) / 2), natural logarithms, the arithmetic-mean
 * normalisation (the paper names no other).  Only pairs with both labels in
 * range are counted (N of them).  The value is 1 when both entropies are 0 or
 * N = 0.  Needs ka*kb <= 2^22; the table and margins come from the context's
 * workspace. */
int fsc_nmi(fsc_context* ctx, const int32_t* a, const int32_t* b, int64_t n, int32_t ka,
            int32_t kb, double* out, void* stream);

/* Sets (fields > 0; slab_kb < 0 turns the slab form off) and then reports in
 * *t the sparse-product launch shape used by later calls on this context
 * (slab_kb reported as -1 when off).  t is a host pointer.  Returns FSC_E_ARG
 * for out-of-range values (tile_nnz < 64, blocks_per_cu outside [1, 16],
 * unroll not 4 or 8, slab_kb above 65536). */
int fsc_tuning_set(fsc_context* ctx, fsc_tuning* t);

/* Kernel timing with HIP events, for profiling (off by default).  While on,
 * every sparse-product launch (one PowerMethod step, Algorithm 1) queued by
 * fsc_embed / fsc_cluster on this context is bracketed by two events recorded
 * on the call's stream.  Turning it off drops unread records. */
int fsc_timing_enable(fsc_context* ctx, int on);

/* Waits for the recorded events, writes the number of timed sparse-product
 * launches and their summed duration in milliseconds (host pointers), and
 * clears the record. */
int fsc_timing_read(fsc_context* ctx, int64_t* launches, double* total_ms);

/* Human-readable text of the last error on the calling thread ("" if none). */
const char* fsc_last_error(void);

/* ABI version: (major << 16) | minor. */
int fsc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FSC_H */
