// Exact k-nearest-neighbour search, the pre-processing Sec. 4.2 applies to
// its real-world data (each point joined to its 10 nearest neighbours).
// Squared Euclidean distances d(q, c) = |q|^2 + |c|^2 - 2 q.c with the dot
// products on the FP32 matrix cores; each block keeps its queries in LDS and
// streams every candidate through, so the result is exact up to FP32
// rounding.  Self is excluded; ties go to the lower index.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>

namespace fsc {

typedef float knn_f4 __attribute__((ext_vector_type(4)));

constexpr int kKnnNW = 4;         // waves per block
constexpr int kKnnQ = 16 * kKnnNW;  // queries per block
constexpr int kKnnC = 64;         // candidates per tile
constexpr int kKnnList = 16;      // entries of each partial list
constexpr int kKnnPerPart = 16;   // candidates of a tile per partial list
constexpr int kKnnMaxSplit = 16;  // candidate ranges per query group

// |x_v|^2 in FP64, one wave per row, rounded to FP32.
__global__ __launch_bounds__(256) void knn_norms_kernel(const float* __restrict__ X, int64_t n, int dim,
                                                        float* __restrict__ nrm) {
  const int lane = threadIdx.x & 63;
  for (int64_t v = ((int64_t)blockIdx.x * 256 + threadIdx.x) / 64; v < n; v += (int64_t)gridDim.x * 4) {
    double s = 0.0;
    for (int c = lane; c < dim; c += 64) {
      const double x = X[v * dim + c];
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) nrm[v] = (float)s;
  }
}

// (distance, index) order: ties go to the lower index.
__device__ __forceinline__ bool knn_less(float d1, int i1, float d2, int i2) {
  return d1 < d2 || (d1 == d2 && i1 < i2);
}

// Lanes l and l ^ s hold sorted lists (d, i) of kKnnList entries; both end
// with the kKnnList smallest entries of the two lists, sorted.  The
// element-wise minimum of one list and the other reversed is a bitonic
// sequence holding those entries; a bitonic merge sorts it.
__device__ __forceinline__ void knn_merge_xor(float (&d)[kKnnList], int (&ix)[kKnnList], int s) {
  float od[kKnnList];
  int oi[kKnnList];
#pragma unroll
  for (int j = 0; j < kKnnList; ++j) {
    od[j] = __shfl_xor(d[j], s, FSC_WAVE);
    oi[j] = __shfl_xor(ix[j], s, FSC_WAVE);
  }
#pragma unroll
  for (int j = 0; j < kKnnList; ++j) {
    const float e = od[kKnnList - 1 - j];
    const int ei = oi[kKnnList - 1 - j];
    if (knn_less(e, ei, d[j], ix[j])) {
      d[j] = e;
      ix[j] = ei;
    }
  }
#pragma unroll
  for (int h = kKnnList / 2; h >= 1; h >>= 1)
#pragma unroll
    for (int j = 0; j < kKnnList; ++j)
      if ((j & h) == 0 && knn_less(d[j + h], ix[j + h], d[j], ix[j])) {
        const float td = d[j];
        d[j] = d[j + h];
        d[j + h] = td;
        const int ti = ix[j];
        ix[j] = ix[j + h];
        ix[j + h] = ti;
      }
}

// Block (b, s) takes queries 64b .. 64b + 63 and streams the candidates of
// range s (one of S contiguous ranges of tiles) past them, so that the grid
// has several blocks per resident slot and no long tail.  Both operands go
// through LDS in chunks of 64 dimensions: the 64 queries' chunk and a tile of
// C = 64 candidates' chunk, loaded with coalesced 16-byte loads (the next
// chunk's loads are in flight while the current one is used).  Nothing stays
// resident, so a block needs 35 KB of LDS and four blocks share a CU.  Wave w
// computes the dot products of queries 16 w + 0..15 with all C candidates of
// the tile (four 16 x 16 accumulators): lane (col, kk) supplies dimensions
// k + 4 kk + s (s = 0..3) of query col and of candidate col of each group,
// and receives the products of queries 4 kk + r with candidate col.  When a
// tile's last chunk is done its products go through LDS (over the candidate
// buffer) to the selection: thread t keeps the 16 nearest of the candidates
// 16 (t % P) + 0..15 of every tile for query t / P (P = 4 partial lists per
// query, held by neighbouring lanes), sorted by (distance, index).  At the
// end the P lanes of a query merge their lists pairwise (two exchange
// rounds) and write the range's 16 nearest to pd/pi[s][query][16] (sorted;
// missing entries are (inf, INT_MAX)).
__global__ __launch_bounds__(64 * kKnnNW, 4) void knn_kernel(const float* __restrict__ X, const float* __restrict__ nrm,
                                                          int n, int dim, float* __restrict__ pd,
                                                          int32_t* __restrict__ pi) {
  constexpr int NT = 64 * kKnnNW;      // threads
  constexpr int C = kKnnC;             // candidates per tile
  constexpr int LDC = 64 + 4;          // padded row of a chunk
  constexpr int P = NT / kKnnQ;        // partial lists per query
  constexpr int CP = C * 16 / NT;      // 16-byte pieces of the candidate chunk per thread
  constexpr int QP = kKnnQ * 16 / NT;  // and of the query chunk
  static_assert(kKnnQ == 16 * kKnnNW && C == 64, "a wave takes 16 queries and the whole tile");
  static_assert(C == P * kKnnPerPart, "each tile candidate belongs to one list");
  static_assert(CP * NT == C * 16 && QP * NT == kKnnQ * 16, "whole pieces per thread");
  static_assert(kKnnQ * (C + 1) <= C * LDC, "the tile's products fit the candidate buffer");
  static_assert(P <= FSC_WAVE && (FSC_WAVE % P) == 0, "a query's lists lie in one wave");
  __shared__ __align__(16) float qs[kKnnQ * LDC];
  __shared__ __align__(16) float cs[C * LDC];
  float(*dt)[C + 1] = reinterpret_cast<float(*)[C + 1]>(cs);  // products of a finished tile
  const int q0 = blockIdx.x * kKnnQ;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, kk = lane >> 4;
  const int qw = wave * 16;
  const int tq = threadIdx.x / P, te = threadIdx.x % P;
  const int gq = q0 + tq;
  const float qn = gq < n ? nrm[gq] : 0.f;
  float bd[kKnnList];
  int bi[kKnnList];
#pragma unroll
  for (int j = 0; j < kKnnList; ++j) {
    bd[j] = __builtin_inff();
    bi[j] = INT_MAX;
  }
  const float* qrow = qs + (qw + col) * LDC + 4 * kk;
  const float* crow = cs + col * LDC + 4 * kk;   // candidate group g at crow + 16 g LDC
  const knn_f4 zero = {0.f, 0.f, 0.f, 0.f};

  // chunk ci covers candidates C (ci / nkc) + 0..C-1, dimensions 64 (ci % nkc) + 0..63;
  // thread t loads candidate pieces t + NT i (i < CP) and query pieces
  // t + NT i (i < QP): row piece / 16, dims 4 (piece % 16)
  const int nkc = (dim + 63) / 64;
  const int64_t tiles = (n + C - 1) / C;
  const int64_t S = gridDim.y, sp = blockIdx.y;
  const int64_t ci_begin = (sp * tiles / S) * nkc, ci_end = ((sp + 1) * tiles / S) * nkc;
  knn_f4 pre[CP], qpre[QP];
  auto load = [&](int64_t ci) {
    const int c0 = (int)(ci / nkc) * C, kc = (int)(ci % nkc) * 64;
#pragma unroll
    for (int i = 0; i < CP; ++i) {
      const int piece = threadIdx.x + NT * i;
      const int r = c0 + (piece >> 4), d = kc + 4 * (piece & 15);
      const bool ok = r < n && d < dim;
      // the address stays inside X even where the load is not wanted
      const knn_f4 v = *reinterpret_cast<const knn_f4*>(X + (int64_t)(ok ? r : 0) * dim + (ok ? d : 0));
      pre[i] = ok ? v : zero;
    }
#pragma unroll
    for (int i = 0; i < QP; ++i) {
      const int piece = threadIdx.x + NT * i;
      const int r = q0 + (piece >> 4), d = kc + 4 * (piece & 15);
      const bool ok = r < n && d < dim;
      const knn_f4 v = *reinterpret_cast<const knn_f4*>(X + (int64_t)(ok ? r : 0) * dim + (ok ? d : 0));
      qpre[i] = ok ? v : zero;
    }
  };
  if (ci_begin < ci_end) load(ci_begin);
  knn_f4 acc[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) acc[g] = zero;
  for (int64_t ci = ci_begin; ci < ci_end; ++ci) {
    const int c0 = (int)(ci / nkc) * C, kc = (int)(ci % nkc) * 64;
    __syncthreads();  // every wave is done with the previous chunk, or with the products
#pragma unroll
    for (int i = 0; i < CP; ++i) {
      const int piece = threadIdx.x + NT * i;
      *reinterpret_cast<knn_f4*>(cs + (piece >> 4) * LDC + 4 * (piece & 15)) = pre[i];
    }
#pragma unroll
    for (int i = 0; i < QP; ++i) {
      const int piece = threadIdx.x + NT * i;
      *reinterpret_cast<knn_f4*>(qs + (piece >> 4) * LDC + 4 * (piece & 15)) = qpre[i];
    }
    __syncthreads();
    if (ci + 1 < ci_end) load(ci + 1);
    if (kc == 0) {
#pragma unroll
      for (int g = 0; g < 4; ++g) acc[g] = zero;
    }
#pragma unroll
    for (int k = 0; k < 64; k += 16) {
      if (kc + k < dim) {
        const knn_f4 a = *reinterpret_cast<const knn_f4*>(qrow + k);
        knn_f4 b[4];
#pragma unroll
        for (int g = 0; g < 4; ++g) b[g] = *reinterpret_cast<const knn_f4*>(crow + 16 * g * LDC + k);
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
          for (int g = 0; g < 4; ++g) acc[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s4], b[g][s4], acc[g], 0, 0, 0);
      }
    }
    if (kc + 64 < dim) continue;  // more dimensions of this tile to come
    __syncthreads();  // the candidate buffer is read by every wave before it takes the products
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) dt[qw + 4 * kk + r][16 * g + col] = acc[g][r];
    __syncthreads();
#pragma unroll 4
    for (int j = 0; j < kKnnPerPart; ++j) {
      const int cl = te * kKnnPerPart + j;
      const int c = c0 + cl;
      if (c < n && c != gq) {
        const float d = fmaxf(qn + nrm[c] - 2.f * dt[tq][cl], 0.f);
        if (d < bd[kKnnList - 1]) {
          bd[kKnnList - 1] = d;
          bi[kKnnList - 1] = c;
#pragma unroll
          for (int p = kKnnList - 1; p > 0; --p) {
            if (bd[p] < bd[p - 1]) {
              const float td = bd[p];
              bd[p] = bd[p - 1];
              bd[p - 1] = td;
              const int ti = bi[p];
              bi[p] = bi[p - 1];
              bi[p - 1] = ti;
            }
          }
        }
      }
    }
  }
  // the P lanes of a query merge their lists
#pragma unroll
  for (int sft = 1; sft < P; sft <<= 1) knn_merge_xor(bd, bi, sft);
  if (te == 0 && gq < n) {
    const int64_t base = (sp * n + gq) * kKnnList;
#pragma unroll
    for (int o = 0; o < kKnnList; ++o) {
      pd[base + o] = bd[o];
      pi[base + o] = bi[o];
    }
  }
}

// The knn nearest of each query from the S sorted range lists.
__global__ __launch_bounds__(256) void knn_merge_kernel(const float* __restrict__ pd, const int32_t* __restrict__ pi,
                                                        int64_t n, int S, int knn, int32_t* __restrict__ nbr,
                                                        float* __restrict__ dist) {
  for (int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (int64_t)gridDim.x * 256) {
    int head[kKnnMaxSplit];
    for (int s = 0; s < S; ++s) head[s] = 0;
    for (int o = 0; o < knn; ++o) {
      int be = 0;
      float bdv = __builtin_inff();
      int biv = INT_MAX;
      for (int s = 0; s < S; ++s) {
        if (head[s] >= kKnnList) continue;
        const int64_t e = ((int64_t)s * n + q) * kKnnList + head[s];
        if (knn_less(pd[e], pi[e], bdv, biv)) {
          be = s;
          bdv = pd[e];
          biv = pi[e];
        }
      }
      head[be] += 1;
      nbr[q * knn + o] = biv;
      dist[q * knn + o] = bdv;
    }
  }
}

// Candidate ranges per query group: about 8 blocks per resident slot (four
// per CU), at most one range per tile and kKnnMaxSplit in all.
static int knn_splits(int64_t n, int num_cu) {
  const int64_t groups = (n + kKnnQ - 1) / kKnnQ;
  const int64_t tiles = (n + kKnnC - 1) / kKnnC;
  const int64_t slots = (int64_t)std::max(num_cu, 1) * 4;
  int64_t S = (8 * slots + groups - 1) / groups;
  S = std::min<int64_t>(S, std::min<int64_t>(tiles, kKnnMaxSplit));
  return (int)std::max<int64_t>(1, S);
}

size_t knn_workspace_bytes(int64_t n, int num_cu) {
  const int64_t S = knn_splits(n, num_cu);
  return align_up((size_t)n * 4) + 2 * align_up((size_t)(S * n * kKnnList) * 4) + 1024;
}

int knn_run(Arena* a, const float* X, int64_t n, int dim, int knn, int num_cu, int32_t* nbr, float* dist,
            hipStream_t s) {
  const int S = knn_splits(n, num_cu);
  float* norms = a->take<float>((size_t)n);
  float* pd = a->take<float>((size_t)(S * n * kKnnList));
  int32_t* pi = a->take<int32_t>((size_t)(S * n * kKnnList));
  if (a->used > a->size) return fail(FSC_E_NOMEM, "knn workspace too small");
  const int nb = (int)std::min<int64_t>((n + 3) / 4, 8192);
  hipLaunchKernelGGL(knn_norms_kernel, dim3(nb), dim3(256), 0, s, X, n, dim, norms);
  const int groups = (int)((n + kKnnQ - 1) / kKnnQ);
  hipLaunchKernelGGL(knn_kernel, dim3(groups, S), dim3(64 * kKnnNW), 0, s, X, norms, (int)n, dim, pd, pi);
  const int mb = (int)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(knn_merge_kernel, dim3(mb), dim3(256), 0, s, pd, pi, n, S, knn, nbr, dist);
  return check_hip(hipGetLastError(), "knn launch");
}

// ---- the symmetrised kNN graph ----
// Directed edge e = u * knn + j (u -> nbr[e]) becomes the pair key
// min * n + max.  After a stable sort of the keys, the first entry of each run
// (the lower-indexed endpoint's list, which comes first in e) emits both
// directions of the pair with weight exp(-d / sigma^2); the other entries emit
// sentinels n * n, which sort after every real entry.  A second sort by
// row * n + col orders the CSR, and a binary search per row finds its start.
__global__ void kg_pair_kernel(const int32_t* __restrict__ nbr, int64_t E, int knn, int64_t n,
                               unsigned long long* __restrict__ key, int32_t* __restrict__ val) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = e / knn, v = nbr[e];
    key[e] = (unsigned long long)(u < v ? u * n + v : v * n + u);
    val[e] = (int32_t)e;
  }
}

// sigma^2: the median of the E sorted directed distances (the mean of the two
// middle values when E is even).
__global__ void kg_median_kernel(const float* __restrict__ sorted, int64_t E, float* __restrict__ sigma2) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t m = E / 2;
    *sigma2 = (E % 2) ? sorted[m] : 0.5f * (sorted[m - 1] + sorted[m]);
  }
}

__global__ void kg_emit_kernel(const unsigned long long* __restrict__ key_s, const int32_t* __restrict__ val_s,
                               const float* __restrict__ dist, const float* __restrict__ sigma2, int64_t E,
                               int64_t n, unsigned long long* __restrict__ key2, float* __restrict__ w2) {
  const float s2 = *sigma2;
  const unsigned long long sentinel = (unsigned long long)n * (unsigned long long)n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = key_s[i];
    if (i == 0 || key_s[i - 1] != k) {
      const float d = dist[val_s[i]];
      const float w = s2 > 0.f ? expf(-d / s2) : 1.f;
      const unsigned long long a = k / (unsigned long long)n, b = k % (unsigned long long)n;
      key2[2 * i] = a * (unsigned long long)n + b;
      key2[2 * i + 1] = b * (unsigned long long)n + a;
      w2[2 * i] = w;
      w2[2 * i + 1] = w;
    } else {
      key2[2 * i] = sentinel;
      key2[2 * i + 1] = sentinel;
      w2[2 * i] = 0.f;
      w2[2 * i + 1] = 0.f;
    }
  }
}

// indptr[r] = first sorted entry with key >= r * n (r = 0..n; indptr[n] = nnz);
// the real entries' columns and weights.
__global__ void kg_csr_kernel(const unsigned long long* __restrict__ key2_s, const float* __restrict__ w2_s,
                              int64_t M, int64_t n, int64_t* __restrict__ indptr, int32_t* __restrict__ indices,
                              float* __restrict__ weights) {
  const unsigned long long nn = (unsigned long long)n;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n; r += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long target = (unsigned long long)r * nn;
    int64_t lo = 0, hi = M;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (key2_s[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    indptr[r] = lo;
  }
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = key2_s[i];
    if (k < nn * nn) {
      indices[i] = (int32_t)(k % nn);
      weights[i] = w2_s[i];
    }
  }
}

static int key_bits(unsigned long long maxkey) {
  int b = 1;
  while (b < 64 && (maxkey >> b) != 0) ++b;
  return b;
}

// Scratch of the three radix sorts, queried with the counts and key widths
// the run uses.
static size_t kg_temp_bytes(int64_t n, int knn) {
  const int64_t E = n * knn, M = 2 * E;
  const unsigned long long nn = (unsigned long long)n * (unsigned long long)n;
  size_t t1 = 0, t2 = 0, t3 = 0;
  hipcub::DeviceRadixSort::SortKeys(nullptr, t1, (const float*)nullptr, (float*)nullptr, (int)E, 0, 32);
  hipcub::DeviceRadixSort::SortPairs(nullptr, t2, (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                     (const int32_t*)nullptr, (int32_t*)nullptr, (int)E, 0, key_bits(nn - 1));
  hipcub::DeviceRadixSort::SortPairs(nullptr, t3, (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                     (const float*)nullptr, (float*)nullptr, (int)M, 0, key_bits(nn));
  return std::max(t1, std::max(t2, t3));
}

size_t knn_graph_workspace_bytes(int64_t n, int knn, int num_cu) {
  const int64_t E = n * knn, M = 2 * E;
  return knn_workspace_bytes(n, num_cu) +                             // the search
         align_up((size_t)E * 4) * 3 +                                // nbr, dist, sorted distances
         align_up((size_t)E * 8) * 2 + align_up((size_t)E * 4) * 2 +  // pair keys and edge ids, sorted
         align_up((size_t)M * 8) * 2 + align_up((size_t)M * 4) * 2 +  // CSR keys and weights, sorted
         align_up(64 * 4) + align_up(kg_temp_bytes(n, knn)) + 4096;
}

int knn_graph_run(Arena* a, const float* X, int64_t n, int dim, int knn, int num_cu, int64_t* indptr,
                  int32_t* indices, float* weights, hipStream_t s) {
  const int64_t E = n * knn, M = 2 * E;
  int32_t* nbr = a->take<int32_t>((size_t)E);
  float* dist = a->take<float>((size_t)E);
  float* dsort = a->take<float>((size_t)E);
  unsigned long long* key = a->take<unsigned long long>((size_t)E);
  unsigned long long* key_s = a->take<unsigned long long>((size_t)E);
  int32_t* val = a->take<int32_t>((size_t)E);
  int32_t* val_s = a->take<int32_t>((size_t)E);
  unsigned long long* key2 = a->take<unsigned long long>((size_t)M);
  unsigned long long* key2_s = a->take<unsigned long long>((size_t)M);
  float* w2 = a->take<float>((size_t)M);
  float* w2_s = a->take<float>((size_t)M);
  float* sigma2 = a->take<float>(64);
  size_t temp_bytes = kg_temp_bytes(n, knn);
  void* temp = a->take<char>(temp_bytes);
  if (a->used > a->size) return fail(FSC_E_NOMEM, "knn graph workspace too small");
  int rc;
  if ((rc = knn_run(a, X, n, dim, knn, num_cu, nbr, dist, s))) return rc;
  const int blocks = (int)std::min<int64_t>((M + 255) / 256, 8192);
  const unsigned long long nn = (unsigned long long)n * (unsigned long long)n;
  if ((rc = check_hip(hipcub::DeviceRadixSort::SortKeys(temp, temp_bytes, dist, dsort, (int)E, 0, 32, s),
                      "sort distances")))
    return rc;
  hipLaunchKernelGGL(kg_median_kernel, dim3(1), dim3(64), 0, s, dsort, E, sigma2);
  hipLaunchKernelGGL(kg_pair_kernel, dim3(blocks), dim3(256), 0, s, nbr, E, knn, n, key, val);
  if ((rc = check_hip(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, key, key_s, val, val_s, (int)E, 0,
                                                         key_bits(nn - 1), s),
                      "sort pairs")))
    return rc;
  hipLaunchKernelGGL(kg_emit_kernel, dim3(blocks), dim3(256), 0, s, key_s, val_s, dist, sigma2, E, n, key2, w2);
  if ((rc = check_hip(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, key2, key2_s, w2, w2_s, (int)M, 0,
                                                         key_bits(nn), s),
                      "sort entries")))
    return rc;
  const int cblocks = (int)std::min<int64_t>((std::max<int64_t>(M, n + 1) + 255) / 256, 8192);
  hipLaunchKernelGGL(kg_csr_kernel, dim3(cblocks), dim3(256), 0, s, key2_s, w2_s, M, n, indptr, indices, weights);
  return check_hip(hipGetLastError(), "knn graph launch");
}

}  // namespace fsc
