// PM with k vectors, the comparison method of Sec. 4 (k mutually orthogonal
// vectors computed with the power method; the algorithm of Boutsidis et al.,
// whose singular value decomposition Sec. 1.1 mentions), and the eigenvector
// baselines of Sec. 4, both as orthogonal iteration on the plain path's power
// steps.  The block is orthonormalised after the start block and after every
// step.  With Y = D^{1/2} Z (Z the z-space rows the step kernels keep):
//   G = Y^T Y = sum_v d_v z_v z_v^T           (FP64, non-isolated rows)
//   G = V diag(sigma^2) V^T                    (cyclic Jacobi, FP64)
//   Z <- Z V diag(1 / sigma)                   (D^{1/2} Z orthonormal)
// so that D^{1/2} Z holds the left singular vectors of Y in descending order
// of sigma.  The step is linear, so each step acts on the orthonormal block
// of the last one, and every direction stays resolved at any number of
// steps.  A direction whose sigma within one step is at most 1e-6 of the
// largest is set to 0: the Gram matrix of stored rows cannot resolve it.
// After the last step each column's sign makes its largest-magnitude entry
// of D^{1/2} Z positive (the first such row on a tie).
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>

namespace fsc {

constexpr int kOrthoBlock = 256;
constexpr int kOrthoMaxGrid = 1024;

int ortho_grid(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kOrthoBlock - 1) / kOrthoBlock, kOrthoMaxGrid));
}

// Per-block partial sums of the upper triangle of G (row-major a <= b).
template <typename S, int LH>
__global__ __launch_bounds__(kOrthoBlock) void ortho_gram_kernel(const S* __restrict__ z,
                                                                 const double* __restrict__ deg, int64_t n,
                                                                 double* __restrict__ partials) {
  using A = typename elem<S>::acc;
  constexpr int NT = LH * (LH + 1) / 2;
  __shared__ double red[kOrthoBlock / FSC_WAVE][NT];
  double g[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) g[i] = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kOrthoBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kOrthoBlock) {
    const double d = deg[v];
    if (d > 0.0) {
      A p[LH];
      rowio<S, LH>::load(z + v * LH, p);
      int i = 0;
#pragma unroll
      for (int a = 0; a < LH; ++a) {
        const double da = d * (double)p[a];
#pragma unroll
        for (int b = a; b < LH; ++b) g[i++] += da * (double)p[b];
      }
    }
  }
  const int w = threadIdx.x / FSC_WAVE;
#pragma unroll
  for (int i = 0; i < NT; ++i) {
    const double s = wave_sum(g[i]);
    if ((threadIdx.x & (FSC_WAVE - 1)) == 0) red[w][i] = s;
  }
  __syncthreads();
  if (threadIdx.x < NT) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kOrthoBlock / FSC_WAVE; ++q) s += red[q][threadIdx.x];
    partials[(int64_t)blockIdx.x * NT + threadIdx.x] = s;
  }
}

// One block: sums the partials (each entry over the blocks in a fixed
// order), then wave 0 diagonalises the leading k x k block of G, lane
// a * LH + b holding G[a][b] and V[a][b], and lane 0 writes
// W = V diag(1/sigma) (LH x LH, row a = input column, zero outside k x k,
// columns in descending order of sigma) and, when sigma_out is given, the k
// singular values.
constexpr int kOrthoFinish = 256;

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int LH>
__global__ __launch_bounds__(kOrthoFinish) void ortho_finish_kernel(const double* __restrict__ partials, int grid,
                                                                    int k, double* __restrict__ W,
                                                                    double* __restrict__ sigma_out) {
  constexpr int NT = LH * (LH + 1) / 2;
  static_assert(LH * LH <= FSC_WAVE, "one lane per element of G");
  __shared__ double red[kOrthoFinish / FSC_WAVE];
  __shared__ double gs[NT];
  __shared__ double G[LH * LH];
  __shared__ double V[LH * LH];
  double acc[NT];
#pragma unroll
  for (int e = 0; e < NT; ++e) acc[e] = 0.0;
  for (int b = threadIdx.x; b < grid; b += kOrthoFinish)
#pragma unroll
    for (int e = 0; e < NT; ++e) acc[e] += partials[(int64_t)b * NT + e];
#pragma unroll
  for (int e = 0; e < NT; ++e) {
    const double t = block_sum<kOrthoFinish>(acc[e], red);
    if (threadIdx.x == 0) gs[e] = t;
  }
  __syncthreads();
  if (threadIdx.x >= FSC_WAVE) return;
  const int lane = threadIdx.x;
  const bool own = lane < LH * LH;
  const int r = lane / LH, c = lane % LH;
  if (own) {
    const int lo = min(r, c), hi = max(r, c);
    G[lane] = gs[lo * LH - lo * (lo - 1) / 2 + (hi - lo)];
    V[lane] = r == c ? 1.0 : 0.0;
  }
  wave_sync_lds();
  // cyclic Jacobi (Golub and Van Loan, the symmetric Schur rotation); a
  // block orthonormalised one step earlier gives a nearly diagonal G after
  // the first few steps, which takes one or two sweeps
  const bool inner = own && r < k && c < k;
  for (int sweep = 0; sweep < 64; ++sweep) {
    const double x = inner ? G[lane] * G[lane] : 0.0;
    const double tot = wave_sum(x), off = wave_sum(r != c ? x : 0.0);
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = G[p * LH + q];
        if (apq == 0.0) continue;
        const double tau = (G[q * LH + q] - G[p * LH + p]) / (2.0 * apq);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(tau * tau + 1.0));
        const double cs = 1.0 / sqrt(tt * tt + 1.0), sn = tt * cs;
        // columns p and q of G, then rows p and q, then columns p and q of V
        double up = 0.0, uq = 0.0;
        if (own) {
          up = G[r * LH + p];
          uq = G[r * LH + q];
        }
        wave_sync_lds();
        if (own && r < k && (c == p || c == q)) G[lane] = c == p ? cs * up - sn * uq : sn * up + cs * uq;
        wave_sync_lds();
        if (own) {
          up = G[p * LH + c];
          uq = G[q * LH + c];
        }
        wave_sync_lds();
        if (own && c < k && (r == p || r == q)) G[lane] = r == p ? cs * up - sn * uq : sn * up + cs * uq;
        if (own) {
          up = V[r * LH + p];
          uq = V[r * LH + q];
        }
        wave_sync_lds();
        if (own && r < k && (c == p || c == q)) V[lane] = c == p ? cs * up - sn * uq : sn * up + cs * uq;
        wave_sync_lds();
      }
  }
  if (lane != 0) return;
  // descending order of eigenvalue, ties to the lower index
  int order[LH];
  bool used[LH];
  for (int j = 0; j < LH; ++j) used[j] = false;
  double lmax = 0.0;
  for (int j = 0; j < k; ++j) {
    int best = -1;
    for (int i = 0; i < k; ++i)
      if (!used[i] && (best < 0 || G[i * LH + i] > G[best * LH + best])) best = i;
    used[best] = true;
    order[j] = best;
    if (j == 0) lmax = fmax(G[best * LH + best], 0.0);
  }
  for (int a = 0; a < LH; ++a)
    for (int j = 0; j < LH; ++j) W[a * LH + j] = 0.0;
  for (int j = 0; j < k; ++j) {
    const int src = order[j];
    const double lam = fmax(G[src * LH + src], 0.0);
    const double sv = sqrt(lam);
    if (sigma_out) sigma_out[j] = sv;
    if (!(lmax > 0.0 && lam > 1e-12 * lmax)) continue;  // sigma <= 1e-6 sigma_max: 0
    for (int a = 0; a < k; ++a) W[a * LH + j] = V[a * LH + src] / sv;
  }
}

// z_v <- z_v W in place (every row; isolated rows are 0 and stay 0).
template <typename S, int LH>
__global__ __launch_bounds__(kOrthoBlock) void ortho_apply_kernel(S* __restrict__ z, int64_t n,
                                                                  const double* __restrict__ W) {
  using A = typename elem<S>::acc;
  __shared__ A w[LH * LH];
  for (int i = threadIdx.x; i < LH * LH; i += kOrthoBlock) w[i] = (A)W[i];
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * kOrthoBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kOrthoBlock) {
    A p[LH], o[LH];
    rowio<S, LH>::load(z + v * LH, p);
#pragma unroll
    for (int j = 0; j < LH; ++j) {
      A acc = A(0);
#pragma unroll
      for (int a = 0; a < LH; ++a) acc = fma(p[a], w[a * LH + j], acc);
      o[j] = acc;
    }
    rowio<S, LH>::store(z + v * LH, o);
  }
}

// (|value|, row) pairs: the larger value wins, the lower row on a tie.
__device__ __forceinline__ void absmax_merge(double& m, int64_t& r, double m2, int64_t r2) {
  if (m2 > m || (m2 == m && r2 >= 0 && (r < 0 || r2 < r))) {
    m = m2;
    r = r2;
  }
}

// Per-block largest |sqrt(d_v) z_vj| of each column and its first row.
template <typename S, int LH>
__global__ __launch_bounds__(kOrthoBlock) void ortho_sign_partial_kernel(const S* __restrict__ z,
                                                                         const double* __restrict__ deg,
                                                                         int64_t n, double* __restrict__ pmax,
                                                                         int64_t* __restrict__ prow) {
  using A = typename elem<S>::acc;
  __shared__ double sm[kOrthoBlock / FSC_WAVE][LH];
  __shared__ int64_t sr[kOrthoBlock / FSC_WAVE][LH];
  double m[LH];
  int64_t r[LH];
#pragma unroll
  for (int j = 0; j < LH; ++j) {
    m[j] = -1.0;
    r[j] = -1;
  }
  for (int64_t v = (int64_t)blockIdx.x * kOrthoBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kOrthoBlock) {
    const double d = deg[v];
    if (!(d > 0.0)) continue;
    const double sd = sqrt(d);
    A p[LH];
    rowio<S, LH>::load(z + v * LH, p);
#pragma unroll
    for (int j = 0; j < LH; ++j) {
      const double q = fabs(sd * (double)p[j]);
      if (q > m[j]) {  // rows ascend within a thread: the first row keeps a tie
        m[j] = q;
        r[j] = v;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < LH; ++j) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double m2 = __shfl_xor(m[j], off, FSC_WAVE);
      const int64_t r2 = __shfl_xor(r[j], off, FSC_WAVE);
      absmax_merge(m[j], r[j], m2, r2);
    }
  }
  const int w = threadIdx.x / FSC_WAVE;
  if ((threadIdx.x & (FSC_WAVE - 1)) == 0)
#pragma unroll
    for (int j = 0; j < LH; ++j) {
      sm[w][j] = m[j];
      sr[w][j] = r[j];
    }
  __syncthreads();
  if (threadIdx.x < LH) {
    const int j = threadIdx.x;
    double bm = -1.0;
    int64_t br = -1;
    for (int q = 0; q < kOrthoBlock / FSC_WAVE; ++q) absmax_merge(bm, br, sm[q][j], sr[q][j]);
    pmax[(int64_t)blockIdx.x * LH + j] = bm;
    prow[(int64_t)blockIdx.x * LH + j] = br;
  }
}

// One block: W = diag(sign_j), sign_j = -1 when the entry at column j's
// largest-magnitude row is negative.  Column j's block maxima are merged by
// the kOrthoFinish / LH threads of its group (merging is order-free: the
// larger magnitude, then the lower row), then across the group.
template <typename S, int LH>
__global__ __launch_bounds__(kOrthoFinish) void ortho_sign_finish_kernel(const S* __restrict__ z,
                                                                         const double* __restrict__ pmax,
                                                                         const int64_t* __restrict__ prow, int grid,
                                                                         double* __restrict__ W) {
  using A = typename elem<S>::acc;
  constexpr int PER = kOrthoFinish / LH;  // threads per column
  __shared__ double sm[kOrthoFinish];
  __shared__ int64_t sr[kOrthoFinish];
  const int j = threadIdx.x / PER, i = threadIdx.x % PER;
  double bm = -1.0;
  int64_t br = -1;
  for (int b = i; b < grid; b += PER) absmax_merge(bm, br, pmax[(int64_t)b * LH + j], prow[(int64_t)b * LH + j]);
  sm[threadIdx.x] = bm;
  sr[threadIdx.x] = br;
  __syncthreads();
  if (i != 0) return;
  for (int t = 1; t < PER; ++t) absmax_merge(bm, br, sm[threadIdx.x + t], sr[threadIdx.x + t]);
  double sg = 1.0;
  if (br >= 0) {
    A p[LH];
    rowio<S, LH>::load(z + br * LH, p);
    if (p[j] < A(0)) sg = -1.0;
  }
  for (int a = 0; a < LH; ++a) W[a * LH + j] = a == j ? sg : 0.0;
}

size_t ortho_workspace_bytes(int64_t n, int LH) {
  const size_t grid = (size_t)ortho_grid(n);
  return align_up(grid * LH * (LH + 1) / 2 * 8) + align_up((size_t)LH * LH * 8) + align_up(grid * LH * 8) +
         align_up(grid * LH * 8);
}

void ortho_bind(Arena* a, int64_t n, int LH, int k, OrthoArgs* oa) {
  oa->k = k;
  oa->grid = ortho_grid(n);
  oa->partials = a->take<double>((size_t)oa->grid * LH * (LH + 1) / 2);
  oa->W = a->take<double>((size_t)LH * LH);
  oa->pmax = a->take<double>((size_t)oa->grid * LH);
  oa->prow = a->take<int64_t>((size_t)oa->grid * LH);
  oa->sigma_out = nullptr;
}

template <typename S, int LH>
static int ortho_typed(const EmbedIO* io, void* zv, bool last, hipStream_t s) {
  const OrthoArgs* oa = io->ortho;
  const int64_t n = io->g->n;
  S* z = reinterpret_cast<S*>(zv);
  const int agrid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kOrthoBlock - 1) / kOrthoBlock, 8192));
  hipLaunchKernelGGL((ortho_gram_kernel<S, LH>), dim3(oa->grid), dim3(kOrthoBlock), 0, s, z, io->deg, n,
                     oa->partials);
  hipLaunchKernelGGL(ortho_finish_kernel<LH>, dim3(1), dim3(kOrthoFinish), 0, s, oa->partials, oa->grid, oa->k, oa->W,
                     last ? oa->sigma_out : nullptr);
  hipLaunchKernelGGL((ortho_apply_kernel<S, LH>), dim3(agrid), dim3(kOrthoBlock), 0, s, z, n, oa->W);
  if (last) {
    hipLaunchKernelGGL((ortho_sign_partial_kernel<S, LH>), dim3(oa->grid), dim3(kOrthoBlock), 0, s, z, io->deg, n,
                       oa->pmax, oa->prow);
    hipLaunchKernelGGL((ortho_sign_finish_kernel<S, LH>), dim3(1), dim3(kOrthoFinish), 0, s, z, oa->pmax, oa->prow, oa->grid,
                       oa->W);
    hipLaunchKernelGGL((ortho_apply_kernel<S, LH>), dim3(agrid), dim3(kOrthoBlock), 0, s, z, n, oa->W);
  }
  return check_hip(hipGetLastError(), "orthonormalisation launch");
}

template <typename S>
static int ortho_lh(const EmbedIO* io, void* z, bool last, hipStream_t s) {
  switch (io->LH) {
    case 1: return ortho_typed<S, 1>(io, z, last, s);
    case 2: return ortho_typed<S, 2>(io, z, last, s);
    case 4: return ortho_typed<S, 4>(io, z, last, s);
    case 8: return ortho_typed<S, 8>(io, z, last, s);
  }
  return fail(FSC_E_UNSUPPORTED, "unsupported block width");
}

int ortho_run(const EmbedIO* io, void* z, bool last, hipStream_t s) {
  switch (io->vec_dtype) {
    case FSC_F64: return ortho_lh<double>(io, z, last, s);
    case FSC_F32: return ortho_lh<float>(io, z, last, s);
  }
  return fail(FSC_E_UNSUPPORTED, "orthogonal iteration takes FP32 or FP64 vectors");
}

// The first k values of each FP32 point row to an n x k array.
__global__ __launch_bounds__(kOrthoBlock) void points_cols_kernel(const float* __restrict__ pts, int64_t n, int KD,
                                                                  int k, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * kOrthoBlock + threadIdx.x; i < n * k; i += (int64_t)gridDim.x * kOrthoBlock) {
    const int64_t v = i / k;
    out[i] = pts[v * KD + (i - v * k)];
  }
}

int points_cols_run(const float* pts, int64_t n, int KD, int k, float* out, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n * k + kOrthoBlock - 1) / kOrthoBlock, 8192));
  hipLaunchKernelGGL(points_cols_kernel, dim3(grid), dim3(kOrthoBlock), 0, s, pts, n, KD, k, out);
  return check_hip(hipGetLastError(), "points_cols launch");
}

}  // namespace fsc
