// PM with k vectors, the comparison method of Sec. 4 (Boutsidis et al.),
// which the paper describes as the power method on k vectors followed by a
// singular value decomposition.  The power steps are the plain path's with
// l = k columns; this file adds the orthonormalisation of Y = D^{1/2} Z_t
// (Z_t the embedding rows) through its Gram matrix:
//   G = Y^T Y = sum_v d_v z_v z_v^T           (FP64, over non-isolated rows)
//   G = V diag(sigma^2) V^T                    (cyclic Jacobi, FP64, one lane)
//   D^{-1/2} U = Z_t V diag(1 / sigma)         (the embedding k-means gets)
// Columns come in descending order of sigma; a column with sigma at most
// 1e-6 of the largest is set to 0 (FP32 rows cannot resolve it); each
// column's sign makes the largest-magnitude entry of its column of V
// positive (the first such entry on a tie).
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>

namespace fsc {

constexpr int kPmkBlock = 256;
constexpr int kPmkMaxGrid = 1024;

int pmk_grid(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kPmkBlock - 1) / kPmkBlock, kPmkMaxGrid)); }

// Per-block partial sums of the upper triangle of G (row-major a <= b).
template <int KD>
__global__ __launch_bounds__(kPmkBlock) void pmk_gram_kernel(const float* __restrict__ pts,
                                                             const double* __restrict__ deg, int64_t n,
                                                             double* __restrict__ partials) {
  constexpr int NT = KD * (KD + 1) / 2;
  __shared__ double red[kPmkBlock / FSC_WAVE][NT];
  double g[NT];
#pragma unroll
  for (int i = 0; i < NT; ++i) g[i] = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * kPmkBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kPmkBlock) {
    const double d = deg[v];
    if (d > 0.0) {
      float p[KD];
      rowio<float, KD>::load(pts + v * KD, p);
      int i = 0;
#pragma unroll
      for (int a = 0; a < KD; ++a) {
        const double da = d * (double)p[a];
#pragma unroll
        for (int b = a; b < KD; ++b) g[i++] += da * (double)p[b];
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
    for (int q = 0; q < kPmkBlock / FSC_WAVE; ++q) s += red[q][threadIdx.x];
    partials[(int64_t)blockIdx.x * NT + threadIdx.x] = s;
  }
}

// One block: sums the partials in block order (deterministic), then one lane
// diagonalises the leading k x k block of G and writes W = V diag(1/sigma)
// (KD x KD, row a = input column, zero outside k x k) and the singular values.
template <int KD>
__global__ __launch_bounds__(64) void pmk_finish_kernel(const double* __restrict__ partials, int grid, int k,
                                                        float* __restrict__ W, double* __restrict__ sigma) {
  constexpr int NT = KD * (KD + 1) / 2;
  __shared__ double gs[NT];
  __shared__ double G[KD][KD];
  __shared__ double V[KD][KD];
  if (threadIdx.x < NT) {
    double s = 0.0;
    for (int b = 0; b < grid; ++b) s += partials[(int64_t)b * NT + threadIdx.x];
    gs[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int a = 0, i = 0; a < KD; ++a)
    for (int b = a; b < KD; ++b, ++i) G[a][b] = G[b][a] = gs[i];
  for (int a = 0; a < KD; ++a)
    for (int b = 0; b < KD; ++b) V[a][b] = a == b ? 1.0 : 0.0;
  // cyclic Jacobi (Golub and Van Loan, the symmetric Schur rotation)
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int p = 0; p < k; ++p)
      for (int q = 0; q < k; ++q) {
        const double x = G[p][q] * G[p][q];
        tot += x;
        if (p != q) off += x;
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < k - 1; ++p)
      for (int q = p + 1; q < k; ++q) {
        const double apq = G[p][q];
        if (apq == 0.0) continue;
        const double tau = (G[q][q] - G[p][p]) / (2.0 * apq);
        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(tau * tau + 1.0));
        const double c = 1.0 / sqrt(tt * tt + 1.0), s = tt * c;
        for (int r = 0; r < k; ++r) {
          const double gp = G[r][p], gq = G[r][q];
          G[r][p] = c * gp - s * gq;
          G[r][q] = s * gp + c * gq;
        }
        for (int r = 0; r < k; ++r) {
          const double gp = G[p][r], gq = G[q][r];
          G[p][r] = c * gp - s * gq;
          G[q][r] = s * gp + c * gq;
        }
        for (int r = 0; r < k; ++r) {
          const double vp = V[r][p], vq = V[r][q];
          V[r][p] = c * vp - s * vq;
          V[r][q] = s * vp + c * vq;
        }
      }
  }
  // descending order of eigenvalue, ties to the lower index
  int order[KD];
  bool used[KD];
  for (int j = 0; j < KD; ++j) used[j] = false;
  double lmax = 0.0;
  for (int j = 0; j < k; ++j) {
    int best = -1;
    for (int i = 0; i < k; ++i)
      if (!used[i] && (best < 0 || G[i][i] > G[best][best])) best = i;
    used[best] = true;
    order[j] = best;
    if (j == 0) lmax = fmax(G[best][best], 0.0);
  }
  for (int a = 0; a < KD; ++a)
    for (int j = 0; j < KD; ++j) W[a * KD + j] = 0.f;
  for (int j = 0; j < k; ++j) {
    const int src = order[j];
    const double lam = fmax(G[src][src], 0.0);
    const double sv = sqrt(lam);
    if (sigma) sigma[j] = sv;
    if (!(lmax > 0.0 && lam > 1e-12 * lmax)) continue;  // sigma <= 1e-6 sigma_max
    int rmax = 0;
    for (int r = 1; r < k; ++r)
      if (fabs(V[r][src]) > fabs(V[rmax][src])) rmax = r;
    const double sg = V[rmax][src] < 0.0 ? -1.0 : 1.0;
    for (int a = 0; a < k; ++a) W[a * KD + j] = (float)(sg * V[a][src] / sv);
  }
}

// p_v <- p_v W in place; the first k values of each row also go to emb.
template <int KD>
__global__ __launch_bounds__(kPmkBlock) void pmk_apply_kernel(float* __restrict__ pts, int64_t n, int k,
                                                              const float* __restrict__ W, float* __restrict__ emb) {
  __shared__ float w[KD * KD];
  for (int i = threadIdx.x; i < KD * KD; i += kPmkBlock) w[i] = W[i];
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * kPmkBlock + threadIdx.x; v < n; v += (int64_t)gridDim.x * kPmkBlock) {
    float p[KD], o[KD];
    rowio<float, KD>::load(pts + v * KD, p);
#pragma unroll
    for (int j = 0; j < KD; ++j) {
      float acc = 0.f;
#pragma unroll
      for (int a = 0; a < KD; ++a) acc = fmaf(p[a], w[a * KD + j], acc);
      o[j] = acc;
    }
    rowio<float, KD>::store(pts + v * KD, o);
    if (emb)
      for (int j = 0; j < k; ++j) emb[v * k + j] = o[j];
  }
}

size_t pmk_workspace_bytes(int64_t n, int KD) {
  return align_up((size_t)pmk_grid(n) * KD * (KD + 1) / 2 * 8) + align_up((size_t)KD * KD * 4);
}

int pmk_run(const EmbedIO* io, float* pts, int KD, int k, double* partials, float* W, double* sigma, float* emb,
            hipStream_t s) {
  const int64_t n = io->g->n;
  const int grid = pmk_grid(n);
  const int agrid = (int)std::max<int64_t>(1, std::min<int64_t>((n + kPmkBlock - 1) / kPmkBlock, 8192));
  if (KD == 4) {
    hipLaunchKernelGGL(pmk_gram_kernel<4>, dim3(grid), dim3(kPmkBlock), 0, s, pts, io->deg, n, partials);
    hipLaunchKernelGGL(pmk_finish_kernel<4>, dim3(1), dim3(64), 0, s, partials, grid, k, W, sigma);
    hipLaunchKernelGGL(pmk_apply_kernel<4>, dim3(agrid), dim3(kPmkBlock), 0, s, pts, n, k, W, emb);
  } else if (KD == 8) {
    hipLaunchKernelGGL(pmk_gram_kernel<8>, dim3(grid), dim3(kPmkBlock), 0, s, pts, io->deg, n, partials);
    hipLaunchKernelGGL(pmk_finish_kernel<8>, dim3(1), dim3(64), 0, s, partials, grid, k, W, sigma);
    hipLaunchKernelGGL(pmk_apply_kernel<8>, dim3(agrid), dim3(kPmkBlock), 0, s, pts, n, k, W, emb);
  } else {
    return fail(FSC_E_ARG, "point width must be 4 or 8");
  }
  return check_hip(hipGetLastError(), "pmk launch");
}

// ---- subspace iteration for the leading eigenvectors of M ----
// After each cycle of power steps the orthonormalised block restarts the
// next: x0 = D^{1/2} (Z_t W) = U (y-space), in FP64 n x m.
__global__ __launch_bounds__(kPmkBlock) void eig_restart_kernel(const float* __restrict__ pts,
                                                                const double* __restrict__ deg, int64_t n,
                                                                int KD, int m, double* __restrict__ x0) {
  for (int64_t i = (int64_t)blockIdx.x * kPmkBlock + threadIdx.x; i < n * m; i += (int64_t)gridDim.x * kPmkBlock) {
    const int64_t v = i / m;
    const int j = (int)(i - v * m);
    const double d = deg[v];
    x0[i] = d > 0.0 ? sqrt(d) * (double)pts[v * KD + j] : 0.0;
  }
}

// Eigenvalue estimates from the last cycle: its start block U is
// orthonormal, so the singular values of M^s U tend to gamma_j^s.
__global__ void eig_gamma_kernel(const double* __restrict__ sigma, int m, int steps, double* __restrict__ gamma) {
  if (threadIdx.x == 0 && blockIdx.x == 0)
    for (int j = 0; j < m; ++j) gamma[j] = steps > 0 && sigma[j] > 0.0 ? pow(sigma[j], 1.0 / steps) : 0.0;
}

int eig_restart_run(const float* pts, const double* deg, int64_t n, int KD, int m, double* x0, hipStream_t s) {
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n * m + kPmkBlock - 1) / kPmkBlock, 8192));
  hipLaunchKernelGGL(eig_restart_kernel, dim3(grid), dim3(kPmkBlock), 0, s, pts, deg, n, KD, m, x0);
  return check_hip(hipGetLastError(), "eig restart launch");
}

int eig_gamma_run(const double* sigma, int m, int steps, double* gamma, hipStream_t s) {
  hipLaunchKernelGGL(eig_gamma_kernel, dim3(1), dim3(64), 0, s, sigma, m, steps, gamma);
  return check_hip(hipGetLastError(), "eig gamma launch");
}

}  // namespace fsc
