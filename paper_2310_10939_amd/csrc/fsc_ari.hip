// Accuracy scores of Sec. 4.2: the adjusted Rand index (Hubert and Arabie)
// and normalised mutual information.  The contingency table is built with
// integer atomics (exact, so the result does not depend on the order of the
// updates), counted per block in LDS when it is small; each score is then
// formed in FP64 by one block.  C(x, 2) of
// integer counts below 2^26 is exact in FP64.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>

namespace fsc {

__global__ void ari_zero(unsigned long long* t, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    t[i] = 0ull;
}

__global__ void ari_count(const int32_t* __restrict__ a, const int32_t* __restrict__ b, int64_t n, int ka, int kb,
                          unsigned long long* __restrict__ table) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int x = a[i], y = b[i];
    if (x >= 0 && x < ka && y >= 0 && y < kb) atomicAdd(&table[(int64_t)x * kb + y], 1ull);
  }
}

// The same with the table first counted in LDS by each block (tables of at
// most kAriLdsCells cells): one global atomic per nonzero cell per block
// instead of one per pair.
constexpr int kAriLdsCells = 8192;

__global__ __launch_bounds__(256) void ari_count_lds(const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                                                     int64_t n, int ka, int kb,
                                                     unsigned long long* __restrict__ table) {
  __shared__ uint32_t t[kAriLdsCells];
  const int cells = ka * kb;
  for (int c = threadIdx.x; c < cells; c += 256) t[c] = 0u;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const int x = a[i], y = b[i];
    if (x >= 0 && x < ka && y >= 0 && y < kb) atomicAdd(&t[x * kb + y], 1u);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cells; c += 256) {
    const uint32_t v = t[c];
    if (v) atomicAdd(&table[c], (unsigned long long)v);
  }
}

__device__ __forceinline__ double comb2(double x) { return x * (x - 1.0) * 0.5; }

__global__ __launch_bounds__(256) void ari_finish(const unsigned long long* __restrict__ table, int64_t n, int ka,
                                                  int kb, double* __restrict__ out) {
  __shared__ double red[4];
  double sij = 0.0, sa = 0.0, sb = 0.0;
  for (int64_t c = threadIdx.x; c < (int64_t)ka * kb; c += blockDim.x) sij += comb2((double)table[c]);
  for (int x = threadIdx.x; x < ka; x += blockDim.x) {
    double row = 0.0;
    for (int y = 0; y < kb; ++y) row += (double)table[(int64_t)x * kb + y];
    sa += comb2(row);
  }
  for (int y = threadIdx.x; y < kb; y += blockDim.x) {
    double colsum = 0.0;
    for (int x = 0; x < ka; ++x) colsum += (double)table[(int64_t)x * kb + y];
    sb += comb2(colsum);
  }
  sij = block_sum<256>(sij, red);
  sa = block_sum<256>(sa, red);
  sb = block_sum<256>(sb, red);
  if (threadIdx.x == 0) {
    const double total = comb2((double)n);
    const double expected = total > 0.0 ? sa * sb / total : 0.0;
    const double denom = 0.5 * (sa + sb) - expected;
    *out = denom == 0.0 ? 1.0 : (sij - expected) / denom;
  }
}

// NMI = I(A; B) / ((H(A) + H(B)) / 2) with natural logarithms, over the N
// pairs whose labels are both in range.  The block first writes the table's
// row and column sums to `margin` (ka + kb doubles), then sums the entropies
// and the information.  Both entropies 0 (or N = 0) gives 1; I is clipped at
// 0 against rounding.
__global__ __launch_bounds__(256) void nmi_finish(const unsigned long long* __restrict__ table, int ka, int kb,
                                                  double* __restrict__ margin, double* __restrict__ out) {
  __shared__ double red[4];
  double* ra = margin;
  double* cb = margin + ka;
  double cnt = 0.0;
  for (int x = threadIdx.x; x < ka; x += blockDim.x) {
    double row = 0.0;
    for (int y = 0; y < kb; ++y) row += (double)table[(int64_t)x * kb + y];
    ra[x] = row;
    cnt += row;
  }
  for (int y = threadIdx.x; y < kb; y += blockDim.x) {
    double colsum = 0.0;
    for (int x = 0; x < ka; ++x) colsum += (double)table[(int64_t)x * kb + y];
    cb[y] = colsum;
  }
  const double N = block_sum<256>(cnt, red);  // ends in a barrier: the margins are visible
  if (N == 0.0) {
    if (threadIdx.x == 0) *out = 1.0;
    return;
  }
  const double logN = log(N);
  double ha = 0.0, hb = 0.0, mi = 0.0;
  for (int x = threadIdx.x; x < ka; x += blockDim.x)
    if (ra[x] > 0.0) ha -= (ra[x] / N) * (log(ra[x]) - logN);
  for (int y = threadIdx.x; y < kb; y += blockDim.x)
    if (cb[y] > 0.0) hb -= (cb[y] / N) * (log(cb[y]) - logN);
  for (int64_t c = threadIdx.x; c < (int64_t)ka * kb; c += blockDim.x) {
    const double nij = (double)table[c];
    if (nij > 0.0) {
      const int x = (int)(c / kb), y = (int)(c % kb);
      mi += (nij / N) * (log(nij) + logN - log(ra[x]) - log(cb[y]));
    }
  }
  ha = block_sum<256>(ha, red);
  hb = block_sum<256>(hb, red);
  mi = block_sum<256>(mi, red);
  if (threadIdx.x == 0) {
    const double h = ha + hb;
    *out = h == 0.0 ? 1.0 : fmax(mi, 0.0) / (0.5 * h);
  }
}

static void contingency(const int32_t* a, const int32_t* b, int64_t n, int ka, int kb, unsigned long long* table,
                        hipStream_t s) {
  const int64_t cells = (int64_t)ka * kb;
  hipLaunchKernelGGL(ari_zero, dim3((int)std::min<int64_t>((cells + 255) / 256, 4096)), dim3(256), 0, s, table, cells);
  if (n > 0 && cells <= kAriLdsCells)
    hipLaunchKernelGGL(ari_count_lds, dim3((int)std::min<int64_t>((n + 255) / 256, 1024)), dim3(256), 0, s, a, b, n,
                       ka, kb, table);
  else if (n > 0)
    hipLaunchKernelGGL(ari_count, dim3((int)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s, a, b, n, ka,
                       kb, table);
}

int ari_run(Context*, const int32_t* a, const int32_t* b, int64_t n, int ka, int kb, double* out,
            unsigned long long* table, hipStream_t s) {
  contingency(a, b, n, ka, kb, table, s);
  hipLaunchKernelGGL(ari_finish, dim3(1), dim3(256), 0, s, table, n, ka, kb, out);
  return check_hip(hipGetLastError(), "ari launch");
}

int nmi_run(Context*, const int32_t* a, const int32_t* b, int64_t n, int ka, int kb, double* out,
            unsigned long long* table, double* margin, hipStream_t s) {
  contingency(a, b, n, ka, kb, table, s);
  hipLaunchKernelGGL(nmi_finish, dim3(1), dim3(256), 0, s, table, ka, kb, margin, out);
  return check_hip(hipGetLastError(), "nmi launch");
}

}  // namespace fsc
