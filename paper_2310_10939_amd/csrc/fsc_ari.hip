// Adjusted Rand index (Hubert and Arabie), the accuracy score of Sec. 4.2.
// The contingency table is built with integer atomics (exact, so the result
// does not depend on the order of the updates); the index is then formed in
// FP64 by one block.  C(x, 2) of integer counts below 2^26 is exact in FP64.
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

int ari_run(Context*, const int32_t* a, const int32_t* b, int64_t n, int ka, int kb, double* out,
            unsigned long long* table, hipStream_t s) {
  const int64_t cells = (int64_t)ka * kb;
  hipLaunchKernelGGL(ari_zero, dim3((int)std::min<int64_t>((cells + 255) / 256, 4096)), dim3(256), 0, s, table, cells);
  if (n > 0)
    hipLaunchKernelGGL(ari_count, dim3((int)std::min<int64_t>((n + 255) / 256, 8192)), dim3(256), 0, s, a, b, n, ka,
                       kb, table);
  hipLaunchKernelGGL(ari_finish, dim3(1), dim3(256), 0, s, table, n, ka, kb, out);
  return check_hip(hipGetLastError(), "ari launch");
}

}  // namespace fsc
