// Symmetry check of a CSR graph (fsc_opts.validate = 2): Sec. 2 takes G
// undirected, so A must equal its transpose.  Duplicate entries of a row add
// up, as they do in the degrees and the sparse product, so the check is
// A(r, c) == A(c, r) for every stored (r, c), each side the FP64 sum of its
// duplicates.
//
// The entries are sorted by (row, column) with their weight as the
// tie-break (a stable radix sort by weight, then a stable one by position),
// so that the duplicates of one position sit together in ascending order of
// weight.  One thread per run of equal positions sums its run, finds the
// mirrored position by binary search and sums that run the same way; an
// absent mirror counts as 0.  Summing both runs in ascending order of weight
// makes the comparison exact whenever the two runs hold the same weights.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <climits>

namespace fsc {

constexpr int kRowBits = 31;  // a row or column index fits 31 bits (n < 2^31)
constexpr unsigned long long kColMask = (1ull << kRowBits) - 1;

// Weight bits whose unsigned order is the numeric order of non-negative
// weights (-0 becomes +0); unit weights give 0.
template <typename W> struct wbits;
template <> struct wbits<void> {
  static constexpr int bits = 0;
  __device__ static unsigned long long get(const void*, int64_t) { return 0; }
  __device__ static double value(unsigned long long) { return 1.0; }
};
template <> struct wbits<double> {
  static constexpr int bits = 64;
  __device__ static unsigned long long get(const double* v, int64_t j) {
    const double x = v[j];
    return x == 0.0 ? 0ull : (unsigned long long)__double_as_longlong(x);
  }
  __device__ static double value(unsigned long long b) { return __longlong_as_double((long long)b); }
};
template <> struct wbits<float> {
  static constexpr int bits = 32;
  __device__ static unsigned long long get(const float* v, int64_t j) {
    const float x = v[j];
    return x == 0.0f ? 0ull : (unsigned long long)__float_as_uint(x);
  }
  __device__ static double value(unsigned long long b) { return (double)__uint_as_float((uint32_t)b); }
};
template <> struct wbits<bf16_t> {
  static constexpr int bits = 16;
  __device__ static unsigned long long get(const bf16_t* v, int64_t j) {
    const uint16_t h = v[j].bits;
    return (h & 0x7fffu) == 0 ? 0ull : (unsigned long long)h;
  }
  __device__ static double value(unsigned long long b) { return (double)bf16_to_f32((uint16_t)b); }
};

// Entry j of the CSR: key (row << 31 | column) and its weight bits.  The row
// is the last r with row_ptr[r] <= j (binary search; empty rows share their
// row_ptr value with the next row).
template <typename W>
__global__ void sym_keys_kernel(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                const W* __restrict__ val, int64_t n, int64_t nnz,
                                unsigned long long* __restrict__ key, unsigned long long* __restrict__ wb) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = 0, hi = n - 1;  // row_ptr[lo] <= j always (row_ptr[0] = 0)
    while (lo < hi) {
      const int64_t mid = (lo + hi + 1) >> 1;
      if (row_ptr[mid] <= j) lo = mid; else hi = mid - 1;
    }
    key[j] = ((unsigned long long)lo << kRowBits) | (unsigned long long)(uint32_t)col[j];
    wb[j] = wbits<W>::get(val, j);
  }
}

// FP64 sum of the run of `key` starting at i (ascending order of weight).
template <typename W>
__device__ double run_sum(const unsigned long long* key, const unsigned long long* wb, int64_t nnz, int64_t i) {
  const unsigned long long k = key[i];
  double s = 0.0;
  for (; i < nnz && key[i] == k; ++i) s += wbits<W>::value(wb[i]);
  return s;
}

template <typename W>
__global__ void sym_check_kernel(const unsigned long long* __restrict__ key, const unsigned long long* __restrict__ wb,
                                 int64_t nnz, int32_t* __restrict__ flag) {
  for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nnz; j += (int64_t)gridDim.x * blockDim.x) {
    const unsigned long long k = key[j];
    if (j > 0 && key[j - 1] == k) continue;  // not the head of its run
    const unsigned long long r = k >> kRowBits, c = k & kColMask;
    const unsigned long long m = (c << kRowBits) | r;
    int64_t lo = 0, hi = nnz;  // first entry >= m
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (key[mid] < m) lo = mid + 1; else hi = mid;
    }
    const double a = run_sum<W>(key, wb, nnz, j);
    const double b = (lo < nnz && key[lo] == m) ? run_sum<W>(key, wb, nnz, lo) : 0.0;
    if (a != b) atomicOr(flag, 1);
  }
}

static int key_width(int64_t n) {
  int b = 1;
  while (b < 62 && ((unsigned long long)(n - 1) << kRowBits) >> b != 0) ++b;
  return std::max(b, kRowBits + 1);
}

static size_t sym_temp_bytes(const fsc_csr* g) {
  size_t t1 = 0, t2 = 0;
  const int cnt = (int)g->nnz;
  hipcub::DeviceRadixSort::SortPairs(nullptr, t1, (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                     (const unsigned long long*)nullptr, (unsigned long long*)nullptr, cnt, 0, 64);
  hipcub::DeviceRadixSort::SortPairs(nullptr, t2, (const unsigned long long*)nullptr, (unsigned long long*)nullptr,
                                     (const unsigned long long*)nullptr, (unsigned long long*)nullptr, cnt, 0,
                                     key_width(g->n));
  return std::max(t1, t2);
}

size_t symmetry_workspace_bytes(const fsc_csr* g) {
  if (g->nnz <= 0 || g->nnz > INT32_MAX) return 0;
  return align_up((size_t)g->nnz * 8) * 4 + align_up(sym_temp_bytes(g)) + align_up(64) + 1024;
}

template <typename W>
static int sym_run(Context* ctx, const fsc_csr* g, Arena* a, hipStream_t s) {
  const int64_t nnz = g->nnz;
  unsigned long long* k0 = a->take<unsigned long long>((size_t)nnz);
  unsigned long long* w0 = a->take<unsigned long long>((size_t)nnz);
  unsigned long long* k1 = a->take<unsigned long long>((size_t)nnz);
  unsigned long long* w1 = a->take<unsigned long long>((size_t)nnz);
  size_t temp_bytes = sym_temp_bytes(g);
  void* temp = a->take<char>(temp_bytes);
  int32_t* flag = a->take<int32_t>(16);
  if (a->used > a->size) return fail(FSC_E_NOMEM, "symmetry check workspace too small");
  int rc;
  const int blocks = (int)std::min<int64_t>((nnz + 255) / 256, 8192);
  if ((rc = fill_zero_i32(flag, 1, s))) return rc;
  hipLaunchKernelGGL(sym_keys_kernel<W>, dim3(blocks), dim3(256), 0, s, g->row_ptr, g->col_idx,
                     static_cast<const W*>(g->val), g->n, nnz, k0, w0);
  if ((rc = check_hip(hipGetLastError(), "symmetry keys launch"))) return rc;
  const int kb = key_width(g->n);
  if (wbits<W>::bits > 0) {
    // stable by weight, then stable by position: (position, weight) order
    if ((rc = check_hip(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, w0, w1, k0, k1, (int)nnz, 0,
                                                           wbits<W>::bits, s),
                        "symmetry sort by weight")))
      return rc;
    if ((rc = check_hip(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, k1, k0, w1, w0, (int)nnz, 0, kb, s),
                        "symmetry sort by position")))
      return rc;
  } else {
    if ((rc = check_hip(hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, k0, k1, w0, w1, (int)nnz, 0, kb, s),
                        "symmetry sort by position")))
      return rc;
    std::swap(k0, k1);
    std::swap(w0, w1);
  }
  hipLaunchKernelGGL(sym_check_kernel<W>, dim3(blocks), dim3(256), 0, s, k0, w0, nnz, flag);
  if ((rc = check_hip(hipGetLastError(), "symmetry check launch"))) return rc;
  if ((rc = check_hip(hipMemcpyAsync(ctx->host_flag, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s),
                      "symmetry flag copy")))
    return rc;
  if ((rc = check_hip(hipStreamSynchronize(s), "symmetry sync"))) return rc;
  if (ctx->host_flag[0]) return fail(FSC_E_GRAPH, "adjacency is not symmetric");
  return FSC_OK;
}

int validate_symmetry(Context* ctx, const fsc_csr* g, Arena scratch, hipStream_t s) {
  if (g->nnz == 0) return FSC_OK;
  if (g->nnz > INT32_MAX) return fail(FSC_E_UNSUPPORTED, "the symmetry check takes fewer than 2^31 nonzeros");
  scratch.used = 0;
  if (!g->val) return sym_run<void>(ctx, g, &scratch, s);
  switch (g->val_dtype) {
    case FSC_F64: return sym_run<double>(ctx, g, &scratch, s);
    case FSC_F32: return sym_run<float>(ctx, g, &scratch, s);
    case FSC_BF16: return sym_run<bf16_t>(ctx, g, &scratch, s);
  }
  return fail(FSC_E_ARG, "bad val_dtype");
}

}  // namespace fsc
