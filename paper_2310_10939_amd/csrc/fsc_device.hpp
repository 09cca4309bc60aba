// Device-side building blocks shared by the libfsc kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FSC_WAVE 64

namespace fsc {

// ---------------------------------------------------------------------------
// bfloat16 storage: the upper 16 bits of a binary32.
// ---------------------------------------------------------------------------
struct bf16_t {
  uint16_t bits;
};

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// Round to nearest, ties to even; NaN stays a (quiet) NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// ---------------------------------------------------------------------------
// Element-type traits: storage type S, accumulation type A.
// ---------------------------------------------------------------------------
template <typename S> struct elem;
template <> struct elem<double> {
  using acc = double;
  __device__ static __forceinline__ double load(const double* p) { return *p; }
  __device__ static __forceinline__ double to_acc(double v) { return v; }
  __device__ static __forceinline__ double from_acc(double v) { return v; }
};
template <> struct elem<float> {
  using acc = float;
  __device__ static __forceinline__ float to_acc(float v) { return v; }
  __device__ static __forceinline__ float from_acc(float v) { return v; }
};
template <> struct elem<bf16_t> {
  using acc = float;
  __device__ static __forceinline__ float to_acc(bf16_t v) { return bf16_to_f32(v.bits); }
  __device__ static __forceinline__ bf16_t from_acc(float v) { return bf16_t{f32_to_bf16(v)}; }
};

// Weight of one nonzero: void means unit weights.
template <typename W, typename A> struct weight {
  __device__ static __forceinline__ A get(const W* v, int64_t j) { return static_cast<A>(v[j]); }
};
template <typename A> struct weight<bf16_t, A> {
  __device__ static __forceinline__ A get(const bf16_t* v, int64_t j) {
    return static_cast<A>(bf16_to_f32(v[j].bits));
  }
};
template <typename A> struct weight<void, A> {
  __device__ static __forceinline__ A get(const void*, int64_t) { return A(1); }
};

// ---------------------------------------------------------------------------
// Row I/O for a padded row of LH values of storage type S, converted to A.
// Rows are LH*sizeof(S) bytes and aligned to that size, so one or two wide
// loads move a whole row.
// ---------------------------------------------------------------------------
template <typename S, int LH> struct rowio;

template <int LH> struct rowio<float, LH> {
  __device__ static __forceinline__ void load(const float* p, float* out) {
    if constexpr (LH == 1) {
      out[0] = p[0];
    } else if constexpr (LH == 2) {
      float2 v = *reinterpret_cast<const float2*>(p);
      out[0] = v.x; out[1] = v.y;
    } else {
#pragma unroll
      for (int q = 0; q < LH / 4; ++q) {
        float4 v = reinterpret_cast<const float4*>(p)[q];
        out[4 * q + 0] = v.x; out[4 * q + 1] = v.y; out[4 * q + 2] = v.z; out[4 * q + 3] = v.w;
      }
    }
  }
  __device__ static __forceinline__ void store(float* p, const float* in) {
    if constexpr (LH == 1) {
      p[0] = in[0];
    } else if constexpr (LH == 2) {
      *reinterpret_cast<float2*>(p) = make_float2(in[0], in[1]);
    } else {
#pragma unroll
      for (int q = 0; q < LH / 4; ++q)
        reinterpret_cast<float4*>(p)[q] = make_float4(in[4 * q], in[4 * q + 1], in[4 * q + 2], in[4 * q + 3]);
    }
  }
};

template <int LH> struct rowio<double, LH> {
  __device__ static __forceinline__ void load(const double* p, double* out) {
    if constexpr (LH == 1) {
      out[0] = p[0];
    } else {
#pragma unroll
      for (int q = 0; q < LH / 2; ++q) {
        double2 v = reinterpret_cast<const double2*>(p)[q];
        out[2 * q] = v.x; out[2 * q + 1] = v.y;
      }
    }
  }
  __device__ static __forceinline__ void store(double* p, const double* in) {
    if constexpr (LH == 1) {
      p[0] = in[0];
    } else {
#pragma unroll
      for (int q = 0; q < LH / 2; ++q)
        reinterpret_cast<double2*>(p)[q] = make_double2(in[2 * q], in[2 * q + 1]);
    }
  }
};

template <int LH> struct rowio<bf16_t, LH> {
  __device__ static __forceinline__ void load(const bf16_t* p, float* out) {
    const uint16_t* h = reinterpret_cast<const uint16_t*>(p);
    if constexpr (LH == 1) {
      out[0] = bf16_to_f32(h[0]);
    } else if constexpr (LH == 2) {
      uint32_t w = *reinterpret_cast<const uint32_t*>(h);
      out[0] = __uint_as_float(w << 16); out[1] = __uint_as_float(w & 0xffff0000u);
    } else if constexpr (LH == 4) {
      uint2 w = *reinterpret_cast<const uint2*>(h);
      out[0] = __uint_as_float(w.x << 16); out[1] = __uint_as_float(w.x & 0xffff0000u);
      out[2] = __uint_as_float(w.y << 16); out[3] = __uint_as_float(w.y & 0xffff0000u);
    } else {
      uint4 w = *reinterpret_cast<const uint4*>(h);
      uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        out[2 * q] = __uint_as_float(ws[q] << 16);
        out[2 * q + 1] = __uint_as_float(ws[q] & 0xffff0000u);
      }
    }
  }
  __device__ static __forceinline__ void store(bf16_t* p, const float* in) {
    uint16_t* h = reinterpret_cast<uint16_t*>(p);
    if constexpr (LH == 1) {
      h[0] = f32_to_bf16(in[0]);
    } else if constexpr (LH == 2) {
      *reinterpret_cast<uint32_t*>(h) = f32_to_bf16(in[0]) | (uint32_t(f32_to_bf16(in[1])) << 16);
    } else if constexpr (LH == 4) {
      uint2 w;
      w.x = f32_to_bf16(in[0]) | (uint32_t(f32_to_bf16(in[1])) << 16);
      w.y = f32_to_bf16(in[2]) | (uint32_t(f32_to_bf16(in[3])) << 16);
      *reinterpret_cast<uint2*>(h) = w;
    } else {
      uint4 w;
      w.x = f32_to_bf16(in[0]) | (uint32_t(f32_to_bf16(in[1])) << 16);
      w.y = f32_to_bf16(in[2]) | (uint32_t(f32_to_bf16(in[3])) << 16);
      w.z = f32_to_bf16(in[4]) | (uint32_t(f32_to_bf16(in[5])) << 16);
      w.w = f32_to_bf16(in[6]) | (uint32_t(f32_to_bf16(in[7])) << 16);
      *reinterpret_cast<uint4*>(h) = w;
    }
  }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the 53-bit uniform.
// ---------------------------------------------------------------------------
struct u32x4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
    const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
    c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
  }
  return c;
}

// ((hi:lo >> 11) + 1/2) * 2^-53, a double in (0, 1).
__device__ __forceinline__ double uniform53(uint32_t hi, uint32_t lo) {
  const uint64_t w = (static_cast<uint64_t>(hi) << 32) | lo;
  return (static_cast<double>(w >> 11) + 0.5) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Wave-level helpers.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T shfl_xor(T v, int mask) {
  return __shfl_xor(v, mask, FSC_WAVE);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, FSC_WAVE);
  return v;
}

// Sum across all threads of a block of BLOCK threads (BLOCK a multiple of 64);
// the result is valid in every thread.  Fixed order, so deterministic.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double* lds /* BLOCK/64 */) {
  v = wave_sum(v);
  const int w = threadIdx.x / FSC_WAVE;
  __syncthreads();
  if ((threadIdx.x & (FSC_WAVE - 1)) == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < BLOCK / FSC_WAVE; ++i) s += lds[i];
  __syncthreads();
  return s;
}

// N sums across a block at once: wave sums of each, then one exchange of the
// wave totals through LDS (one barrier for all N instead of N block_sums).
// The results are valid in every thread; fixed order, so deterministic.
template <int BLOCK, int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double* lds /* N * BLOCK/64 */) {
  constexpr int W = BLOCK / FSC_WAVE;
  const int w = threadIdx.x / FSC_WAVE;
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if ((threadIdx.x & (FSC_WAVE - 1)) == 0)
#pragma unroll
    for (int q = 0; q < N; ++q) lds[q * W + w] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < W; ++i) s += lds[q * W + i];
    v[q] = s;
  }
  __syncthreads();
}

// Inclusive scan across a block of BLOCK threads (wave shuffles, then the
// wave totals through LDS); fixed order, so deterministic.  Also returns the
// block total in *total.  `lds` holds BLOCK/64 + 1 values.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_scan_inclusive(T v, T* lds, T* total) {
  const int lane = threadIdx.x & (FSC_WAVE - 1);
  const int w = threadIdx.x / FSC_WAVE;
#pragma unroll
  for (int off = 1; off < FSC_WAVE; off <<= 1) {
    const T x = __shfl_up(v, off, FSC_WAVE);
    if (lane >= off) v += x;
  }
  __syncthreads();
  if (lane == FSC_WAVE - 1) lds[w] = v;
  __syncthreads();
  T before = T(0), all = T(0);
#pragma unroll
  for (int i = 0; i < BLOCK / FSC_WAVE; ++i) {
    const T x = lds[i];
    if (i < w) before += x;
    all += x;
  }
  __syncthreads();
  *total = all;
  return before + v;
}

template <typename T>
__device__ __forceinline__ T nt_load(const T* p) {
  return __builtin_nontemporal_load(p);
}

}  // namespace fsc
