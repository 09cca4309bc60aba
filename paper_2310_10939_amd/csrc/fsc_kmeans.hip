// k-means on the embedding rows (Sec. 2.2): k-means++ seeding, then Lloyd.
//
// Points are FP32 rows of KD = 4 or 8 values (the embedding padded with
// zeros; padding changes no distance).
//
// Seeding: one launch per centre.  Each block owns a contiguous run of rows,
// updates D2(v) = min(D2(v), ||p_v - c_{r-1}||^2) and writes the FP64 sum of
// its weights; the last block to finish scans the block sums, locates the
// block holding the sample u * sum(D2) and rescans that block's rows (same
// summation order) to find the sampled row.  No host round trip.
//
// Lloyd: one launch per step.  Distances come from MFMA
// (v_mfma_f32_16x16x4_f32): a 16-row tile of points times the 16-centre tiles
// of C^T gives e.c for 16 x 16 pairs, and ||c||^2 - 2 e.c is minimised over
// the centres with wave shuffles (ties to the lower index).  The centre
// update is a second contraction on the same unit: the one-hot matrix of the
// labels (transposed) times the point tile, with a ones column for the
// counts, accumulated over the wave's tiles.  Per-block FP64 partial sums are
// combined by the last block in a fixed order, so results are deterministic.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>

namespace fsc {

constexpr int kKB = 256;   // threads per block
constexpr int kRPT = 8;    // rows per thread in the seeding kernel
constexpr int kMaxK = 64;

typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// k-means++ seeding round r (r = 0: uniform over eligible rows).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double seed_weight(int first, const uint8_t* elig, int64_t v, float d2v) {
  const bool e = elig ? elig[v] != 0 : true;
  if (!e) return 0.0;
  return first ? 1.0 : (double)d2v;
}

// Inclusive scan of one double per thread over the block (fixed order).
__device__ __forceinline__ double block_inclusive_scan(double v, double* buf /* kKB */) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kKB; off <<= 1) {
    const double x = threadIdx.x >= off ? buf[threadIdx.x - off] : 0.0;
    __syncthreads();
    buf[threadIdx.x] += x;
    __syncthreads();
  }
  const double r = buf[threadIdx.x];
  __syncthreads();
  return r;
}

template <int KD>
__global__ __launch_bounds__(kKB) void kpp_round(int64_t n, const float* __restrict__ pts,
                                                 const uint8_t* __restrict__ elig, float* __restrict__ d2,
                                                 double* __restrict__ bsum, int32_t* __restrict__ counter,
                                                 float* __restrict__ centres, int32_t* __restrict__ chosen,
                                                 int r, uint32_t k0, uint32_t k1) {
  __shared__ double buf[kKB];
  __shared__ int is_last;
  __shared__ int32_t found;
  __shared__ double sh_base;
  __shared__ int32_t sh_block;
  const int first = (r == 0);
  const int64_t rpb = (int64_t)kKB * kRPT;
  const int nblk = gridDim.x;

  // phase A: weights of this block's rows
  {
    float c[KD];
    if (!first) {
#pragma unroll
      for (int q = 0; q < KD; ++q) c[q] = centres[(r - 1) * KD + q];
    }
    const int64_t v0 = (int64_t)blockIdx.x * rpb + (int64_t)threadIdx.x * kRPT;
    double ts = 0.0;
    float dv[kRPT];
    if (!first) {
      float p[kRPT][KD];
      float old[kRPT];
#pragma unroll
      for (int i = 0; i < kRPT; ++i) {
        const int64_t v = v0 + i;
        if (v < n) {
          rowio<float, KD>::load(pts + v * KD, p[i]);
          old[i] = r == 1 ? __builtin_inff() : d2[v];
        }
      }
#pragma unroll
      for (int i = 0; i < kRPT; ++i) {
        float dist = 0.f;
#pragma unroll
        for (int q = 0; q < KD; ++q) {
          const float e = p[i][q] - c[q];
          dist += e * e;
        }
        dv[i] = fminf(old[i], dist);
        if (v0 + i < n) d2[v0 + i] = dv[i];
      }
    }
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const int64_t v = v0 + i;
      if (v < n) ts += seed_weight(first, elig, v, first ? 0.f : dv[i]);
    }
    const double inc = block_inclusive_scan(ts, buf);
    if (threadIdx.x == kKB - 1) bsum[blockIdx.x] = inc;
  }
  // hand-off to the last block
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const int prev = atomicAdd(counter, 1);
    is_last = (prev == nblk - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();

  // phase B (last block): sample u * sum(weights) over the block sums, then
  // inside the block that holds it.  Both passes over the block sums use the
  // same chunked scan, so the prefixes they see are bit-identical.
  const u32x4 rr = philox4x32_10(u32x4{first ? 0u : (uint32_t)r, 0u, 0u, first ? 1u : 2u}, k0, k1);
  const double u = uniform53(rr.x, rr.y);
  double total = 0.0;
  for (int base = 0; base < nblk; base += kKB) {
    const int b = base + threadIdx.x;
    const double inc = block_inclusive_scan(b < nblk ? bsum[b] : 0.0, buf) + total;
    buf[threadIdx.x] = inc;
    __syncthreads();
    total = buf[kKB - 1];
    __syncthreads();
  }
  const double target = u * total;
  int64_t pick = -1;
  if (total > 0.0) {
    if (threadIdx.x == 0) {
      sh_block = -1;
      sh_base = 0.0;
    }
    __syncthreads();
    double carry = 0.0;
    for (int base = 0; base < nblk; base += kKB) {
      const int b = base + threadIdx.x;
      const double inc = block_inclusive_scan(b < nblk ? bsum[b] : 0.0, buf) + carry;
      buf[threadIdx.x] = inc;
      __syncthreads();
      const double excl = threadIdx.x == 0 ? carry : buf[threadIdx.x - 1];
      if (b < nblk && inc > target && excl <= target) {
        sh_block = b;
        sh_base = excl;
      }
      carry = buf[kKB - 1];
      __syncthreads();
      if (sh_block >= 0) break;
    }
    if (sh_block < 0 && threadIdx.x == 0) {  // rounding at the very end
      for (int b = nblk - 1; b >= 0; --b)
        if (bsum[b] > 0.0) {
          sh_block = b;
          double e = 0.0;
          sh_base = e;  // the in-block search below falls back to the last row
          break;
        }
    }
    __syncthreads();
    const int B = sh_block;
    const double before = sh_base;
    // rescan block B's rows in the order of phase A
    const int64_t v0 = (int64_t)B * rpb + (int64_t)threadIdx.x * kRPT;
    double w[kRPT];
    double ts = 0.0;
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      const int64_t v = v0 + i;
      w[i] = v < n ? seed_weight(first, elig, v, first ? 0.f : d2[v]) : 0.0;
      ts += w[i];
    }
    const double inc = block_inclusive_scan(ts, buf);
    buf[threadIdx.x] = inc;
    if (threadIdx.x == 0) found = INT32_MAX;
    __syncthreads();
    double run = before + (threadIdx.x == 0 ? 0.0 : buf[threadIdx.x - 1]);
#pragma unroll
    for (int i = 0; i < kRPT; ++i) {
      run += w[i];
      if (w[i] > 0.0 && run > target) {
        atomicMin(&found, (int32_t)(threadIdx.x * kRPT + i));
        break;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0 && found == INT32_MAX) {  // rounding: last positive row of B
      for (int i = kKB * kRPT - 1; i >= 0; --i) {
        const int64_t v = (int64_t)B * rpb + i;
        if (v < n && seed_weight(first, elig, v, first ? 0.f : d2[v]) > 0.0) {
          found = i;
          break;
        }
      }
    }
    __syncthreads();
    pick = (int64_t)B * rpb + found;
  } else {
    // every weight is 0: the smallest eligible row not chosen yet, else the
    // smallest row not chosen yet
    if (threadIdx.x == 0) found = INT32_MAX;
    __syncthreads();
    for (int pass = 0; pass < 2 && found == INT32_MAX; ++pass) {
      for (int64_t base = 0; base < n; base += kKB) {
        const int64_t v = base + threadIdx.x;
        bool ok = v < n;
        if (ok && pass == 0 && elig) ok = elig[v] != 0;
        if (ok)
          for (int j = 0; j < r; ++j)
            if (chosen[j] == v) {
              ok = false;
              break;
            }
        if (ok) atomicMin(&found, (int32_t)v);
        __syncthreads();
        if (found != INT32_MAX) break;
      }
      __syncthreads();
    }
    pick = found;
  }
  if (threadIdx.x == 0) {
    chosen[r] = (int32_t)pick;
    *counter = 0;
  }
  if (threadIdx.x < KD) centres[r * KD + threadIdx.x] = pts[pick * KD + threadIdx.x];
}

// ---------------------------------------------------------------------------
// Lloyd step: assignment (MFMA distances) and, with UPDATE, the centre update.
// ---------------------------------------------------------------------------
template <int KD, int KT, bool UPDATE>
__global__ __launch_bounds__(kKB) void lloyd_step(int64_t n, const float* __restrict__ pts,
                                                  const uint8_t* __restrict__ elig, float* __restrict__ centres,
                                                  int k, int32_t* __restrict__ labels, double* __restrict__ cpart,
                                                  int32_t* __restrict__ counter, int tpw) {
  __shared__ float wsum[UPDATE ? 4 : 1][UPDATE ? KT * 16 : 1][UPDATE ? 16 : 1];
  __shared__ int is_last;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;   // output column (centre within a tile)
  const int kk = lane >> 4;    // contraction index / output row group

  // centre operands and squared norms for this lane's output column
  float b0[KT], b1[KT], cn[KT];
#pragma unroll
  for (int jt = 0; jt < KT; ++jt) {
    const int j = jt * 16 + col;
    float c[KD];
    float nrm = 0.f;
#pragma unroll
    for (int q = 0; q < KD; ++q) {
      c[q] = j < k ? centres[j * KD + q] : 0.f;
      nrm += c[q] * c[q];
    }
    b0[jt] = c[kk];
    b1[jt] = KD == 8 ? c[4 + kk] : 0.f;
    cn[jt] = j < k ? nrm : __builtin_inff();
  }

  floatx4 uacc[KT];
#pragma unroll
  for (int jt = 0; jt < KT; ++jt) uacc[jt] = floatx4{0.f, 0.f, 0.f, 0.f};

  const int64_t tile0 = ((int64_t)blockIdx.x * 4) * tpw;
  constexpr int kB = 4;  // tiles whose loads are in flight together
  for (int it0 = 0; it0 < tpw; it0 += kB) {
    float a0s[kB], a1s[kB];
#pragma unroll
    for (int bi = 0; bi < kB; ++bi) {
      const int64_t tile = tile0 + (int64_t)(it0 + bi) * 4 + wave;
      const int64_t ra = tile * 16 + col;
      a0s[bi] = 0.f;
      a1s[bi] = 0.f;
      if (it0 + bi < tpw && ra < n) {
        a0s[bi] = pts[ra * KD + kk];
        if (KD == 8) a1s[bi] = pts[ra * KD + 4 + kk];
      }
    }
#pragma unroll
    for (int bi = 0; bi < kB; ++bi) {
    const int64_t tile = tile0 + (int64_t)(it0 + bi) * 4 + wave;
    const int64_t row0 = tile * 16;
    if (it0 + bi >= tpw || row0 >= n) break;
    const float a0 = a0s[bi], a1 = a1s[bi];
    float bd[4];
    int bj[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      bd[r] = __builtin_inff();
      bj[r] = 0;
    }
#pragma unroll
    for (int jt = 0; jt < KT; ++jt) {
      floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0[jt], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      if (KD == 8) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1[jt], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float d = cn[jt] - 2.f * acc[r];
        if (d < bd[r]) {
          bd[r] = d;
          bj[r] = jt * 16 + col;
        }
      }
    }
    // argmin over the 16 lanes of the group (lexicographic on (d, j))
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float od = __shfl_xor(bd[r], m, 64);
        const int oj = __shfl_xor(bj[r], m, 64);
        if (od < bd[r] || (od == bd[r] && oj < bj[r])) {
          bd[r] = od;
          bj[r] = oj;
        }
      }
    }
    // row i = 4*kk + r of the tile is held by the lanes of group kk, reg r
    if (col < 4) {
      const int64_t row = row0 + 4 * kk + col;
      const int lab = col == 0 ? bj[0] : col == 1 ? bj[1] : col == 2 ? bj[2] : bj[3];
      if (row < n) labels[row] = lab;
    }
    if constexpr (UPDATE) {
      const int sel = lane & 3;
      const int lab_src = sel == 0 ? bj[0] : sel == 1 ? bj[1] : sel == 2 ? bj[2] : bj[3];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int lab = __shfl(lab_src, 16 * q + kk, 64);     // label of row 4q + kk
        const int64_t rb = row0 + 4 * q + kk;
        const bool valid = rb < n && (elig == nullptr || elig[rb] != 0);
        const int src = (4 * q + kk) + 16 * (col & 3);
        const float v0 = __shfl(a0, src, 64);
        const float v1 = __shfl(a1, src, 64);
        float bval = col < 4 ? v0 : (col < 8 && KD == 8 ? v1 : 0.f);
        if (col == KD) bval = 1.f;
        if (!valid) bval = 0.f;
#pragma unroll
        for (int jt = 0; jt < KT; ++jt) {
          const float aval = (valid && lab == jt * 16 + col) ? 1.f : 0.f;
          uacc[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(aval, bval, uacc[jt], 0, 0, 0);
        }
      }
    }
    }
  }

  if constexpr (UPDATE) {
    // uacc[jt][r] = sum over this wave's rows for centre jt*16 + 4*kk + r, dim col
#pragma unroll
    for (int jt = 0; jt < KT; ++jt)
#pragma unroll
      for (int r = 0; r < 4; ++r) wsum[wave][jt * 16 + 4 * kk + r][col] = uacc[jt][r];
    __syncthreads();
    const int O = k * (KD + 1);
    for (int o = threadIdx.x; o < O; o += kKB) {
      const int j = o / (KD + 1), d = o % (KD + 1);
      const int dd = d == KD ? KD : d;  // dim KD holds the count
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < 4; ++w) s += (double)wsum[w][j][dd];
      cpart[(int64_t)blockIdx.x * O + o] = s;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
      const int prev = atomicAdd(counter, 1);
      is_last = (prev == (int)gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    __shared__ double tot[kMaxK * 9];
    __shared__ double part[kKB];
    // outputs o < O; each summed by S threads over interleaved block subsets,
    // the S partial sums then combined in subset order
    const int nblk = (int)gridDim.x;
    for (int o0 = 0; o0 < O; o0 += kKB) {
      const int cnt = min(kKB, O - o0);
      const int S = kKB / cnt;
      const int o = o0 + threadIdx.x % cnt, sidx = threadIdx.x / cnt;
      double acc = 0.0;
      if (sidx < S) {
        int b = sidx;
        for (; b + 3 * S < nblk; b += 4 * S) {
          const double x0 = cpart[(int64_t)b * O + o], x1 = cpart[(int64_t)(b + S) * O + o];
          const double x2 = cpart[(int64_t)(b + 2 * S) * O + o], x3 = cpart[(int64_t)(b + 3 * S) * O + o];
          acc += x0;
          acc += x1;
          acc += x2;
          acc += x3;
        }
        for (; b < nblk; b += S) acc += cpart[(int64_t)b * O + o];
      }
      part[threadIdx.x] = acc;
      __syncthreads();
      if (threadIdx.x < cnt) {
        double s2 = 0.0;
        for (int i = 0; i < S; ++i) s2 += part[i * cnt + threadIdx.x];
        tot[o0 + threadIdx.x] = s2;
      }
      __syncthreads();
    }
    for (int o = threadIdx.x; o < k * KD; o += kKB) {
      const int j = o / KD, d = o % KD;
      const double cnt = tot[j * (KD + 1) + KD];
      if (cnt > 0.0) centres[j * KD + d] = (float)(tot[j * (KD + 1) + d] / cnt);
    }
    if (threadIdx.x == 0) *counter = 0;
  }
}

__global__ void centres_out_kernel(const float* __restrict__ c, int k, int KD, int l, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k * l) out[i] = c[(i / l) * KD + (i % l)];
}

template <typename T>
__global__ void pad_points(const T* __restrict__ in, int64_t n, int l, int KD, float* __restrict__ out) {
  const int64_t total = n * KD;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / KD;
    const int q = (int)(i - r * KD);
    out[i] = q < l ? (float)in[r * l + q] : 0.f;
  }
}

__global__ void zero_i32(int32_t* p, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = 0;
}

// ===========================================================================
// Host side
// ===========================================================================
static int lloyd_tpw(int64_t n, int num_cu) {
  const int64_t tiles = (n + 15) / 16;
  const int64_t target_blocks = 2LL * num_cu;
  int64_t tpw = (tiles + 4 * target_blocks - 1) / (4 * target_blocks);
  if (tpw < 1) tpw = 1;
  if (tpw > 64) tpw = 64;
  return (int)tpw;
}

size_t kmeans_workspace_bytes(int64_t n, int KD) {
  const int64_t nblk_pp = (n + kKB * kRPT - 1) / (kKB * kRPT);
  const int64_t nblk_ll = (n + 63) / 64 + 1;  // upper bound (tpw >= 1)
  size_t b = 0;
  b += align_up(n * 4);                              // d2
  b += align_up(nblk_pp * 8);                        // bsum
  b += align_up(kMaxK * KD * 4);                     // centres
  b += align_up((size_t)nblk_ll * kMaxK * (KD + 1) * 8);  // cpart
  b += align_up(kMaxK * 4) + align_up(16);           // chosen, counter
  return b + 8 * 256;
}

int kmeans_bind_workspace(Arena* a, KmeansIO* io) {
  const int64_t n = io->n;
  io->nblk_pp = (int)((n + kKB * kRPT - 1) / (kKB * kRPT));
  io->d2 = a->take<float>(n);
  io->bsum = a->take<double>(io->nblk_pp);
  io->centres = a->take<float>(kMaxK * io->KD);
  io->cpart = a->take<double>((size_t)((n + 63) / 64 + 1) * kMaxK * (io->KD + 1));
  io->chosen = a->take<int32_t>(kMaxK);
  io->counter = a->take<int32_t>(4);
  if (a->used > a->size) return fail(FSC_E_NOMEM, "workspace arena too small");
  return FSC_OK;
}

template <int KD, int KT>
static int lloyd_all(Context* ctx, KmeansIO* io, hipStream_t s) {
  const int tpw = lloyd_tpw(io->n, ctx->num_cu);
  const int64_t tiles = (io->n + 15) / 16;
  const int nblk = (int)((tiles + 4LL * tpw - 1) / (4LL * tpw));
  for (int it = 0; it < io->iters; ++it) {
    hipLaunchKernelGGL((lloyd_step<KD, KT, true>), dim3(nblk), dim3(kKB), 0, s, io->n, io->pts, io->elig,
                       io->centres, io->k, io->labels, io->cpart, io->counter, tpw);
  }
  hipLaunchKernelGGL((lloyd_step<KD, KT, false>), dim3(nblk), dim3(kKB), 0, s, io->n, io->pts, io->elig,
                     io->centres, io->k, io->labels, io->cpart, io->counter, tpw);
  return check_hip(hipGetLastError(), "lloyd_step launch");
}

template <int KD>
static int kmeans_typed(Context* ctx, KmeansIO* io, hipStream_t s) {
  hipLaunchKernelGGL(zero_i32, dim3(1), dim3(64), 0, s, io->counter, 4);
  const uint32_t k0 = (uint32_t)(io->seed & 0xffffffffu), k1 = (uint32_t)(io->seed >> 32);
  for (int r = 0; r < io->k; ++r) {
    hipLaunchKernelGGL(kpp_round<KD>, dim3(io->nblk_pp), dim3(kKB), 0, s, io->n, io->pts, io->elig, io->d2,
                       io->bsum, io->counter, io->centres, io->chosen, r, k0, k1);
  }
  int rc = check_hip(hipGetLastError(), "kpp_round launch");
  if (rc) return rc;
  const int KT = (io->k + 15) / 16;
  switch (KT) {
    case 1: rc = lloyd_all<KD, 1>(ctx, io, s); break;
    case 2: rc = lloyd_all<KD, 2>(ctx, io, s); break;
    case 3: rc = lloyd_all<KD, 3>(ctx, io, s); break;
    default: rc = lloyd_all<KD, 4>(ctx, io, s); break;
  }
  if (rc) return rc;
  if (io->centres_out) {
    hipLaunchKernelGGL(centres_out_kernel, dim3((io->k * io->l + 255) / 256), dim3(256), 0, s, io->centres,
                       io->k, KD, io->l, io->centres_out);
    rc = check_hip(hipGetLastError(), "centres_out launch");
  }
  return rc;
}

int kmeans_run(Context* ctx, KmeansIO* io, hipStream_t s) {
  if (io->KD == 4) return kmeans_typed<4>(ctx, io, s);
  if (io->KD == 8) return kmeans_typed<8>(ctx, io, s);
  return fail(FSC_E_UNSUPPORTED, "k-means point width must be 4 or 8");
}

int points_from_user(Context*, const void* pts, int dtype, int64_t n, int l, int KD, float* out, hipStream_t s) {
  const int blocks = (int)std::min<int64_t>((n * KD + 255) / 256, 8192);
  if (dtype == FSC_F32)
    hipLaunchKernelGGL(pad_points<float>, dim3(blocks), dim3(256), 0, s, (const float*)pts, n, l, KD, out);
  else if (dtype == FSC_F64)
    hipLaunchKernelGGL(pad_points<double>, dim3(blocks), dim3(256), 0, s, (const double*)pts, n, l, KD, out);
  else
    return fail(FSC_E_UNSUPPORTED, "k-means points must be FSC_F32 or FSC_F64");
  return check_hip(hipGetLastError(), "pad_points launch");
}

}  // namespace fsc
