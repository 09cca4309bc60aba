// k-means on the embedding rows (Sec. 2.2): k-means++ seeding, then Lloyd.
//
// Points are FP32 rows of KD = 4 or 8 values (the embedding padded with
// zeros; padding changes no distance).  One k-means problem is a "job"; the
// single-graph entry points launch one job, the batched form launches many in
// one grid (blocks map to (job, local block) through a prefix table).
//
// Seeding (greedy k-means++): per centre r >= 1, a pass over the rows and a
// one-block kernel, twice.  First each block owns a contiguous run of rows,
// updates D2(v) = min(D2(v), ||p_v - c_{r-1}||^2) and writes the FP64 sum of
// its weights; then L = 2 + floor(ln k) blocks draw one candidate each: each
// scans the block sums, locates the block holding the sample u_j * sum(D2)
// and rescans that block's rows (same summation order) to find the sampled
// row.  Second, each block sums, per candidate,
// min(D2(v), ||p_v - cand_j||^2) over its eligible rows, and one block keeps
// the candidate with the smallest total (ties to the lower j).  Centre 0 is
// one uniform draw over the eligible rows.  No host round trip, and no block
// waits on a device-scope fence (the stream orders the kernels).
//
// Lloyd: one launch per step.  Distances come from MFMA
// (v_mfma_f32_16x16x4_f32): a 16-centre tile of C times a 16-point tile of
// P^T gives c.e for 16 x 16 pairs, so each lane holds 4 centres of one point;
// ||c||^2 - 2 c.e is minimised over them in the lane and then across the 4
// lane groups of the point (ties to the lower index).  The centre
// update is a second contraction on the same unit: the one-hot matrix of the
// labels (transposed) times the point tile, with a ones column for the
// counts, accumulated over the wave's tiles.  The 16 waves of a block are
// summed in FP64 in wave order, and the per-block sums are combined in a fixed
// order by a one-block kernel per job after the step, so results are
// deterministic.
//
// Convergence: every step after the first counts the points whose label it
// changes.  A step that changes none leaves the centres where they were (the
// same labels give the same sums in the same order), so every later step
// would repeat it exactly; its centre update then marks the job converged and
// the remaining steps' launches return at once.  The result is bit for bit
// that of running all the steps.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace fsc {

constexpr int kKB = 256;    // threads per seeding block
constexpr int kRPT = 8;     // rows per thread in the seeding kernel
constexpr int kLB = 1024;   // threads per Lloyd block (16 waves)
constexpr int kLW = kLB / FSC_WAVE;
constexpr int kMaxK = 64;
constexpr int kMaxTrials = 6;  // 2 + floor(ln 64)

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, FSC_WAVE);
  return v;
}

// Shared state of a block, declared once per kernel (the segmented kernels
// instantiate several block bodies, which must not each own LDS).
struct KppShared {
  double sbuf[kKB / FSC_WAVE + 1];
  double inc[kKB];
  double base;
  int32_t found;
  int32_t block;
};
struct LloydShared {
  float cn[kMaxK];  // ||c_j||^2, +inf past k
  float wsum[kLW][kMaxK][9];
  int lab[kLW][16];
};

// ---------------------------------------------------------------------------
// k-means++ seeding round r (r = 0: uniform over eligible rows).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double seed_weight(int first, const uint8_t* elig, int64_t v, float d2v) {
  const bool e = elig ? elig[v] != 0 : true;
  if (!e) return 0.0;
  return first ? 1.0 : (double)d2v;
}

// The row holding `target` in the inclusive running sum of the seeding
// weights (run by one whole block; every thread returns it).  The block sums
// are scanned in chunks, then the found block's rows are rescanned in the
// order of phase A, so the prefixes are bit-identical to phase A's.
template <int KD>
__device__ int64_t kpp_sample(const KmJob& J, int first, double target, KppShared& sh) {
  double* sbuf = sh.sbuf;
  const int64_t n = J.n;
  const int64_t rpb = (int64_t)kKB * kRPT;
  const int nblk = J.nblk_pp;
  if (threadIdx.x == 0) {
    sh.block = -1;
    sh.base = 0.0;
  }
  __syncthreads();
  double carry = 0.0;
  for (int base = 0; base < nblk; base += kKB) {
    const int b = base + threadIdx.x;
    double ct;
    const double inc = block_scan_inclusive<kKB>(b < nblk ? J.bsum[b] : 0.0, sbuf, &ct) + carry;
    sh.inc[threadIdx.x] = inc;
    if (threadIdx.x == 0) sh.found = INT32_MAX;
    __syncthreads();
    if (b < nblk && inc > target) atomicMin(&sh.found, b);
    __syncthreads();
    if (sh.found != INT32_MAX) {
      // the prefix before the block, exactly as the scan computed it
      if (threadIdx.x == 0) {
        sh.block = sh.found;
        sh.base = sh.found == base ? carry : sh.inc[sh.found - base - 1];
      }
      __syncthreads();
      break;
    }
    carry += ct;  // equals the chunk's last inclusive value bit for bit
  }
  if (sh.block < 0 && threadIdx.x == 0) {  // rounding at the very end
    for (int b = nblk - 1; b >= 0; --b)
      if (J.bsum[b] > 0.0) {
        sh.block = b;
        sh.base = 0.0;  // the in-block search below falls back to the last row
        break;
      }
  }
  __syncthreads();
  const int B = sh.block;
  const double before = sh.base;
  const int64_t v0 = (int64_t)B * rpb + (int64_t)threadIdx.x * kRPT;
  double w[kRPT];
  double ts = 0.0;
#pragma unroll
  for (int i = 0; i < kRPT; ++i) {
    const int64_t v = v0 + i;
    w[i] = v < n ? seed_weight(first, J.elig, v, first ? 0.f : J.d2[v]) : 0.0;
    ts += w[i];
  }
  double bt;
  const double inc = block_scan_inclusive<kKB>(ts, sbuf, &bt);
  if (threadIdx.x == 0) sh.found = INT32_MAX;
  __syncthreads();
  double run = before + (inc - ts);
#pragma unroll
  for (int i = 0; i < kRPT; ++i) {
    run += w[i];
    if (w[i] > 0.0 && run > target) {
      atomicMin(&sh.found, (int32_t)(threadIdx.x * kRPT + i));
      break;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && sh.found == INT32_MAX) {  // rounding: last positive row of B
    for (int i = kKB * kRPT - 1; i >= 0; --i) {
      const int64_t v = (int64_t)B * rpb + i;
      if (v < n && seed_weight(first, J.elig, v, first ? 0.f : J.d2[v]) > 0.0) {
        sh.found = i;
        break;
      }
    }
  }
  __syncthreads();
  const int64_t pick = (int64_t)B * rpb + sh.found;
  __syncthreads();  // sh is reused by the next search
  return pick;
}

// Every weight is 0: the smallest eligible row not chosen yet, else the
// smallest row not chosen yet (every thread returns it).
__device__ int64_t kpp_unchosen(const KmJob& J, int r, KppShared& sh) {
  const int64_t n = J.n;
  if (threadIdx.x == 0) sh.found = INT32_MAX;
  __syncthreads();
  for (int pass = 0; pass < 2 && sh.found == INT32_MAX; ++pass) {
    for (int64_t base = 0; base < n; base += kKB) {
      const int64_t v = base + threadIdx.x;
      bool ok = v < n;
      if (ok && pass == 0 && J.elig) ok = J.elig[v] != 0;
      if (ok)
        for (int j = 0; j < r; ++j)
          if (J.chosen[j] == v) {
            ok = false;
            break;
          }
      if (ok) atomicMin(&sh.found, (int32_t)v);
      __syncthreads();
      if (sh.found != INT32_MAX) break;
    }
    __syncthreads();
  }
  const int64_t pick = sh.found;
  __syncthreads();
  return pick;
}

template <int KD>
__device__ void kpp_block(const KmJob& J, int blk, int r, KppShared& sh) {
  double* sbuf = sh.sbuf;
  const int64_t n = J.n;
  const int first = (r == 0);
  const int64_t rpb = (int64_t)kKB * kRPT;
  const float* pts = J.pts;
  const uint8_t* elig = J.elig;
  float* d2 = J.d2;

  // phase A: weights of this block's rows
  {
    float c[KD];
    if (!first) {
#pragma unroll
      for (int q = 0; q < KD; ++q) c[q] = J.centres[(r - 1) * KD + q];
    }
    const int64_t v0 = (int64_t)blk * rpb + (int64_t)threadIdx.x * kRPT;
    double ts = 0.0;
    float dv[kRPT];
    if (!first) {
      float p[kRPT][KD];
      float old[kRPT];
#pragma unroll
      for (int i = 0; i < kRPT; ++i) {
        const int64_t v = v0 + i;
        old[i] = __builtin_inff();
        if (v < n) {
          rowio<float, KD>::load(pts + v * KD, p[i]);
          if (r > 1) old[i] = d2[v];
        } else {
#pragma unroll
          for (int q = 0; q < KD; ++q) p[i][q] = 0.f;
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
    double total;
    block_scan_inclusive<kKB>(ts, sbuf, &total);
    if (threadIdx.x == 0) J.bsum[blk] = total;
  }
}

// Phase B of round r (one block per candidate j of each job, after phase A on
// the same stream): the total weight, then the draw u_j * total located by
// kpp_sample.
template <int KD>
__device__ void kpp_sample_block(const KmJob& J, int r, int j, KppShared& sh) {
  double* sbuf = sh.sbuf;
  const int first = (r == 0);
  if (j >= (first ? 1 : J.trials)) return;
  const int nblk = J.nblk_pp;
  const float* pts = J.pts;
  double total = 0.0;
  for (int base = 0; base < nblk; base += kKB) {
    const int b = base + threadIdx.x;
    double ct;
    block_scan_inclusive<kKB>(b < nblk ? J.bsum[b] : 0.0, sbuf, &ct);
    total += ct;
  }
  int64_t pick;
  if (total > 0.0) {
    // centre 0: stream 1, counter 0; candidate j of round r: stream 3,
    // counter r * L + j
    const uint32_t ctr = first ? 0u : (uint32_t)(r * J.trials + j);
    const u32x4 rr = philox4x32_10(u32x4{ctr, 0u, 0u, first ? 1u : 3u}, J.k0, J.k1);
    pick = kpp_sample<KD>(J, first, uniform53(rr.x, rr.y) * total, sh);
  } else {
    pick = kpp_unchosen(J, r, sh);  // every candidate is this row
  }
  if (first) {
    if (threadIdx.x == 0) J.chosen[r] = (int32_t)pick;
    if (threadIdx.x < KD) J.centres[r * KD + threadIdx.x] = pts[pick * KD + threadIdx.x];
  } else {
    if (threadIdx.x == 0) J.cand_row[j] = (int32_t)pick;
    if (threadIdx.x < KD) J.cand[j * KD + threadIdx.x] = pts[pick * KD + threadIdx.x];
  }
}

// Round r >= 1, second pass: the potential of each candidate over this
// block's rows (kpp_select_block then keeps the best candidate as centre r).
template <int KD>
__device__ void kpp_pick_block(const KmJob& J, int blk, int r, KppShared& sh) {
  const int64_t n = J.n;
  const int L = J.trials;
  const int64_t rpb = (int64_t)kKB * kRPT;
  const int nblk = J.nblk_pp;
  float c[kMaxTrials][KD];
#pragma unroll
  for (int j = 0; j < kMaxTrials; ++j)
#pragma unroll
    for (int q = 0; q < KD; ++q) c[j][q] = j < L ? J.cand[j * KD + q] : 0.f;
  double pot[kMaxTrials];
#pragma unroll
  for (int j = 0; j < kMaxTrials; ++j) pot[j] = 0.0;
  const int64_t v0 = (int64_t)blk * rpb + (int64_t)threadIdx.x * kRPT;
#pragma unroll 2
  for (int i = 0; i < kRPT; ++i) {
    const int64_t v = v0 + i;
    if (v >= n || (J.elig && !J.elig[v])) continue;
    float p[KD];
    rowio<float, KD>::load(J.pts + v * KD, p);
    const float dv = J.d2[v];
#pragma unroll
    for (int j = 0; j < kMaxTrials; ++j) {
      float dist = 0.f;
#pragma unroll
      for (int q = 0; q < KD; ++q) {
        const float e = p[q] - c[j][q];
        dist += e * e;
      }
      pot[j] += (double)fminf(dv, dist);
    }
  }
#pragma unroll
  for (int j = 0; j < kMaxTrials; ++j) {
    if (j >= L) break;
    const double t = block_sum<kKB>(pot[j], sh.sbuf);
    if (threadIdx.x == 0) J.bsum[(int64_t)blk * kMaxTrials + j] = t;
  }
}

// Round r >= 1 (one block per job, after the potentials): the candidate with
// the smallest total potential becomes centre r.
__device__ void kpp_select_block(const KmJob& J, int r, KppShared& sh) {
  const int L = J.trials;
  const int nblk = J.nblk_pp;
  const int KD = J.KD;
  double best = 0.0;
  int bj = 0;
  for (int j = 0; j < L; ++j) {
    double part = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kKB) part += J.bsum[(int64_t)b * kMaxTrials + j];
    const double t = block_sum<kKB>(part, sh.sbuf);
    if (j == 0 || t < best) {
      best = t;
      bj = j;
    }
  }
  const int32_t row = J.cand_row[bj];
  if (threadIdx.x == 0) J.chosen[r] = row;
  if (threadIdx.x < KD) J.centres[r * KD + threadIdx.x] = J.cand[bj * KD + threadIdx.x];
}

// ---------------------------------------------------------------------------
// Lloyd step: assignment (MFMA distances) and, with UPDATE, the centre update.
// ---------------------------------------------------------------------------
// Lexicographic (distance, index) minimum with the lane `mask` away.
__device__ __forceinline__ void argmin_xor(float& d, int& j, int mask) {
  const float od = shfl_xor(d, mask);
  const int oj = shfl_xor(j, mask);
  if (od < d || (od == d && oj < j)) {
    d = od;
    j = oj;
  }
}

template <int KD, int KT, bool UPDATE>
__device__ void lloyd_block(const KmJob& J, int blk, LloydShared& sh, bool count) {
  auto& wsum = sh.wsum;
  auto& lab_s = sh.lab;
  const int64_t n = J.n;
  const int k = J.k;
  const float* pts = J.pts;
  const uint8_t* elig = J.elig;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;   // output column: the point within a tile
  const int kk = lane >> 4;    // contraction index / output row group

  // The distance MFMA computes D = C P^T for 16 centres x 16 points: lane
  // (col, kk) supplies centre col's dimension kk (A) and point col's
  // dimension kk (B), and receives D[4 kk + r][col], the products of centres
  // 4 kk + r with point col.  So each lane scans 4 centres of one point and
  // the 4 lane groups of a point combine in two cross-lane steps.
  float b0[KT], b1[KT];
#pragma unroll
  for (int jt = 0; jt < KT; ++jt) {
    const int j = jt * 16 + col;
    float c[KD];
#pragma unroll
    for (int q = 0; q < KD; ++q) c[q] = j < k ? J.centres[j * KD + q] : 0.f;
    b0[jt] = c[kk];
    b1[jt] = KD == 8 ? c[4 + kk] : 0.f;
  }
  float* cn = sh.cn;
  if (threadIdx.x < 16 * KT) {
    const int j = threadIdx.x;
    float nrm = 0.f;
#pragma unroll
    for (int q = 0; q < KD; ++q) {
      const float v = j < k ? J.centres[j * KD + q] : 0.f;
      nrm += v * v;
    }
    cn[j] = j < k ? nrm : __builtin_inff();
  }
  __syncthreads();

  floatx4 uacc[KT];
#pragma unroll
  for (int jt = 0; jt < KT; ++jt) uacc[jt] = floatx4{0.f, 0.f, 0.f, 0.f};
  int changed = 0;  // labels this lane changed (counted steps only)

  const int tpw = J.tpw;
  const int64_t tile0 = ((int64_t)blk * kLW + wave) * tpw;  // this wave's first tile
  constexpr int kB = 4;  // tiles whose loads are in flight together
  // Lane (col, kk) loads dimension kk (and 4 + kk) of row col of a tile: the
  // A operand of the distance MFMA.  The update MFMA needs the transpose --
  // lane (col, kk) holding dimension col of row 4q + kk -- which comes from
  // the same registers by a cross-lane permute, not a second load.
  // Batches of kB tiles are software-pipelined: the next batch's loads are in
  // flight while this one computes.
  float a0n[kB], a1n[kB];
  auto load_batch = [&](int it0, float* a0, float* a1) {
#pragma unroll
    for (int bi = 0; bi < kB; ++bi) {
      const int64_t ra = (tile0 + it0 + bi) * 16 + col;
      a0[bi] = 0.f;
      a1[bi] = 0.f;
      if (it0 + bi < tpw && ra < n) {
        a0[bi] = pts[ra * KD + kk];
        if (KD == 8) a1[bi] = pts[ra * KD + 4 + kk];
      }
    }
  };
  load_batch(0, a0n, a1n);
  for (int it0 = 0; it0 < tpw; it0 += kB) {
    float a0s[kB], a1s[kB];
#pragma unroll
    for (int bi = 0; bi < kB; ++bi) {
      a0s[bi] = a0n[bi];
      a1s[bi] = a1n[bi];
    }
    if (it0 + kB < tpw) load_batch(it0 + kB, a0n, a1n);
#pragma unroll
    for (int bi = 0; bi < kB; ++bi) {
      const int64_t row0 = (tile0 + it0 + bi) * 16;
      if (it0 + bi >= tpw || row0 >= n) break;
      // nearest centre of point col: ||c||^2 - 2 c.p, ties to the lowest
      // centre index (centres are scanned in increasing order in a lane, and
      // the cross-lane steps compare (distance, index) pairs)
      float bd = __builtin_inff();
      int bj = 0;
#pragma unroll
      for (int jt = 0; jt < KT; ++jt) {
        floatx4 acc = __builtin_amdgcn_mfma_f32_16x16x4f32(b0[jt], a0s[bi], floatx4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
        if (KD == 8) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(b1[jt], a1s[bi], acc, 0, 0, 0);
        const floatx4 c4 = *reinterpret_cast<const floatx4*>(cn + jt * 16 + 4 * kk);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float d = c4[r] - 2.f * acc[r];
          if (d < bd) {
            bd = d;
            bj = jt * 16 + 4 * kk + r;
          }
        }
      }
      argmin_xor(bd, bj, 16);
      argmin_xor(bd, bj, 32);
      if (kk == 0) {
        const int64_t row = row0 + col;
        if (row < n) {
          if (UPDATE && count) changed += J.labels[row] != bj ? 1 : 0;
          J.labels[row] = bj;
        }
        if constexpr (UPDATE) lab_s[wave][col] = bj;
      }
      if constexpr (UPDATE) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // dimension col of row 4q + kk sits in lane (4q + kk, col & 3),
          // register a0 (col < 4) or a1 (4 <= col < 8)
          const int src = ((col & 3) * 16 + 4 * q + kk) * 4;
          const float t0 = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(a0s[bi])));
          float bval = t0;
          if (KD == 8) {
            const float t1 = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(a1s[bi])));
            bval = col < 4 ? t0 : t1;
          }
          const int lab = lab_s[wave][4 * q + kk];   // label of row 4q + kk
          const int64_t rb = row0 + 4 * q + kk;
          const bool valid = rb < n && (elig == nullptr || elig[rb] != 0);
          if (col >= KD) bval = 0.f;
          if (col == KD) bval = 1.f;
          if (!valid) bval = 0.f;
#pragma unroll
          for (int jt = 0; jt < KT; ++jt) {
            const float aval = (valid && lab == jt * 16 + col) ? 1.f : 0.f;
            uacc[jt] = __builtin_amdgcn_mfma_f32_16x16x4f32(aval, bval, uacc[jt], 0, 0, 0);
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  }

  if (UPDATE && count) {
    changed = wave_sum_i32(changed);
    if (lane == 0 && changed > 0) atomicAdd(J.conv, changed);
  }
  if constexpr (UPDATE) {
    // uacc[jt][r] = sum over this wave's rows for centre jt*16 + 4*kk + r, dim col
    if (col <= KD) {
#pragma unroll
      for (int jt = 0; jt < KT; ++jt)
#pragma unroll
        for (int r = 0; r < 4; ++r) wsum[wave][jt * 16 + 4 * kk + r][col] = uacc[jt][r];
    }
    __syncthreads();
    const int O = k * (KD + 1);
    double* cpart = J.cpart;
    for (int o = threadIdx.x; o < O; o += kLB) {
      const int j = o / (KD + 1), d = o % (KD + 1);
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kLW; ++w) s += (double)wsum[w][j][d];
      cpart[(int64_t)blk * O + o] = s;
    }
  }
}

// Centre update of a Lloyd step: the per-block sums of the step's kernel,
// added in a fixed order, then the means (one block per job, launched after
// the step on the same stream, so no block of the step waits on a
// device-scope fence).
__device__ void lloyd_finish(const KmJob& J, double* tot, double* part) {
  const int KD = J.KD, k = J.k;
  const int O = k * (KD + 1);
  const double* cpart = J.cpart;
  // outputs o < O; each summed by S threads over interleaved block subsets,
  // the S partial sums then combined in subset order
  const int nblk = J.nblk_ll;
  for (int o0 = 0; o0 < O; o0 += kLB) {
    const int cnt = min(kLB, O - o0);
    const int S = kLB / cnt;
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
  for (int o = threadIdx.x; o < k * KD; o += kLB) {
    const int j = o / KD, d = o % KD;
    const double cnt = tot[j * (KD + 1) + KD];
    if (cnt > 0.0) J.centres[j * KD + d] = (float)(tot[j * (KD + 1) + d] / cnt);
  }
}

// ---------------------------------------------------------------------------
// Kernels: one job, or many jobs in one grid
// ---------------------------------------------------------------------------
template <int KD>
__global__ __launch_bounds__(kKB) void kpp_kernel(KmJob J, int r) {
  __shared__ KppShared sh;
  kpp_block<KD>(J, blockIdx.x, r, sh);
}

template <int KD>
__global__ __launch_bounds__(kKB) void kpp_pick_kernel(KmJob J, int r) {
  __shared__ KppShared sh;
  kpp_pick_block<KD>(J, blockIdx.x, r, sh);
}

template <int KD>
__global__ __launch_bounds__(kKB) void kpp_sample_kernel(KmJob J, int r) {
  __shared__ KppShared sh;
  kpp_sample_block<KD>(J, r, blockIdx.x, sh);
}

__global__ __launch_bounds__(kKB) void kpp_select_kernel(KmJob J, int r) {
  __shared__ KppShared sh;
  kpp_select_block(J, r, sh);
}

// Step `it` of Lloyd (the final assignment when !UPDATE); a converged job
// returns at once.
template <int KD, int KT, bool UPDATE>
__global__ __launch_bounds__(kLB) void lloyd_kernel(KmJob J, int it) {
  __shared__ LloydShared sh;
  if (UPDATE && J.conv[1]) return;
  lloyd_block<KD, KT, UPDATE>(J, blockIdx.x, sh, it > 0);
}

// The centre update of step `it`, then the convergence state: a counted step
// that changed no label marks the job converged; the count restarts at 0.
__device__ void lloyd_finish_step(const KmJob& J, int it, double* tot, double* part) {
  if (J.conv[1]) return;
  lloyd_finish(J, tot, part);
  if (threadIdx.x == 0) {
    if (it > 0 && J.conv[0] == 0) J.conv[1] = 1;
    J.conv[0] = 0;
  }
}

__global__ __launch_bounds__(kLB) void lloyd_finish_kernel(KmJob J, int it) {
  __shared__ double tot[kMaxK * 9];
  __shared__ double part[kLB];
  lloyd_finish_step(J, it, tot, part);
}

// Clears the convergence state of every job before the Lloyd steps.
__global__ void kmeans_conv_reset(const KmJob* __restrict__ jobs, int njobs) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < njobs) {
    jobs[g].conv[0] = 0;
    jobs[g].conv[1] = 0;
  }
}

__device__ __forceinline__ int find_job(const int32_t* off, int njobs, int b) {
  int lo = 0, hi = njobs;  // off[0] = 0, off[njobs] = total
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kKB) void kpp_kernel_seg(const KmJob* __restrict__ jobs, const int32_t* __restrict__ off,
                                                      int njobs, int r) {
  __shared__ KppShared sh;
  const int g = find_job(off, njobs, blockIdx.x);
  const KmJob J = jobs[g];
  if (r >= J.k) return;
  const int b = blockIdx.x - off[g];
  if (J.KD == 4) kpp_block<4>(J, b, r, sh);
  else kpp_block<8>(J, b, r, sh);
}

// One block per (job, candidate): block b is candidate b % kMaxTrials of job
// b / kMaxTrials.
__global__ __launch_bounds__(kKB) void kpp_sample_kernel_seg(const KmJob* __restrict__ jobs, int r) {
  __shared__ KppShared sh;
  const KmJob J = jobs[blockIdx.x / kMaxTrials];
  if (r >= J.k) return;
  const int j = blockIdx.x % kMaxTrials;
  if (J.KD == 4) kpp_sample_block<4>(J, r, j, sh);
  else kpp_sample_block<8>(J, r, j, sh);
}

__global__ __launch_bounds__(kKB) void kpp_select_kernel_seg(const KmJob* __restrict__ jobs, int r) {
  __shared__ KppShared sh;
  const KmJob J = jobs[blockIdx.x];
  if (r >= J.k) return;
  kpp_select_block(J, r, sh);
}

__global__ __launch_bounds__(kKB) void kpp_pick_kernel_seg(const KmJob* __restrict__ jobs,
                                                           const int32_t* __restrict__ off, int njobs, int r) {
  __shared__ KppShared sh;
  const int g = find_job(off, njobs, blockIdx.x);
  const KmJob J = jobs[g];
  if (r >= J.k) return;
  const int b = blockIdx.x - off[g];
  if (J.KD == 4) kpp_pick_block<4>(J, b, r, sh);
  else kpp_pick_block<8>(J, b, r, sh);
}

template <bool UPDATE>
__global__ __launch_bounds__(kLB) void lloyd_kernel_seg(const KmJob* __restrict__ jobs,
                                                        const int32_t* __restrict__ off, int njobs, int it) {
  __shared__ LloydShared sh;
  const int g = find_job(off, njobs, blockIdx.x);
  const KmJob J = jobs[g];
  if (UPDATE && J.conv[1]) return;
  const int b = blockIdx.x - off[g];
  const int KT = (J.k + 15) / 16;
  const bool count = it > 0;
  if (J.KD == 4) {
    if (KT == 1) lloyd_block<4, 1, UPDATE>(J, b, sh, count);
    else if (KT == 2) lloyd_block<4, 2, UPDATE>(J, b, sh, count);
    else lloyd_block<4, 4, UPDATE>(J, b, sh, count);
  } else {
    if (KT == 1) lloyd_block<8, 1, UPDATE>(J, b, sh, count);
    else if (KT == 2) lloyd_block<8, 2, UPDATE>(J, b, sh, count);
    else lloyd_block<8, 4, UPDATE>(J, b, sh, count);
  }
}

// One block per job.
__global__ __launch_bounds__(kLB) void lloyd_finish_kernel_seg(const KmJob* __restrict__ jobs, int it) {
  __shared__ double tot[kMaxK * 9];
  __shared__ double part[kLB];
  lloyd_finish_step(jobs[blockIdx.x], it, tot, part);
}

// Normalised k-means cost of the final assignment over the eligible rows:
// out[0] = sum ||p - mu_label||^2 / sum ||p - mean||^2 (FP64 partials, the
// last block combines them in block order).
__global__ __launch_bounds__(kKB) void kmeans_cost_kernel(KmJob J, double* __restrict__ partials,
                                                          int32_t* __restrict__ counter, double* __restrict__ out) {
  __shared__ double red[kKB / FSC_WAVE];
  __shared__ int is_last;
  double cost = 0.0, sq = 0.0, cnt = 0.0, s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t v = (int64_t)blockIdx.x * kKB + threadIdx.x; v < J.n; v += (int64_t)gridDim.x * kKB) {
    if (J.elig && !J.elig[v]) continue;
    const int lab = J.labels[v];
    for (int q = 0; q < J.KD; ++q) {
      const double x = J.pts[v * J.KD + q];
      const double e = x - (double)J.centres[lab * J.KD + q];
      cost += e * e;
      sq += x * x;
      s[q] += x;
    }
    cnt += 1.0;
  }
  double vals[11] = {cost, sq, cnt, s[0], s[1], s[2], s[3], s[4], s[5], s[6], s[7]};
  for (int i = 0; i < 11; ++i) {
    const double t = block_sum<kKB>(vals[i], red);
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 11 + i] = t;
  }
  if (threadIdx.x == 0) {
    __threadfence();
    is_last = atomicAdd(counter, 1) == (int)gridDim.x - 1;
  }
  __syncthreads();
  if (!is_last || threadIdx.x != 0) return;
  __threadfence();
  double tot[11] = {0};
  for (int g = 0; g < (int)gridDim.x; ++g)
    for (int i = 0; i < 11; ++i) tot[i] += partials[(int64_t)g * 11 + i];
  double var = tot[1];
  if (tot[2] > 0.0)
    for (int q = 0; q < 8; ++q) var -= tot[3 + q] * tot[3 + q] / tot[2];
  out[0] = var > 0.0 ? tot[0] / var : 1.0;
  *counter = 0;
}

int kmeans_cost_run(Context* ctx, const KmeansIO* io, double* partials, int32_t* counter, double* out,
                    hipStream_t s) {
  const KmJob J = make_job(ctx, io);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((io->n + kKB - 1) / kKB, 2 * ctx->num_cu));
  hipLaunchKernelGGL(kmeans_cost_kernel, dim3(grid), dim3(kKB), 0, s, J, partials, counter, out);
  return check_hip(hipGetLastError(), "kmeans cost launch");
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

// ===========================================================================
// Host side
// ===========================================================================
// Lloyd launch shape for n points: tiles of 16 rows, blocks of 16 waves, about
// one block per CU and at least one tile per wave.
int kpp_trials(int k) { return std::min(kMaxTrials, 2 + (int)std::floor(std::log((double)std::max(k, 1)))); }

void kmeans_shape(int64_t n, int num_cu, int* nblk_pp, int* nblk_ll, int* tpw) {
  *nblk_pp = (int)((n + kKB * kRPT - 1) / (kKB * kRPT));
  const int64_t tiles = (n + 15) / 16;
  // at most one block per CU, and at least 8 tiles per wave so that small
  // problems do not pay a block's fixed reduction cost many times over
  int64_t blocks = std::min<int64_t>(num_cu, (tiles + 8 * kLW - 1) / (8 * kLW));
  if (blocks < 1) blocks = 1;
  int64_t t = (tiles + blocks * kLW - 1) / (blocks * kLW);
  blocks = (tiles + t * kLW - 1) / (t * kLW);
  *nblk_ll = (int)blocks;
  *tpw = (int)t;
}

size_t kmeans_workspace_bytes(int64_t n, int KD) {
  const int64_t nblk_pp = (n + kKB * kRPT - 1) / (kKB * kRPT);
  const int64_t nblk_ll = (n + 15) / 16 / kLW + 1;  // upper bound
  size_t b = 0;
  b += align_up(n * 4);                                   // d2
  b += align_up(nblk_pp * kMaxTrials * 8);                // bsum: block sums, or per-candidate potentials
  b += align_up(kMaxTrials * KD * 4) + align_up(kMaxTrials * 4);  // candidates
  b += align_up(kMaxK * KD * 4);                          // centres
  b += align_up((size_t)nblk_ll * kMaxK * (KD + 1) * 8);  // cpart
  b += align_up(kMaxK * 4);                               // chosen
  b += align_up(4 * 4);                                   // conv
  return b + 8 * 256;
}

int kmeans_bind_workspace(Arena* a, KmeansIO* io) {
  const int64_t n = io->n;
  io->nblk_pp = (int)((n + kKB * kRPT - 1) / (kKB * kRPT));
  io->d2 = a->take<float>(n);
  io->bsum = a->take<double>((size_t)io->nblk_pp * kMaxTrials);
  io->cand = a->take<float>(kMaxTrials * io->KD);
  io->cand_row = a->take<int32_t>(kMaxTrials);
  io->centres = a->take<float>(kMaxK * io->KD);
  io->cpart = a->take<double>((size_t)((n + 15) / 16 / kLW + 1) * kMaxK * (io->KD + 1));
  io->chosen = a->take<int32_t>(kMaxK);
  io->conv = a->take<int32_t>(4);
  if (a->used > a->size) return fail(FSC_E_NOMEM, "workspace arena too small");
  return FSC_OK;
}

KmJob make_job(Context* ctx, const KmeansIO* io) {
  KmJob J;
  J.n = io->n;
  J.pts = io->pts;
  J.elig = io->elig;
  J.KD = io->KD;
  J.k = io->k;
  J.d2 = io->d2;
  J.bsum = io->bsum;
  J.cand = io->cand;
  J.cand_row = io->cand_row;
  J.trials = kpp_trials(io->k);
  J.centres = io->centres;
  J.chosen = io->chosen;
  J.labels = io->labels;
  J.cpart = io->cpart;
  J.k0 = (uint32_t)(io->seed & 0xffffffffu);
  J.k1 = (uint32_t)(io->seed >> 32);
  J.conv = io->conv;
  kmeans_shape(io->n, ctx->num_cu, &J.nblk_pp, &J.nblk_ll, &J.tpw);
  return J;
}

template <int KD, int KT>
static int lloyd_all(const KmJob& J, int iters, hipStream_t s) {
  int rc;
  if ((rc = fill_zero_i32(J.conv, 4, s))) return rc;
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL((lloyd_kernel<KD, KT, true>), dim3(J.nblk_ll), dim3(kLB), 0, s, J, it);
    hipLaunchKernelGGL(lloyd_finish_kernel, dim3(1), dim3(kLB), 0, s, J, it);
  }
  hipLaunchKernelGGL((lloyd_kernel<KD, KT, false>), dim3(J.nblk_ll), dim3(kLB), 0, s, J, iters);
  return check_hip(hipGetLastError(), "lloyd_kernel launch");
}

template <int KD>
static int kmeans_typed(Context* ctx, KmeansIO* io, hipStream_t s) {
  const KmJob J = make_job(ctx, io);
  for (int r = 0; r < io->k; ++r) {
    hipLaunchKernelGGL(kpp_kernel<KD>, dim3(J.nblk_pp), dim3(kKB), 0, s, J, r);
    hipLaunchKernelGGL(kpp_sample_kernel<KD>, dim3(r == 0 ? 1 : J.trials), dim3(kKB), 0, s, J, r);
    if (r > 0) {
      hipLaunchKernelGGL(kpp_pick_kernel<KD>, dim3(J.nblk_pp), dim3(kKB), 0, s, J, r);
      hipLaunchKernelGGL(kpp_select_kernel, dim3(1), dim3(kKB), 0, s, J, r);
    }
  }
  int rc = check_hip(hipGetLastError(), "kpp_kernel launch");
  if (rc) return rc;
  const int KT = (io->k + 15) / 16;
  switch (KT) {
    case 1: rc = lloyd_all<KD, 1>(J, io->iters, s); break;
    case 2: rc = lloyd_all<KD, 2>(J, io->iters, s); break;
    case 3: rc = lloyd_all<KD, 3>(J, io->iters, s); break;
    default: rc = lloyd_all<KD, 4>(J, io->iters, s); break;
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

int kmeans_run_batched(Context* ctx, const KmJob* jobs_dev, const int32_t* pp_off_dev, int pp_total,
                       const int32_t* ll_off_dev, int ll_total, int njobs, int kmax, int iters, hipStream_t s) {
  for (int r = 0; r < kmax; ++r) {
    hipLaunchKernelGGL(kpp_kernel_seg, dim3(pp_total), dim3(kKB), 0, s, jobs_dev, pp_off_dev, njobs, r);
    hipLaunchKernelGGL(kpp_sample_kernel_seg, dim3(njobs * kMaxTrials), dim3(kKB), 0, s, jobs_dev, r);
    if (r > 0) {
      hipLaunchKernelGGL(kpp_pick_kernel_seg, dim3(pp_total), dim3(kKB), 0, s, jobs_dev, pp_off_dev, njobs, r);
      hipLaunchKernelGGL(kpp_select_kernel_seg, dim3(njobs), dim3(kKB), 0, s, jobs_dev, r);
    }
  }
  hipLaunchKernelGGL(kmeans_conv_reset, dim3((njobs + 255) / 256), dim3(256), 0, s, jobs_dev, njobs);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL(lloyd_kernel_seg<true>, dim3(ll_total), dim3(kLB), 0, s, jobs_dev, ll_off_dev, njobs, it);
    hipLaunchKernelGGL(lloyd_finish_kernel_seg, dim3(njobs), dim3(kLB), 0, s, jobs_dev, it);
  }
  hipLaunchKernelGGL(lloyd_kernel_seg<false>, dim3(ll_total), dim3(kLB), 0, s, jobs_dev, ll_off_dev, njobs, iters);
  return check_hip(hipGetLastError(), "batched k-means launch");
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
