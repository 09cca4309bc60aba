// The MLP of the learned form: 9 features -> 3 hidden layers of 128 (ReLU)
// -> 2 outputs (alpha, beta), in FP32, with hand-written forward, backward
// and Adam kernels, and the fixed head that turns the outputs into the
// filter's coefficients.
//
// The head: the outputs fix an interval [a, b] of the spectrum to damp,
// b = 1 - e^beta and a = b - e^alpha (so a < b < 1), and the filter is the
// Chebyshev polynomial of that interval normalised to p(1) = 1,
// p(gamma) = T_8(u(gamma)) / T_8(u(1)), u = (2 gamma - a - b) / (b - a): the
// degree-8 polynomial with the smallest maximum on [a, b] among those with
// p(1) = 1.  With x = 2 gamma - 1, u = s x + r (s = 1 / (b - a),
// r = (1 - a - b) / (b - a)), and the coefficients of T_8(s x + r) in the
// T_j(x) = T*_j(gamma) basis follow from the three-term recurrence applied to
// Chebyshev series, P_{m+1} = 2 (r + s x) P_m - P_{m-1}, with
// x T_0 = T_1 and x T_j = (T_{j+1} + T_{j-1}) / 2; their derivatives in s
// and r are carried along the same recurrence (forward mode), in FP64.
//
// Parameters are one flat FP32 array: for each layer, W (out x in, row-major)
// then b (out).  The training loss of a graph is the normalised k-means cost
// (Sec. 2.2) of its filtered embedding under the plain method's labels:
// within-cluster over total scatter, q^T W q / q^T T q in its FP64 scatter
// statistics (the ratio does not depend on the scale of the coefficients q);
// the batch loss is the mean.  Every reduction runs in a fixed order, so
// training is deterministic.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>

namespace fsc {

constexpr int kNF = 9, kH = 128, kNO = 2;
constexpr int kLayerIn[4] = {kNF, kH, kH, kH};
constexpr int kLayerOut[4] = {kH, kH, kH, kNO};

int mlp_param_count() {
  int c = 0;
  for (int i = 0; i < 4; ++i) c += kLayerIn[i] * kLayerOut[i] + kLayerOut[i];
  return c;
}

static int layer_offset(int li) {
  int c = 0;
  for (int i = 0; i < li; ++i) c += kLayerIn[i] * kLayerOut[i] + kLayerOut[i];
  return c;
}

// out[b][o] = act(sum_i in[b][i] W[o][i] + bias[o]), one thread per (b, o).
__global__ void mlp_fwd_kernel(const float* __restrict__ W, const float* __restrict__ bias,
                               const float* __restrict__ in, float* __restrict__ out, int B, int nin, int nout,
                               int relu) {
  const int64_t total = (int64_t)B * nout;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(i / nout), o = (int)(i % nout);
    const float* x = in + (int64_t)b * nin;
    const float* w = W + (int64_t)o * nin;
    float s = bias[o];
    for (int k = 0; k < nin; ++k) s += x[k] * w[k];
    out[i] = relu ? fmaxf(s, 0.f) : s;
  }
}

// x * P for a Chebyshev series P of degree < 9 (result truncated to 9 terms;
// the recurrence below never needs a term beyond T_8).
__device__ __forceinline__ void cheb_mulx(const double* p, double* out) {
#pragma unroll
  for (int j = 0; j < 9; ++j) out[j] = 0.0;
  out[1] += p[0];
#pragma unroll
  for (int j = 1; j < 9; ++j) {
    if (j + 1 < 9) out[j + 1] += 0.5 * p[j];
    out[j - 1] += 0.5 * p[j];
  }
}

// q (9 coefficients of T_8(u) in the T*_j basis) and dq/dalpha, dq/dbeta.
__device__ void interval_head(double alpha, double beta, double* q, double* dqa, double* dqb) {
  const double eb = exp(beta), ea = exp(alpha);
  const double b = 1.0 - eb, a = b - ea;
  const double w = b - a;
  const double s = 1.0 / w, r = (1.0 - a - b) / w;
  // P_{m-1}, P_m and their s- and r-derivatives
  double p0[9], p1[9], s0[9], s1[9], r0[9], r1[9];
#pragma unroll
  for (int j = 0; j < 9; ++j) p0[j] = p1[j] = s0[j] = s1[j] = r0[j] = r1[j] = 0.0;
  p0[0] = 1.0;
  p1[0] = r;
  p1[1] = s;
  s1[1] = 1.0;
  r1[0] = 1.0;
  for (int m = 1; m < 8; ++m) {
    double xp[9], xs[9], xr[9];
    cheb_mulx(p1, xp);
    cheb_mulx(s1, xs);
    cheb_mulx(r1, xr);
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      // P' = 2 (r P + s xP) - P0;  dP'/ds = 2 (xP + r dP/ds + s x dP/ds) - dP0/ds;
      // dP'/dr = 2 (P + r dP/dr + s x dP/dr) - dP0/dr
      const double pn = 2.0 * (r * p1[j] + s * xp[j]) - p0[j];
      const double sn = 2.0 * (xp[j] + r * s1[j] + s * xs[j]) - s0[j];
      const double rn = 2.0 * (p1[j] + r * r1[j] + s * xr[j]) - r0[j];
      p0[j] = p1[j];
      s0[j] = s1[j];
      r0[j] = r1[j];
      p1[j] = pn;
      s1[j] = sn;
      r1[j] = rn;
    }
  }
  const double w2 = w * w;
  const double ds_da = 1.0 / w2, ds_db = -1.0 / w2;
  const double dr_da = (1.0 - 2.0 * b) / w2, dr_db = (2.0 * a - 1.0) / w2;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const double dqda = s1[j] * ds_da + r1[j] * dr_da;
    const double dqdb = s1[j] * ds_db + r1[j] * dr_db;
    q[j] = p1[j];
    dqa[j] = dqda * (-ea);            // a = b - e^alpha
    dqb[j] = (dqda + dqdb) * (-eb);   // b = 1 - e^beta moves a as well
  }
}

// c_1..c_8 = q_1..q_8 / p_q(1), p_q(1) = sum_j q_j, one thread per row.
__global__ void mlp_head_kernel(const float* __restrict__ raw, int B, float* __restrict__ c_out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double q[9], qa[9], qb[9];
  interval_head((double)raw[b * 2], (double)raw[b * 2 + 1], q, qa, qb);
  double sum = 0.0;
  for (int j = 0; j < 9; ++j) sum += q[j];
  for (int j = 0; j < 8; ++j) c_out[b * 8 + j] = (float)(q[j + 1] / sum);
}

// Per-graph loss L = q^T W q / q^T T q and dL/d(alpha, beta) / B (FP64 from
// the FP32 outputs): dL/dq = 2 (W q - L T q) / q^T T q, then the head's
// derivatives.  A graph with q^T T q = 0 (all its rows equal) has no defined
// ratio and contributes 0 with a zero gradient.
__global__ void mlp_loss_kernel(const float* __restrict__ raw, const double* __restrict__ W,
                                const double* __restrict__ T, int B, float* __restrict__ delta,
                                double* __restrict__ loss_per) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double q[9], qa[9], qb[9];
  interval_head((double)raw[b * 2], (double)raw[b * 2 + 1], q, qa, qb);
  const double* Wb = W + (int64_t)b * 81;
  const double* Tb = T + (int64_t)b * 81;
  double Wq[9], Tq[9];
  double num = 0.0, den = 0.0;
  for (int i = 0; i < 9; ++i) {
    double sw = 0.0, st = 0.0;
    for (int j = 0; j < 9; ++j) {
      sw += Wb[i * 9 + j] * q[j];
      st += Tb[i * 9 + j] * q[j];
    }
    Wq[i] = sw;
    Tq[i] = st;
    num += q[i] * sw;
    den += q[i] * st;
  }
  if (!(den > 0.0)) {
    loss_per[b] = 0.0;
    delta[b * 2] = delta[b * 2 + 1] = 0.f;
    return;
  }
  const double L = num / den;
  loss_per[b] = L;
  double ga = 0.0, gb = 0.0;
  for (int j = 0; j < 9; ++j) {
    const double gq = 2.0 * (Wq[j] - L * Tq[j]) / den;
    ga += gq * qa[j];
    gb += gq * qb[j];
  }
  delta[b * 2] = (float)(ga / (double)B);
  delta[b * 2 + 1] = (float)(gb / (double)B);
}

// gW[o][i] = sum_b delta[b][o] in[b][i];  gb[o] = sum_b delta[b][o].
__global__ void mlp_wgrad_kernel(const float* __restrict__ delta, const float* __restrict__ in, float* __restrict__ gW,
                                 float* __restrict__ gb, int B, int nin, int nout) {
  const int64_t total = (int64_t)nout * (nin + 1);
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int o = (int)(t / (nin + 1)), i = (int)(t % (nin + 1));
    float s = 0.f;
    if (i < nin) {
      for (int b = 0; b < B; ++b) s += delta[(int64_t)b * nout + o] * in[(int64_t)b * nin + i];
      gW[(int64_t)o * nin + i] = s;
    } else {
      for (int b = 0; b < B; ++b) s += delta[(int64_t)b * nout + o];
      gb[o] = s;
    }
  }
}

// din[b][i] = (sum_o delta[b][o] W[o][i]) * (act[b][i] > 0).
__global__ void mlp_dgrad_kernel(const float* __restrict__ delta, const float* __restrict__ W,
                                 const float* __restrict__ act, float* __restrict__ din, int B, int nin, int nout) {
  const int64_t total = (int64_t)B * nin;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int b = (int)(t / nin), i = (int)(t % nin);
    float s = 0.f;
    for (int o = 0; o < nout; ++o) s += delta[(int64_t)b * nout + o] * W[(int64_t)o * nin + i];
    din[t] = act[t] > 0.f ? s : 0.f;
  }
}

// Adam (Kingma and Ba), bias-corrected, FP32 state.
__global__ void mlp_adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                const float* __restrict__ g, int count, float lr, float b1, float b2, float eps,
                                float corr1, float corr2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / corr1) / (sqrtf(vi / corr2) + eps);
}

// Mean of the per-graph losses in a fixed order (one block).
__global__ void mlp_loss_mean_kernel(const double* __restrict__ loss_per, int B, double* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) s += loss_per[b];
  s = block_sum<256>(s, red);
  if (threadIdx.x == 0) *out = s / B;
}

static int grid_of(int64_t work) { return (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 4096)); }

size_t mlp_workspace_bytes(int B) {
  size_t b = 0;
  b += align_up((size_t)B * (kNF + 3 * kH + kNO) * 4);  // activations
  b += 2 * align_up((size_t)B * kH * 4);                // deltas
  b += align_up((size_t)B * 8);                         // per-graph loss
  return b + 1024;
}

// acts: a1, a2, a3 (B x 128); raw: the outputs (B x 2)
int mlp_forward_run(const float* params, int B, const float* feats, float* acts, float* raw, hipStream_t s) {
  const float* in = feats;
  float* a = acts;
  for (int li = 0; li < 4; ++li) {
    const float* W = params + layer_offset(li);
    const float* bias = W + kLayerIn[li] * kLayerOut[li];
    float* out = li < 3 ? a : raw;
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(grid_of((int64_t)B * kLayerOut[li])), dim3(256), 0, s, W, bias, in, out,
                       B, kLayerIn[li], kLayerOut[li], li < 3 ? 1 : 0);
    in = out;
    a += (int64_t)B * kH;
  }
  return check_hip(hipGetLastError(), "mlp forward launch");
}

// The filter coefficients c_1..c_8 (B x 8) for B feature rows; ws holds
// mlp_workspace_bytes(B).
int mlp_coefficients_run(const float* params, int B, const float* feats, char* ws, float* c_out, hipStream_t s) {
  float* acts = reinterpret_cast<float*>(ws);
  float* raw = acts + (int64_t)B * 3 * kH;
  int rc = mlp_forward_run(params, B, feats, acts, raw, s);
  if (rc) return rc;
  hipLaunchKernelGGL(mlp_head_kernel, dim3((B + 255) / 256), dim3(256), 0, s, raw, B, c_out);
  return check_hip(hipGetLastError(), "mlp head launch");
}

int mlp_loss_grad_run(const float* params, int B, const float* feats, const double* W, const double* T,
                      float* grad, double* loss_out, char* ws, hipStream_t s) {
  Arena a;
  a.base = ws;
  a.size = mlp_workspace_bytes(B);
  a.used = 0;
  float* acts = a.take<float>((size_t)B * 3 * kH);
  float* c = a.take<float>((size_t)B * kNO);
  float* d0 = a.take<float>((size_t)B * kH);
  float* d1 = a.take<float>((size_t)B * kH);
  double* lp = a.take<double>(B);
  int rc = mlp_forward_run(params, B, feats, acts, c, s);
  if (rc) return rc;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3((B + 255) / 256), dim3(256), 0, s, c, W, T, B, d0, lp);
  hipLaunchKernelGGL(mlp_loss_mean_kernel, dim3(1), dim3(256), 0, s, lp, B, loss_out);
  // backward: layer 3 (delta d0 is B x 2) down to layer 0
  float* delta = d0;
  float* other = d1;
  for (int li = 3; li >= 0; --li) {
    const float* in = li == 0 ? feats : acts + (int64_t)(li - 1) * B * kH;
    float* gW = grad + layer_offset(li);
    float* gb = gW + kLayerIn[li] * kLayerOut[li];
    hipLaunchKernelGGL(mlp_wgrad_kernel, dim3(grid_of((int64_t)kLayerOut[li] * (kLayerIn[li] + 1))), dim3(256), 0, s,
                       delta, in, gW, gb, B, kLayerIn[li], kLayerOut[li]);
    if (li > 0) {
      const float* W = params + layer_offset(li);
      hipLaunchKernelGGL(mlp_dgrad_kernel, dim3(grid_of((int64_t)B * kLayerIn[li])), dim3(256), 0, s, delta, W, in,
                         other, B, kLayerIn[li], kLayerOut[li]);
      std::swap(delta, other);
    }
  }
  return check_hip(hipGetLastError(), "mlp backward launch");
}

int mlp_adam_run(float* p, float* m, float* v, const float* g, float lr, int step, hipStream_t s) {
  const int count = mlp_param_count();
  const float b1 = 0.9f, b2 = 0.999f;
  const float corr1 = 1.f - std::pow(b1, (float)step), corr2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, m, v, g, count, lr, b1, b2, 1e-8f,
                     corr1, corr2);
  return check_hip(hipGetLastError(), "adam launch");
}

}  // namespace fsc
