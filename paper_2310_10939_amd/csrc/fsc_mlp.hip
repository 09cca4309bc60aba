// The MLP of the learned form: 9 features -> 3 hidden layers of 128 (ReLU)
// -> 8 filter coefficients c_1..c_8, in FP32, with hand-written forward,
// backward and Adam kernels.
//
// Parameters are one flat FP32 array: for each layer, W (out x in, row-major)
// then b (out).  The training loss of a graph is the normalised k-means cost
// (Sec. 2.2) of its filtered embedding under the plain method's labels:
// within-cluster over total scatter, c^T W c / c^T T c in its FP64 scatter
// statistics (c = (1 - sum c_rest, c_rest)); the batch loss is the mean.
// Every reduction runs in a fixed order, so training is deterministic.
#include "fsc_device.hpp"
#include "fsc_internal.hpp"

#include <algorithm>

namespace fsc {

constexpr int kNF = 9, kH = 128, kNO = 8;
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

// Per-graph loss L = c^T W c / c^T T c and dL/dc_rest / B (FP64 from the
// FP32 outputs): dL/dc = 2 (W c - L T c) / c^T T c, and c_0 = 1 - sum c_rest
// gives dL/dc_j - dL/dc_0.  A graph with c^T T c = 0 (all its rows equal)
// has no defined ratio and contributes 0 with a zero gradient.
__global__ void mlp_loss_kernel(const float* __restrict__ c_rest, const double* __restrict__ W,
                                const double* __restrict__ T, int B, float* __restrict__ delta,
                                double* __restrict__ loss_per) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double c[9];
  double sum = 0.0;
  for (int j = 0; j < 8; ++j) {
    c[j + 1] = (double)c_rest[b * 8 + j];
    sum += c[j + 1];
  }
  c[0] = 1.0 - sum;
  const double* Wb = W + (int64_t)b * 81;
  const double* Tb = T + (int64_t)b * 81;
  double Wc[9], Tc[9];
  double num = 0.0, den = 0.0;
  for (int i = 0; i < 9; ++i) {
    double sw = 0.0, st = 0.0;
    for (int j = 0; j < 9; ++j) {
      sw += Wb[i * 9 + j] * c[j];
      st += Tb[i * 9 + j] * c[j];
    }
    Wc[i] = sw;
    Tc[i] = st;
    num += c[i] * sw;
    den += c[i] * st;
  }
  if (!(den > 0.0)) {
    loss_per[b] = 0.0;
    for (int j = 0; j < 8; ++j) delta[b * 8 + j] = 0.f;
    return;
  }
  const double L = num / den;
  loss_per[b] = L;
  const double g0 = 2.0 * (Wc[0] - L * Tc[0]) / den;
  for (int j = 0; j < 8; ++j) {
    const double gj = 2.0 * (Wc[j + 1] - L * Tc[j + 1]) / den;
    delta[b * 8 + j] = (float)((gj - g0) / (double)B);
  }
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

// acts: x (B x 9), a1, a2, a3 (B x 128), c (B x 8)
int mlp_forward_run(const float* params, int B, const float* feats, float* acts, float* c_out, hipStream_t s) {
  const float* in = feats;
  float* a = acts;
  for (int li = 0; li < 4; ++li) {
    const float* W = params + layer_offset(li);
    const float* bias = W + kLayerIn[li] * kLayerOut[li];
    float* out = li < 3 ? a : c_out;
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(grid_of((int64_t)B * kLayerOut[li])), dim3(256), 0, s, W, bias, in, out,
                       B, kLayerIn[li], kLayerOut[li], li < 3 ? 1 : 0);
    in = out;
    a += (int64_t)B * kH;
  }
  return check_hip(hipGetLastError(), "mlp forward launch");
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
  // backward: layer 3 (delta d0 is B x 8) down to layer 0
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
