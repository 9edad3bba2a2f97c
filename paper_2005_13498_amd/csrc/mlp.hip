// FP32 multilayer perceptron of the learned Krylov controller:
//   x (8) -> 64 -> GELU -> 64 -> GELU -> 2  (exact erf GELU),
// forward, gradient of the mean squared error, and Adam.  One wavefront per
// row: lane k owns hidden unit k of both layers, so the 64-wide hidden
// layers map one to one onto a CDNA wavefront; the previous layer's
// activations are broadcast with lane reads.  Gradient partial sums are
// kept per wavefront and reduced by the Adam kernel in a fixed order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hub.h"
#include "mlp.h"

namespace hub {
namespace dev {

constexpr int kIn = HUB_MLP_IN, kHid = HUB_MLP_HID, kOut = HUB_MLP_OUT, kP = HUB_MLP_NPARAM;
constexpr int oW1 = 0, oB1 = oW1 + kHid * kIn, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid, oW3 = oB2 + kHid,
              oB3 = oW3 + kOut * kHid;
static_assert(oB3 + kOut == kP, "parameter layout");
constexpr int kMlpBlock = 256, kMlpWaves = kMlpBlock / 64;
constexpr int kMaxGradWaves = 256;  // wavefronts (gradient partial rows) of one train step
constexpr int kGradStride = kP + 1;  // per-wave partial: gradient, then the loss

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}
__device__ __forceinline__ float lane_bcast(float v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per-lane parameter slice: lane k holds row k of W1 and W2, column k of W3.
struct Slice {
  float w1[kIn], b1, w2[kHid], b2, w3[kOut], b3[kOut];
};

__device__ __forceinline__ void load_slice(const float* __restrict__ P, int k, Slice& S) {
#pragma unroll
  for (int i = 0; i < kIn; ++i) S.w1[i] = P[oW1 + k * kIn + i];
  S.b1 = P[oB1 + k];
#pragma unroll
  for (int j = 0; j < kHid; ++j) S.w2[j] = P[oW2 + k * kHid + j];
  S.b2 = P[oB2 + k];
#pragma unroll
  for (int o = 0; o < kOut; ++o) {
    S.w3[o] = P[oW3 + o * kHid + k];
    S.b3[o] = P[oB3 + o];
  }
}

// Forward of one row on one wavefront; every lane ends with both outputs.
__device__ __forceinline__ void forward_row(const Slice& S, const float* __restrict__ x, float& z1, float& h1,
                                            float& z2, float& h2, float (&out)[kOut]) {
  float xi[kIn];
#pragma unroll
  for (int i = 0; i < kIn; ++i) xi[i] = x[i];
  z1 = S.b1;
#pragma unroll
  for (int i = 0; i < kIn; ++i) z1 = fmaf(S.w1[i], xi[i], z1);
  h1 = gelu(z1);
  z2 = S.b2;
#pragma unroll
  for (int j = 0; j < kHid; ++j) z2 = fmaf(S.w2[j], lane_bcast(h1, j), z2);
  h2 = gelu(z2);
#pragma unroll
  for (int o = 0; o < kOut; ++o) out[o] = wave_sum_f(S.w3[o] * h2) + S.b3[o];
}

__global__ __launch_bounds__(kMlpBlock) void k_mlp_forward(const float* __restrict__ P, int n_rows,
                                                           const float* __restrict__ feats,
                                                           float* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * kMlpWaves + (threadIdx.x >> 6);
  const int nw = gridDim.x * kMlpWaves;
  Slice S;
  load_slice(P, lane, S);
  for (int r = wave; r < n_rows; r += nw) {
    float z1, h1, z2, h2, o[kOut];
    forward_row(S, feats + (size_t)r * kIn, z1, h1, z2, h2, o);
#pragma unroll
    for (int q = 0; q < kOut; ++q)
      if (lane == q) out[(size_t)r * kOut + q] = o[q];
  }
}

// Gradient partial sums of L = (1/n) sum_r |out_r - y_r|^2 for the rows of
// each wavefront, written to part[wave][kGradStride] (last entry: the
// wavefront's share of L).  W2 is staged in LDS for the backward pass
// through layer 2, which needs its columns.
__global__ __launch_bounds__(kMlpBlock) void k_mlp_grad(const float* __restrict__ P, int n_rows,
                                                        const float* __restrict__ feats,
                                                        const float* __restrict__ targets,
                                                        float* __restrict__ part) {
  __shared__ float w2s[kHid * kHid];
  for (int t = threadIdx.x; t < kHid * kHid; t += kMlpBlock) w2s[t] = P[oW2 + t];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * kMlpWaves + (threadIdx.x >> 6);
  const int nw = gridDim.x * kMlpWaves;
  Slice S;
  load_slice(P, lane, S);
  const float inv_n = 1.0f / static_cast<float>(n_rows);
  float gw1[kIn], gb1 = 0.f, gw2[kHid], gb2 = 0.f, gw3[kOut], gb3[kOut], loss = 0.f;
#pragma unroll
  for (int i = 0; i < kIn; ++i) gw1[i] = 0.f;
#pragma unroll
  for (int j = 0; j < kHid; ++j) gw2[j] = 0.f;
#pragma unroll
  for (int o = 0; o < kOut; ++o) {
    gw3[o] = 0.f;
    gb3[o] = 0.f;
  }
  for (int r = wave; r < n_rows; r += nw) {
    const float* x = feats + (size_t)r * kIn;
    float z1, h1, z2, h2, o[kOut];
    forward_row(S, x, z1, h1, z2, h2, o);
    float d[kOut];
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
      const float e = o[q] - targets[(size_t)r * kOut + q];
      loss += e * e * inv_n;
      d[q] = 2.0f * e * inv_n;  // dL/d out_q
    }
    float dh2 = 0.f;
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
      gw3[q] = fmaf(d[q], h2, gw3[q]);
      gb3[q] += d[q];
      dh2 = fmaf(S.w3[q], d[q], dh2);
    }
    const float dz2 = dh2 * gelu_d(z2);
    gb2 += dz2;
#pragma unroll
    for (int j = 0; j < kHid; ++j) gw2[j] = fmaf(dz2, lane_bcast(h1, j), gw2[j]);
    // lane j: dh1_j = sum_k W2[k][j] dz2_k
    float dh1 = 0.f;
#pragma unroll 8
    for (int k = 0; k < kHid; ++k) dh1 = fmaf(w2s[k * kHid + lane], lane_bcast(dz2, k), dh1);
    const float dz1 = dh1 * gelu_d(z1);
    gb1 += dz1;
#pragma unroll
    for (int i = 0; i < kIn; ++i) gw1[i] = fmaf(dz1, x[i], gw1[i]);
  }
  float* G = part + (size_t)wave * kGradStride;
#pragma unroll
  for (int i = 0; i < kIn; ++i) G[oW1 + lane * kIn + i] = gw1[i];
  G[oB1 + lane] = gb1;
#pragma unroll
  for (int j = 0; j < kHid; ++j) G[oW2 + lane * kHid + j] = gw2[j];
  G[oB2 + lane] = gb2;
#pragma unroll
  for (int q = 0; q < kOut; ++q) G[oW3 + q * kHid + lane] = gw3[q];
#pragma unroll
  for (int q = 0; q < kOut; ++q)
    if (lane == q) G[oB3 + q] = gb3[q];  // equal on every lane
  if (lane == 0) G[kP] = loss;                                   // equal on every lane
}

// Adam on the fixed-order sum of the wavefront partials; thread kP reports L.
__global__ __launch_bounds__(kMlpBlock) void k_mlp_adam(const float* __restrict__ part, int n_waves,
                                                        float* __restrict__ P, float* __restrict__ m,
                                                        float* __restrict__ v, int t, float lr,
                                                        float* __restrict__ loss) {
  const int p = blockIdx.x * kMlpBlock + threadIdx.x;
  if (p > kP) return;
  float g = 0.f;
  for (int w = 0; w < n_waves; ++w) g += part[(size_t)w * kGradStride + p];
  if (p == kP) {
    *loss = g;
    return;
  }
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mt = b1 * m[p] + (1.f - b1) * g;
  const float vt = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mt;
  v[p] = vt;
  const float mh = mt / (1.f - powf(b1, static_cast<float>(t)));
  const float vh = vt / (1.f - powf(b2, static_cast<float>(t)));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace dev

int mlp_grad_waves(int n_rows) {
  int w = (n_rows + 7) / 8;  // at least eight rows per wavefront
  w = w < 1 ? 1 : w;
  w = w > dev::kMaxGradWaves ? dev::kMaxGradWaves : w;
  return (w + dev::kMlpWaves - 1) / dev::kMlpWaves * dev::kMlpWaves;  // whole workgroups
}

int64_t mlp_workspace_bytes(int n_rows) {
  return static_cast<int64_t>(mlp_grad_waves(n_rows)) * dev::kGradStride * sizeof(float);
}

hipError_t launch_mlp_forward(const float* params, int n_rows, const float* feats, float* out, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  int grid = (n_rows + dev::kMlpWaves - 1) / dev::kMlpWaves;
  grid = grid > 1024 ? 1024 : grid;
  hipLaunchKernelGGL(dev::k_mlp_forward, dim3(grid), dim3(dev::kMlpBlock), 0, s, params, n_rows, feats, out);
  return hipGetLastError();
}

hipError_t launch_mlp_train_step(float* params, float* m, float* v, int t, float lr, int n_rows, const float* feats,
                                 const float* targets, float* loss, void* workspace, hipStream_t s) {
  const int waves = mlp_grad_waves(n_rows);
  float* part = static_cast<float*>(workspace);
  hipLaunchKernelGGL(dev::k_mlp_grad, dim3(waves / dev::kMlpWaves), dim3(dev::kMlpBlock), 0, s, params, n_rows,
                     feats, targets, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int grid = (dev::kP + 1 + dev::kMlpBlock - 1) / dev::kMlpBlock;
  hipLaunchKernelGGL(dev::k_mlp_adam, dim3(grid), dim3(dev::kMlpBlock), 0, s, part, waves, params, m, v, t, lr,
                     loss);
  return hipGetLastError();
}

}  // namespace hub
