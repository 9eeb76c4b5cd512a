// The (k, q) predictor network and its training kernels (FP32).
//
// x (128 features) -> h1 = tanh(W1 x + b1) (64) -> h2 = tanh(W2 h1 + b2) (64)
// -> y = W3 h2 + b3 (4): y_q estimates log2 of the smallest sketch width k
// whose SOR-SVD with q power steps meets the tolerance, q = 0..3.
// Parameters are one flat FP32 vector: W1 (64 x 128, row-major), b1, W2
// (64 x 64), b2, W3 (4 x 64), b3 -- 12676 values.
//
// Loss of a minibatch of B samples: mean over the B x 4 outputs of
// (y - t)^2. The backward pass writes the gradient of that loss; every
// gradient entry is summed over the batch by one thread in sample order, so
// the result is deterministic. Adam (Kingma & Ba) updates the parameters.
#include <cmath>

#include "common.hpp"

namespace sor {

namespace {

constexpr int kIn = 128, kH = 64, kOut = 4;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;
static_assert(kParams == 12676, "parameter count");

// Work layout (floats) for a batch of B: H1 B x 64 | H2 B x 64 | Y B x 4 | DY B x 4 |
// D2 B x 64 | D1 B x 64 | per-sample loss B.
struct Work {
  float *H1, *H2, *Y, *DY, *D2, *D1, *lossb;
  __host__ __device__ Work(float* w, int B)
      : H1(w), H2(w + (size_t)B * kH), Y(w + (size_t)2 * B * kH), DY(w + (size_t)2 * B * kH + (size_t)B * kOut),
        D2(w + (size_t)2 * B * kH + (size_t)2 * B * kOut), D1(w + (size_t)3 * B * kH + (size_t)2 * B * kOut),
        lossb(w + (size_t)4 * B * kH + (size_t)2 * B * kOut) {}
};

// One workgroup of 64 threads per sample.
__global__ void __launch_bounds__(64) k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ X, int B,
                                                float* __restrict__ H1, float* __restrict__ H2,
                                                float* __restrict__ Y) {
  __shared__ float x[kIn], h1[kH], h2[kH];
  const int b = blockIdx.x, t = threadIdx.x;
  x[t] = X[(size_t)b * kIn + t];
  x[t + 64] = X[(size_t)b * kIn + 64 + t];
  __syncthreads();
  float s = P[oB1 + t];
  for (int j = 0; j < kIn; ++j) s += P[oW1 + t * kIn + j] * x[j];
  h1[t] = tanhf(s);
  H1[(size_t)b * kH + t] = h1[t];
  __syncthreads();
  s = P[oB2 + t];
  for (int j = 0; j < kH; ++j) s += P[oW2 + t * kH + j] * h1[j];
  h2[t] = tanhf(s);
  H2[(size_t)b * kH + t] = h2[t];
  __syncthreads();
  if (t < kOut) {
    s = P[oB3 + t];
    for (int j = 0; j < kH; ++j) s += P[oW3 + t * kH + j] * h2[j];
    Y[(size_t)b * kOut + t] = s;
  }
}

// Output and hidden-layer errors of one sample (64 threads per sample).
__global__ void __launch_bounds__(64) k_mlp_delta(const float* __restrict__ P, const float* __restrict__ T, int B,
                                                  Work w) {
  __shared__ float dy[kOut], d2[kH], lsum[kOut];
  const int b = blockIdx.x, t = threadIdx.x;
  const float scale = 1.0f / (float)(B * kOut);
  if (t < kOut) {
    const float r = w.Y[(size_t)b * kOut + t] - T[(size_t)b * kOut + t];
    dy[t] = 2.0f * r * scale;
    w.DY[(size_t)b * kOut + t] = dy[t];
    lsum[t] = r * r * scale;
  }
  __syncthreads();
  if (t == 0) w.lossb[b] = (lsum[0] + lsum[1]) + (lsum[2] + lsum[3]);
  const float h2 = w.H2[(size_t)b * kH + t];
  float s = 0.0f;
  for (int q = 0; q < kOut; ++q) s += P[oW3 + q * kH + t] * dy[q];
  d2[t] = s * (1.0f - h2 * h2);
  w.D2[(size_t)b * kH + t] = d2[t];
  __syncthreads();
  const float h1 = w.H1[(size_t)b * kH + t];
  s = 0.0f;
  for (int j = 0; j < kH; ++j) s += P[oW2 + j * kH + t] * d2[j];
  w.D1[(size_t)b * kH + t] = s * (1.0f - h1 * h1);
}

// One thread per parameter (and one more for the loss): sums over the batch in sample order.
__global__ void __launch_bounds__(256) k_mlp_grad(const float* __restrict__ X, int B, Work w,
                                                  float* __restrict__ G, float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p > kParams) return;
  float g = 0.0f;
  if (p == kParams) {
    for (int b = 0; b < B; ++b) g += w.lossb[b];
    *loss = g;
    return;
  }
  if (p < oB1) {
    const int i = p / kIn, j = p % kIn;
    for (int b = 0; b < B; ++b) g += w.D1[(size_t)b * kH + i] * X[(size_t)b * kIn + j];
  } else if (p < oW2) {
    const int i = p - oB1;
    for (int b = 0; b < B; ++b) g += w.D1[(size_t)b * kH + i];
  } else if (p < oB2) {
    const int i = (p - oW2) / kH, j = (p - oW2) % kH;
    for (int b = 0; b < B; ++b) g += w.D2[(size_t)b * kH + i] * w.H1[(size_t)b * kH + j];
  } else if (p < oW3) {
    const int i = p - oB2;
    for (int b = 0; b < B; ++b) g += w.D2[(size_t)b * kH + i];
  } else if (p < oB3) {
    const int q = (p - oW3) / kH, j = (p - oW3) % kH;
    for (int b = 0; b < B; ++b) g += w.DY[(size_t)b * kOut + q] * w.H2[(size_t)b * kH + j];
  } else {
    const int q = p - oB3;
    for (int b = 0; b < B; ++b) g += w.DY[(size_t)b * kOut + q];
  }
  G[p] = g;
}

// Adam with bias corrections c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void __launch_bounds__(256) k_mlp_adam(float* __restrict__ P, const float* __restrict__ G,
                                                  float* __restrict__ M, float* __restrict__ V, int n, float lr,
                                                  float beta1, float beta2, float eps, float c1, float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = beta1 * M[i] + (1.0f - beta1) * g;
  const float v = beta2 * V[i] + (1.0f - beta2) * g * g;
  M[i] = m;
  V[i] = v;
  P[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

// Features of the probe: f_j = log10(s_j / s_1) / 8 clamped to [-1, 0] for
// the l leading singular values of the probe sketch, -1 beyond l.
__global__ void __launch_bounds__(kIn) k_features(const double* __restrict__ sv, int l, float* __restrict__ feat) {
  const int t = threadIdx.x;
  const double s1 = sv[0];
  float f = -1.0f;
  if (t < l && s1 > 0.0) {
    const double r = sv[t] / s1;
    f = r > 1e-8 ? (float)(log10(r) / 8.0) : -1.0f;
  }
  feat[t] = f;
}

}  // namespace

hipError_t launch_features(const double* sv, int l, float* feat, hipStream_t st) {
  hipLaunchKernelGGL(k_features, dim3(1), dim3(kIn), 0, st, sv, l, feat);
  return hipGetLastError();
}

int mlp_param_count() { return kParams; }
size_t mlp_work_floats(int B) { return (size_t)B * (4 * kH + 2 * kOut + 1); }

hipError_t launch_mlp_forward(const float* P, const float* X, int B, float* Y, float* work, hipStream_t st) {
  Work w(work, B);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, st, P, X, B, w.H1, w.H2, Y ? Y : w.Y);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* P, const float* X, const float* T, int B, float* G, float* loss,
                               float* work, hipStream_t st) {
  Work w(work, B);
  hipLaunchKernelGGL(k_mlp_fwd, dim3(B), dim3(64), 0, st, P, X, B, w.H1, w.H2, w.Y);
  hipLaunchKernelGGL(k_mlp_delta, dim3(B), dim3(64), 0, st, P, T, B, w);
  hipLaunchKernelGGL(k_mlp_grad, dim3((kParams + 1 + 255) / 256), dim3(256), 0, st, X, B, w, G, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* P, const float* G, float* M, float* V, int64_t step, float lr, float beta1,
                           float beta2, float eps, hipStream_t st) {
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)step)));
  hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, P, G, M, V, kParams, lr, beta1,
                     beta2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace sor
