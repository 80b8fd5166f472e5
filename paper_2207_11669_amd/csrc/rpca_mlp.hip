// The controller's MLP (include/rpca.h, RPCA_MLP_*): inference and one
// gradient-descent step, as hand-written HIP kernels. One 64-lane wave per
// sample: lane j owns hidden unit j of both layers.
#include "../../include/rpca.h"

#include <hip/hip_runtime.h>

namespace {

constexpr int kIn = RPCA_MLP_IN, kH = RPCA_MLP_HIDDEN, kOut = RPCA_MLP_OUT;
static_assert(kH == 64, "one wave per sample, one lane per hidden unit");
static_assert(kOut == 2, "two outputs: the decay and the step multiplier");
// Parameter offsets: W1 (kH x kIn), b1, W2 (kH x kH), b2, W3 (kOut x kH), b3.
constexpr int kW1 = 0, kB1 = kW1 + kH * kIn, kW2 = kB1 + kH, kB2 = kW2 + kH * kH,
              kW3 = kB2 + kH, kB3 = kW3 + kOut * kH, kP = kB3 + kOut;
// Output k = lo_k + (hi_k - lo_k) sigmoid(z_k): the decay in [GMIN, 1], the
// step multiplier in [WMIN, WMAX].
__device__ __forceinline__ float out_lo(int k) { return k == 0 ? RPCA_MLP_GMIN : RPCA_MLP_WMIN; }
__device__ __forceinline__ float out_span(int k) {
  return k == 0 ? 1.f - RPCA_MLP_GMIN : RPCA_MLP_WMAX - RPCA_MLP_WMIN;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

struct Fwd {
  float h1, h2;              // lane j: hidden units j of both layers
  float sg[kOut], y[kOut];   // sigmoids and outputs (every lane)
};

// Forward pass of sample x for lane j; h1 of all lanes is left in sh1.
__device__ __forceinline__ Fwd forward(const float* __restrict__ P, const float* __restrict__ x,
                                       float* sh1) {
  const int j = threadIdx.x;
  Fwd f;
  float a1 = P[kB1 + j];
#pragma unroll
  for (int i = 0; i < kIn; ++i) a1 = fmaf(P[kW1 + j * kIn + i], x[i], a1);
  f.h1 = tanhf(a1);
  sh1[j] = f.h1;
  __syncthreads();
  float a2 = P[kB2 + j];
#pragma unroll 8
  for (int k = 0; k < kH; ++k) a2 = fmaf(P[kW2 + j * kH + k], sh1[k], a2);
  f.h2 = tanhf(a2);
#pragma unroll
  for (int k = 0; k < kOut; ++k) {
    const float z = wave_sum(P[kW3 + k * kH + j] * f.h2) + P[kB3 + k];
    f.sg[k] = 1.f / (1.f + expf(-z));
    f.y[k] = out_lo(k) + out_span(k) * f.sg[k];
  }
  return f;
}

__global__ __launch_bounds__(64) void k_mlp_forward(const float* __restrict__ P,
                                                    const float* __restrict__ X, int64_t n,
                                                    float* __restrict__ Y) {
  __shared__ float sh1[kH];
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
    const Fwd f = forward(P, X + i * kIn, sh1);
    if (threadIdx.x < kOut) Y[i * kOut + threadIdx.x] = threadIdx.x == 0 ? f.y[0] : f.y[1];
    __syncthreads();  // sh1 is rewritten by the next sample
  }
}

// Per-sample gradient of 1/2 sum_k (y_k - t_k)^2 by back-propagation, into G[i].
__global__ __launch_bounds__(64) void k_mlp_grad(const float* __restrict__ P,
                                                 const float* __restrict__ X,
                                                 const float* __restrict__ T,
                                                 float* __restrict__ G) {
  __shared__ float sh1[kH], sdz2[kH];
  const int64_t i = blockIdx.x;
  const int j = threadIdx.x;
  const float* x = X + i * kIn;
  const Fwd f = forward(P, x, sh1);
  float* g = G + i * (int64_t)kP;
  float back = 0.f;  // d loss / d h2_j
#pragma unroll
  for (int k = 0; k < kOut; ++k) {
    const float dz = (f.y[k] - T[i * kOut + k]) * out_span(k) * f.sg[k] * (1.f - f.sg[k]);
    g[kW3 + k * kH + j] = dz * f.h2;
    if (j == 0) g[kB3 + k] = dz;
    back = fmaf(dz, P[kW3 + k * kH + j], back);
  }
  const float dz2 = back * (1.f - f.h2 * f.h2);
  g[kB2 + j] = dz2;
  for (int k = 0; k < kH; ++k) g[kW2 + j * kH + k] = dz2 * sh1[k];
  sdz2[j] = dz2;
  __syncthreads();
  float dh1 = 0.f;
#pragma unroll 8
  for (int k = 0; k < kH; ++k) dh1 = fmaf(sdz2[k], P[kW2 + k * kH + j], dh1);
  const float dz1 = dh1 * (1.f - f.h1 * f.h1);
  g[kB1 + j] = dz1;
#pragma unroll
  for (int q = 0; q < kIn; ++q) g[kW1 + j * kIn + q] = dz1 * x[q];
}

// params -= lr * mean over samples (summed in index order, FP64).
__global__ __launch_bounds__(256) void k_mlp_sgd(float* __restrict__ P, const float* __restrict__ G,
                                                 int64_t n, float lr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kP) return;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += (double)G[i * kP + p];
  P[p] = (float)((double)P[p] - (double)lr * s / (double)n);
}

}  // namespace

extern "C" {

int64_t rpca_mlp_param_count(void) { return kP; }

rpca_status rpca_mlp_forward(const float* params, const float* x, int64_t n, float* y,
                             void* stream) {
  if (n < 0 || (n > 0 && (!params || !x || !y))) return RPCA_EINVAL;
  if (n == 0) return RPCA_OK;
  const unsigned blocks = (unsigned)(n < 65535 ? n : 65535);
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks), dim3(64), 0, static_cast<hipStream_t>(stream),
                     params, x, n, y);
  return hipGetLastError() == hipSuccess ? RPCA_OK : RPCA_EDEVICE;
}

rpca_status rpca_mlp_train_step(float* params, const float* x, const float* target, int64_t n,
                                float lr, float* grad_ws, void* stream) {
  if (n < 1 || n > 65535 || !params || !x || !target || !grad_ws) return RPCA_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)n), dim3(64), 0, st, params, x, target, grad_ws);
  hipLaunchKernelGGL(k_mlp_sgd, dim3((kP + 255) / 256), dim3(256), 0, st, params, grad_ws, n, lr);
  return hipGetLastError() == hipSuccess ? RPCA_OK : RPCA_EDEVICE;
}

}  // extern "C"
