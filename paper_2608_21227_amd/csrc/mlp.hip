// Learned cost model of the auto-tuner: a 3-layer perceptron (6 -> 64 -> 64 -> 1,
// ReLU, float32) that predicts the log run time of a configuration, with its
// training (gradient of the mean squared error, Adam) as GPU kernels.
//
// Parameters, one float32 vector (svdv.h gives the offsets):
//   W1[6][64], b1[64], W2[64][64], b2[64], w3[64], b3
// Per sample s:  z1 = x W1 + b1,  a1 = relu(z1),  z2 = a1 W2 + b2,  a2 = relu(z2),
//                y = a2 . w3 + b3;   loss = (1/N) sum_s (y_s - t_s)^2.
// Gradients:     gy = 2 (y - t) / N,  g_z2 = gy w3 [z2 > 0],  g_z1 = (W2 g_z2) [z1 > 0],
//                g_W2 = sum_s a1^T g_z2, g_W1 = sum_s x^T g_z1, and so on for the biases.
// Every sum over samples is taken by one thread in sample order (deterministic).
#include "common.hpp"
#include "kernels.hpp"
#include "../../include/svdv.h"

namespace svdv {

constexpr int kIn = SVDV_MLP_IN, kH = SVDV_MLP_HIDDEN;
constexpr int oW1 = 0, oB1 = kIn * kH, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH, oB3 = oW3 + kH;
static_assert(oB3 + 1 == SVDV_MLP_NPARAM, "parameter layout");

// Workspace (floats): A1[n][64], A2[n][64], G1[n][64], G2[n][64], y[n], gy[n].
struct MlpWork {
  float *a1, *a2, *g1, *g2, *y, *gy;
};
__host__ __device__ inline MlpWork mlp_work(float* w, int64_t n) {
  MlpWork m;
  m.a1 = w;
  m.a2 = w + n * kH;
  m.g1 = w + 2 * n * kH;
  m.g2 = w + 3 * n * kH;
  m.y = w + 4 * n * kH;
  m.gy = w + 4 * n * kH + n;
  return m;
}

// Forward, one thread per sample, parameters staged in LDS.  Stores the
// activations when a1/a2 are given (for the backward pass).
__global__ void __launch_bounds__(256) k_mlp_forward(const float* __restrict__ p, const float* __restrict__ X,
                                                     int64_t n, float* __restrict__ y, float* __restrict__ a1o,
                                                     float* __restrict__ a2o) {
  __shared__ float sp[SVDV_MLP_NPARAM];
  for (int i = threadIdx.x; i < SVDV_MLP_NPARAM; i += blockDim.x) sp[i] = p[i];
  __syncthreads();
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  float x[kIn];
#pragma unroll
  for (int f = 0; f < kIn; ++f) x[f] = X[s * kIn + f];
  float a1[kH];
#pragma unroll
  for (int h = 0; h < kH; ++h) {
    float z = sp[oB1 + h];
#pragma unroll
    for (int f = 0; f < kIn; ++f) z += x[f] * sp[oW1 + f * kH + h];
    a1[h] = z > 0.f ? z : 0.f;
  }
  float out = sp[oB3];
  for (int j = 0; j < kH; ++j) {
    float z = sp[oB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) z += a1[i] * sp[oW2 + i * kH + j];
    const float a = z > 0.f ? z : 0.f;
    if (a2o) a2o[s * kH + j] = a;
    out += a * sp[oW3 + j];
  }
  if (a1o)
#pragma unroll
    for (int h = 0; h < kH; ++h) a1o[s * kH + h] = a1[h];
  y[s] = out;
}

// Per-sample backward: gy, g_z2 (G2) and g_z1 (G1).  ReLU masks come from the
// stored activations (a > 0 exactly when z > 0).
__global__ void __launch_bounds__(256) k_mlp_backward(const float* __restrict__ p, const float* __restrict__ t,
                                                      int64_t n, MlpWork w) {
  __shared__ float sp[SVDV_MLP_NPARAM];
  for (int i = threadIdx.x; i < SVDV_MLP_NPARAM; i += blockDim.x) sp[i] = p[i];
  __syncthreads();
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float gy = 2.f * (w.y[s] - t[s]) / (float)n;
  w.gy[s] = gy;
  float g2[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    g2[j] = w.a2[s * kH + j] > 0.f ? gy * sp[oW3 + j] : 0.f;
    w.g2[s * kH + j] = g2[j];
  }
  for (int i = 0; i < kH; ++i) {
    float g = 0.f;
#pragma unroll
    for (int j = 0; j < kH; ++j) g += sp[oW2 + i * kH + j] * g2[j];
    w.g1[s * kH + i] = w.a1[s * kH + i] > 0.f ? g : 0.f;
  }
}

// Parameter gradients: one thread per parameter, summing over the samples in order.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float* __restrict__ X, int64_t n, MlpWork w,
                                                    float* __restrict__ grad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= SVDV_MLP_NPARAM) return;
  float acc = 0.f;
  if (q < oB1) {  // W1[f][h]
    const int f = q / kH, h = q % kH;
    for (int64_t s = 0; s < n; ++s) acc += X[s * kIn + f] * w.g1[s * kH + h];
  } else if (q < oW2) {  // b1[h]
    const int h = q - oB1;
    for (int64_t s = 0; s < n; ++s) acc += w.g1[s * kH + h];
  } else if (q < oB2) {  // W2[i][j]
    const int i = (q - oW2) / kH, j = (q - oW2) % kH;
    for (int64_t s = 0; s < n; ++s) acc += w.a1[s * kH + i] * w.g2[s * kH + j];
  } else if (q < oW3) {  // b2[j]
    const int j = q - oB2;
    for (int64_t s = 0; s < n; ++s) acc += w.g2[s * kH + j];
  } else if (q < oB3) {  // w3[j]
    const int j = q - oW3;
    for (int64_t s = 0; s < n; ++s) acc += w.gy[s] * w.a2[s * kH + j];
  } else {  // b3
    for (int64_t s = 0; s < n; ++s) acc += w.gy[s];
  }
  grad[q] = acc;
}

// loss = (1/N) sum (y - t)^2, one workgroup, fixed order (per-thread strided sums, then a tree).
__global__ void __launch_bounds__(256) k_mlp_loss(const float* __restrict__ y, const float* __restrict__ t, int64_t n,
                                                  float* __restrict__ loss) {
  __shared__ double part[256];
  double acc = 0.0;
  for (int64_t s = threadIdx.x; s < n; s += blockDim.x) {
    const double d = (double)y[s] - (double)t[s];
    acc += d * d;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) part[threadIdx.x] += part[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(part[0] / (double)n);
}

// Adam (Kingma & Ba): m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// p <- p - lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps), k = step >= 1.
__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= SVDV_MLP_NPARAM) return;
  const float gq = g[q];
  const float mq = b1 * m[q] + (1.f - b1) * gq;
  const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
  m[q] = mq;
  v[q] = vq;
  p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

}  // namespace svdv

using namespace svdv;

extern "C" {

int64_t svdv_mlp_work_size(int64_t n) { return n < 0 ? 0 : 4 * n * kH + 2 * n; }

int svdv_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* stream) {
  if (n < 0 || (n > 0 && (!params || !X || !y))) return report_error(SVDV_ERR_INVALID_ARG, "mlp_forward: bad arguments");
  if (n == 0) return SVDV_OK;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, params, X, n, y,
                     (float*)nullptr, (float*)nullptr);
  return hipGetLastError() == hipSuccess ? SVDV_OK : report_error(SVDV_ERR_HIP, "mlp_forward: launch failed");
}

int svdv_mlp_gradient(const float* params, const float* X, const float* t, int64_t n, float* grad, float* loss,
                      float* work, void* stream) {
  if (n <= 0 || !params || !X || !t || !grad || !work)
    return report_error(SVDV_ERR_INVALID_ARG, "mlp_gradient: bad arguments");
  hipStream_t st = (hipStream_t)stream;
  const MlpWork w = mlp_work(work, n);
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)blocks), dim3(256), 0, st, params, X, n, w.y, w.a1, w.a2);
  hipLaunchKernelGGL(k_mlp_backward, dim3((unsigned)blocks), dim3(256), 0, st, params, t, n, w);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((SVDV_MLP_NPARAM + 255) / 256), dim3(256), 0, st, X, n, w, grad);
  if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, st, w.y, t, n, loss);
  return hipGetLastError() == hipSuccess ? SVDV_OK : report_error(SVDV_ERR_HIP, "mlp_gradient: launch failed");
}

int svdv_mlp_adam_step(float* params, const float* grad, float* m, float* v, int64_t step, float lr, float beta1,
                       float beta2, float eps, void* stream) {
  if (!params || !grad || !m || !v || step < 1) return report_error(SVDV_ERR_INVALID_ARG, "mlp_adam_step: bad arguments");
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((SVDV_MLP_NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, params, grad,
                     m, v, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? SVDV_OK : report_error(SVDV_ERR_HIP, "mlp_adam_step: launch failed");
}

}  // extern "C"
