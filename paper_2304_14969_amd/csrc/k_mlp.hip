// Separability-proposal network on the GPU: 32 -> 64 (tanh) -> 64 (tanh) -> 1
// logit; score = sigmoid(logit). Float32 forward, backward and Adam.
//
// Parameter vector (6,337 floats): W1[32][64], b1[64], W2[64][64], b2[64],
// W3[64], b3 -- row-major, x @ W + b.
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kIn = 32, kH = 64;
constexpr int oW1 = 0, oB1 = oW1 + kIn * kH, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kH, kParams = oB3 + 1;
constexpr int kBlock = 256;

// One row per thread; parameters in LDS (every lane reads the same weight).
// Stores h1, h2 (rows x 64) and the logit when the pointers are set.
__global__ void __launch_bounds__(kBlock) k_mlp_forward(const float* __restrict__ P,
                                                        const float* __restrict__ X, int rows,
                                                        float* __restrict__ logit,
                                                        float* __restrict__ H1,
                                                        float* __restrict__ H2) {
  __shared__ float w[kParams];
  for (int i = threadIdx.x; i < kParams; i += kBlock) w[i] = P[i];
  __syncthreads();
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= rows) return;
  float x[kIn], h1[kH];
#pragma unroll
  for (int i = 0; i < kIn; ++i) x[i] = X[size_t(r) * kIn + i];
#pragma unroll 4
  for (int j = 0; j < kH; ++j) {
    float s = w[oB1 + j];
#pragma unroll
    for (int i = 0; i < kIn; ++i) s += x[i] * w[oW1 + i * kH + j];
    h1[j] = tanhf(s);
  }
  float z = w[oB3];
#pragma unroll 4
  for (int j = 0; j < kH; ++j) {
    float s = w[oB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) s += h1[i] * w[oW2 + i * kH + j];
    const float h2 = tanhf(s);
    z += h2 * w[oW3 + j];
    if (H2) H2[size_t(r) * kH + j] = h2;
  }
  if (H1)
    for (int j = 0; j < kH; ++j) H1[size_t(r) * kH + j] = h1[j];
  logit[r] = z;
}

// Scoring of a few rows: one wavefront per row, lane j owns hidden unit j of
// both layers (weight columns read coalesced), the output dot product summed
// across the wavefront in a fixed butterfly order. X and logit may live in
// mapped host memory.
__global__ void __launch_bounds__(kH) k_mlp_score(const float* __restrict__ P,
                                                  const float* __restrict__ X,
                                                  float* __restrict__ logit) {
  __shared__ float x[kIn], h1[kH];
  const int r = blockIdx.x, j = threadIdx.x;
  if (j < kIn) x[j] = X[size_t(r) * kIn + j];
  __syncthreads();
  float s = P[oB1 + j];
#pragma unroll 8
  for (int i = 0; i < kIn; ++i) s += x[i] * P[oW1 + i * kH + j];
  h1[j] = tanhf(s);
  __syncthreads();
  float s2 = P[oB2 + j];
#pragma unroll 8
  for (int i = 0; i < kH; ++i) s2 += h1[i] * P[oW2 + i * kH + j];
  float v = tanhf(s2) * P[oW3 + j];
#pragma unroll
  for (int off = kH / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kH);
  if (j == 0) logit[r] = v + P[oB3];
}

// Per-row backward of the mean binary cross-entropy over `rows` rows:
// dz3 = (sigmoid(z) - y)/rows, dz2 = dz3 W3 * (1 - h2^2), dz1 = (dz2 W2^T) * (1 - h1^2).
__global__ void __launch_bounds__(kBlock) k_mlp_delta(const float* __restrict__ P,
                                                      const float* __restrict__ z,
                                                      const float* __restrict__ y,
                                                      const float* __restrict__ H1,
                                                      const float* __restrict__ H2, int rows,
                                                      float* __restrict__ D3,
                                                      float* __restrict__ D2,
                                                      float* __restrict__ D1,
                                                      float* __restrict__ L) {
  __shared__ float w2[kH * kH];
  __shared__ float w3[kH];
  for (int i = threadIdx.x; i < kH * kH; i += kBlock) w2[i] = P[oW2 + i];
  for (int i = threadIdx.x; i < kH; i += kBlock) w3[i] = P[oW3 + i];
  __syncthreads();
  const int r = blockIdx.x * kBlock + threadIdx.x;
  if (r >= rows) return;
  const float zr = z[r], yr = y[r];
  const float s = 1.0f / (1.0f + expf(-zr));
  const float d3 = (s - yr) / float(rows);
  D3[r] = d3;
  L[r] = fmaxf(zr, 0.0f) - yr * zr + log1pf(expf(-fabsf(zr)));
  float d2[kH];
#pragma unroll
  for (int j = 0; j < kH; ++j) {
    const float h2 = H2[size_t(r) * kH + j];
    d2[j] = d3 * w3[j] * (1.0f - h2 * h2);
    D2[size_t(r) * kH + j] = d2[j];
  }
#pragma unroll 4
  for (int i = 0; i < kH; ++i) {
    float s1 = 0.0f;
#pragma unroll
    for (int j = 0; j < kH; ++j) s1 += d2[j] * w2[i * kH + j];
    const float h1 = H1[size_t(r) * kH + i];
    D1[size_t(r) * kH + i] = s1 * (1.0f - h1 * h1);
  }
}

// One thread per parameter, summing over the rows in order (repeatable).
__global__ void __launch_bounds__(kBlock) k_mlp_wgrad(const float* __restrict__ X,
                                                      const float* __restrict__ H1,
                                                      const float* __restrict__ H2,
                                                      const float* __restrict__ D3,
                                                      const float* __restrict__ D2,
                                                      const float* __restrict__ D1, int rows,
                                                      float* __restrict__ G) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= kParams) return;
  float s = 0.0f;
  if (p < oB1) {
    const int i = (p - oW1) / kH, j = (p - oW1) % kH;
    for (int r = 0; r < rows; ++r) s += X[size_t(r) * kIn + i] * D1[size_t(r) * kH + j];
  } else if (p < oW2) {
    const int j = p - oB1;
    for (int r = 0; r < rows; ++r) s += D1[size_t(r) * kH + j];
  } else if (p < oB2) {
    const int i = (p - oW2) / kH, j = (p - oW2) % kH;
    for (int r = 0; r < rows; ++r) s += H1[size_t(r) * kH + i] * D2[size_t(r) * kH + j];
  } else if (p < oW3) {
    const int j = p - oB2;
    for (int r = 0; r < rows; ++r) s += D2[size_t(r) * kH + j];
  } else if (p < oB3) {
    const int i = p - oW3;
    for (int r = 0; r < rows; ++r) s += H2[size_t(r) * kH + i] * D3[r];
  } else {
    for (int r = 0; r < rows; ++r) s += D3[r];
  }
  G[p] = s;
}

// Adam with bias-corrected moments; c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t).
__global__ void __launch_bounds__(kBlock) k_mlp_adam(float* __restrict__ P, float* __restrict__ M,
                                                     float* __restrict__ V,
                                                     const float* __restrict__ G, float lr,
                                                     float b1, float b2, float eps, float c1,
                                                     float c2) {
  const int p = blockIdx.x * kBlock + threadIdx.x;
  if (p >= kParams) return;
  const float g = G[p];
  const float m = b1 * M[p] + (1.0f - b1) * g;
  const float v = b2 * V[p] + (1.0f - b2) * g * g;
  M[p] = m;
  V[p] = v;
  P[p] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

unsigned blocks(int n) { return unsigned((n + kBlock - 1) / kBlock); }

}  // namespace

int mlp_param_count() { return kParams; }

hipError_t launch_mlp_score(const float* P, const float* X, int rows, float* logit,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_score, dim3(rows), dim3(kH), 0, s, P, X, logit);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* P, const float* X, int rows, float* logit, float* H1,
                              float* H2, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks(rows)), dim3(kBlock), 0, s, P, X, rows, logit, H1, H2);
  return hipGetLastError();
}

hipError_t launch_mlp_backward(const float* P, const float* X, const float* y, int rows,
                               const float* z, const float* H1, const float* H2, float* D3,
                               float* D2, float* D1, float* L, float* G, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_delta, dim3(blocks(rows)), dim3(kBlock), 0, s, P, z, y, H1, H2, rows, D3,
                     D2, D1, L);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(blocks(kParams)), dim3(kBlock), 0, s, X, H1, H2, D3, D2, D1,
                     rows, G);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(float* P, float* M, float* V, const float* G, float lr, float b1,
                           float b2, float eps, float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3(blocks(kParams)), dim3(kBlock), 0, s, P, M, V, G, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

}  // namespace qs
