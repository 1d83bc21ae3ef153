// Separability-proposal network (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/qs.h"

struct qs_mlp {
  void* block = nullptr;  // P, M, V, G (parameters, Adam moments, gradient)
  float* P = nullptr;
  float* M = nullptr;
  float* V = nullptr;
  float* G = nullptr;
  hipStream_t stream = nullptr;
  float* hscore = nullptr;  // pinned, mapped: kScoreRows x 32 inputs, then kScoreRows logits
  float* dscore = nullptr;  // its device address
};

namespace qs {
constexpr int kScoreRows = 64;  // rows scored through the pinned staging
int mlp_param_count();
hipError_t launch_mlp_forward(const float* P, const float* X, int rows, float* logit, float* H1,
                              float* H2, hipStream_t s);
// One wavefront per row; X and logit may be mapped host memory.
hipError_t launch_mlp_score(const float* P, const float* X, int rows, float* logit,
                            hipStream_t s);
hipError_t launch_mlp_backward(const float* P, const float* X, const float* y, int rows,
                               const float* z, const float* H1, const float* H2, float* D3,
                               float* D2, float* D1, float* L, float* G, hipStream_t s);
hipError_t launch_mlp_adam(float* P, float* M, float* V, const float* G, float lr, float b1,
                           float b2, float eps, float c1, float c2, hipStream_t s);
// sigmoid scores of host rows (rows x 32) on the network's stream; synchronizes
int mlp_scores(qs_mlp* net, const float* X, uint64_t rows, float* scores);
}  // namespace qs
