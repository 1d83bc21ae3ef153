// Dense k-qubit block applied with vector FMA (the path for k <= 3, and the
// reference point for the matrix-core kernel of larger blocks).
//
// For every assignment of the n-k bits outside the block (a "group"), the 2^k
// amplitudes of the group are multiplied by the block matrix. One thread owns
// one group: it gathers the 2^k amplitudes into registers, forms each output
// row against the matrix held in LDS (every lane reads the same entry, a
// broadcast) and scatters the result. Consecutive threads own groups that
// differ in the lowest free bits, so each gather/scatter instruction of a
// wavefront touches consecutive addresses whenever bit 0 is outside the block.
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBlock = 256;

template <typename R> struct Cx { R r, i; };

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int pos) {
  const uint64_t lo = x & ((uint64_t(1) << pos) - 1);
  return lo | ((x ^ lo) << 1);
}

struct Block6 {
  int k;
  int q[6];       // bit of row/column bit j
  int sorted[6];  // the same bits ascending
};

template <typename R, int K, bool NT>
__global__ void __launch_bounds__(kBlock) k_fused_vec(R* __restrict__ a, uint64_t groups, Block6 b,
                                                      const R* __restrict__ mat) {
  constexpr int D = 1 << K;
  __shared__ Cx<R> M[D * D];
  for (int e = threadIdx.x; e < D * D; e += kBlock) M[e] = {mat[2 * e], mat[2 * e + 1]};
  __syncthreads();
  for (uint64_t g = uint64_t(blockIdx.x) * kBlock + threadIdx.x; g < groups;
       g += uint64_t(gridDim.x) * kBlock) {
    uint64_t base = g;
#pragma unroll
    for (int j = 0; j < K; ++j) base = insert_zero(base, b.sorted[j]);
    uint64_t off[D];
    Cx<R> v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      uint64_t o = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) o |= uint64_t((c >> j) & 1) << b.q[j];
      off[c] = base | o;
      ld_amp<NT>(a + 2 * off[c], &v[c].r, &v[c].i);
    }
#pragma unroll
    for (int r = 0; r < D; ++r) {
      // complex128: read the matrix row by row (left to itself the compiler
      // holds all of M in registers, 256 VGPRs at k = 3, one wave per SIMD)
      if constexpr (sizeof(R) == 8) asm volatile("" ::: "memory");
      R yr = 0, yi = 0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const Cx<R> m = M[r * D + c];
        yr = fmadd(m.r, v[c].r, fmadd(-m.i, v[c].i, yr));
        yi = fmadd(m.r, v[c].i, fmadd(m.i, v[c].r, yi));
      }
      st_amp<NT>(a + 2 * off[r], yr, yi);
    }
  }
}

// Blocks of one or two qubits with the matrix passed by value (no upload):
// the same arithmetic as k_fused_vec, the matrix read from kernel arguments.
template <typename R, int K>
struct MatArg {
  R v[2 << (2 * K)];
};

template <typename R, int K, bool NT>
__global__ void __launch_bounds__(kBlock) k_fused_arg(R* __restrict__ a, uint64_t groups, Block6 b,
                                                      MatArg<R, K> mat) {
  constexpr int D = 1 << K;
  for (uint64_t g = uint64_t(blockIdx.x) * kBlock + threadIdx.x; g < groups;
       g += uint64_t(gridDim.x) * kBlock) {
    uint64_t base = g;
#pragma unroll
    for (int j = 0; j < K; ++j) base = insert_zero(base, b.sorted[j]);
    uint64_t off[D];
    Cx<R> v[D];
#pragma unroll
    for (int c = 0; c < D; ++c) {
      uint64_t o = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) o |= uint64_t((c >> j) & 1) << b.q[j];
      off[c] = base | o;
      ld_amp<NT>(a + 2 * off[c], &v[c].r, &v[c].i);
    }
#pragma unroll
    for (int r = 0; r < D; ++r) {
      R yr = 0, yi = 0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const R mr = mat.v[2 * (r * D + c)], mi = mat.v[2 * (r * D + c) + 1];
        yr = fmadd(mr, v[c].r, fmadd(-mi, v[c].i, yr));
        yi = fmadd(mr, v[c].i, fmadd(mi, v[c].r, yi));
      }
      st_amp<NT>(a + 2 * off[r], yr, yi);
    }
  }
}

unsigned fused_grid(uint64_t groups) {
  const uint64_t want = (groups + kBlock - 1) / kBlock, cap = uint64_t(1) << 20;
  return static_cast<unsigned>(want < cap ? (want > 0 ? want : 1) : cap);
}

Block6 make_block(const int* qubits, int k) {
  Block6 b{};
  b.k = k;
  for (int j = 0; j < k; ++j) b.q[j] = b.sorted[j] = qubits[j];
  for (int i = 1; i < k; ++i)
    for (int j = i; j > 0 && b.sorted[j - 1] > b.sorted[j]; --j) {
      const int t = b.sorted[j];
      b.sorted[j] = b.sorted[j - 1];
      b.sorted[j - 1] = t;
    }
  return b;
}

template <typename R, int K>
hipError_t launch_arg(R* a, int n, const Block6& b, const double* m, hipStream_t s) {
  MatArg<R, K> mat;
  for (int i = 0; i < (2 << (2 * K)); ++i) mat.v[i] = static_cast<R>(m[i]);
  const uint64_t groups = uint64_t(1) << (n - K);
  if (stream_sweep(n, 2 * sizeof(R), b.sorted[0]))
    hipLaunchKernelGGL((k_fused_arg<R, K, true>), dim3(fused_grid(groups)), dim3(kBlock), 0, s, a,
                       groups, b, mat);
  else
    hipLaunchKernelGGL((k_fused_arg<R, K, false>), dim3(fused_grid(groups)), dim3(kBlock), 0, s, a,
                       groups, b, mat);
  return hipGetLastError();
}

template <typename R, int K>
hipError_t launch_k(R* a, int n, const Block6& b, const R* mat, hipStream_t s) {
  const uint64_t groups = uint64_t(1) << (n - K);
  const uint64_t want = (groups + kBlock - 1) / kBlock, cap = uint64_t(1) << 20;
  const unsigned grid = static_cast<unsigned>(want < cap ? want : cap);
  if (stream_sweep(n, 2 * sizeof(R), b.sorted[0]))
    hipLaunchKernelGGL((k_fused_vec<R, K, true>), dim3(grid), dim3(kBlock), 0, s, a, groups, b,
                       mat);
  else
    hipLaunchKernelGGL((k_fused_vec<R, K, false>), dim3(grid), dim3(kBlock), 0, s, a, groups, b,
                       mat);
  return hipGetLastError();
}

}  // namespace

template <typename R>
hipError_t launch_apply_small(R* a, int n, const int* qubits, int k, const double* host_mat,
                              hipStream_t s) {
  const Block6 b = make_block(qubits, k);
  switch (k) {
    case 1: return launch_arg<R, 1>(a, n, b, host_mat, s);
    case 2: return launch_arg<R, 2>(a, n, b, host_mat, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename R>
hipError_t launch_apply_fused(R* a, int n, const int* qubits, int k, const R* mat,
                              hipStream_t s) {
  const Block6 b = make_block(qubits, k);
  switch (k) {
    case 1: return launch_k<R, 1>(a, n, b, mat, s);
    case 2: return launch_k<R, 2>(a, n, b, mat, s);
    case 3: return launch_k<R, 3>(a, n, b, mat, s);
    case 4: return launch_k<R, 4>(a, n, b, mat, s);
    case 5: return launch_k<R, 5>(a, n, b, mat, s);
    case 6: return launch_k<R, 6>(a, n, b, mat, s);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_apply_fused<float>(float*, int, const int*, int, const float*,
                                              hipStream_t);
template hipError_t launch_apply_small<float>(float*, int, const int*, int, const double*,
                                              hipStream_t);
template hipError_t launch_apply_small<double>(double*, int, const int*, int, const double*,
                                               hipStream_t);
template hipError_t launch_apply_fused<double>(double*, int, const int*, int, const double*,
                                               hipStream_t);

}  // namespace qs
