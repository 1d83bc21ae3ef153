// Float64 reductions and readout kernels.
//
// Sums are accumulated in float64 in a fixed order: a fixed number of blocks,
// each thread striding through the vector, a fixed tree inside the block, then
// one block adding the block partials in index order. The result is bitwise
// repeatable for a given length.
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBlock = 256;
constexpr int kNormBlocks = 2048;

template <typename R> struct Vec16;
template <> struct Vec16<float> { using T = float4; static constexpr int AMPS = 2; };
template <> struct Vec16<double> { using T = double2; static constexpr int AMPS = 1; };

__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_norm_partial(const R* __restrict__ a, uint64_t vecs,
                                                         double* __restrict__ partial) {
  using V = typename Vec16<R>::T;
  __shared__ double sh[kBlock];
  const V* p = reinterpret_cast<const V*>(a);
  double acc = 0.0;
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  for (uint64_t u = uint64_t(blockIdx.x) * kBlock + threadIdx.x; u < vecs; u += stride) {
    const V v = p[u];
    if constexpr (Vec16<R>::AMPS == 2) {
      acc += double(v.x) * v.x + double(v.y) * v.y + double(v.z) * v.z + double(v.w) * v.w;
    } else {
      acc += v.x * v.x + v.y * v.y;
    }
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kBlock) k_sum_partials(const double* __restrict__ partial,
                                                         int count, double* __restrict__ out) {
  __shared__ double sh[kBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += kBlock) acc += partial[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = s;
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_probs(const R* __restrict__ a, uint64_t count,
                                                  double* __restrict__ pr) {
  for (uint64_t u = uint64_t(blockIdx.x) * kBlock + threadIdx.x; u < count;
       u += uint64_t(gridDim.x) * kBlock) {
    const double re = a[2 * u], im = a[2 * u + 1];
    pr[u] = re * re + im * im;
  }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_gather(const R* __restrict__ a,
                                                   const uint64_t* __restrict__ idx, uint64_t m,
                                                   Perm64 perm, double* __restrict__ out) {
  for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < m;
       j += uint64_t(gridDim.x) * kBlock) {
    const uint64_t x = idx[j];
    uint64_t y = 0;
    for (int q = 0; q < perm.n; ++q) y |= ((x >> q) & 1) << perm.p[q];
    out[2 * j] = a[2 * y];
    out[2 * j + 1] = a[2 * y + 1];
  }
}

unsigned capped_grid(uint64_t n) {
  const uint64_t b = (n + kBlock - 1) / kBlock;
  const uint64_t cap = uint64_t(1) << 20;
  return unsigned(b < cap ? (b > 0 ? b : 1) : cap);
}

}  // namespace

int reduce_blocks(uint64_t) { return kNormBlocks; }

template <typename R>
hipError_t launch_norm(const R* a, uint64_t count, double* partial, double* out, hipStream_t s) {
  const uint64_t vecs = count / Vec16<R>::AMPS;
  if (count % Vec16<R>::AMPS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_norm_partial<R>, dim3(kNormBlocks), dim3(kBlock), 0, s, a, vecs, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, partial, kNormBlocks, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_probs(const R* a, uint64_t count, double* pr, hipStream_t s) {
  hipLaunchKernelGGL(k_probs<R>, dim3(capped_grid(count)), dim3(kBlock), 0, s,
                     a, count, pr);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_gather(const R* a, const uint64_t* idx, uint64_t m, Perm64 perm, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_gather<R>, dim3(capped_grid(m)), dim3(kBlock), 0, s,
                     a, idx, m, perm, out);
  return hipGetLastError();
}

template hipError_t launch_norm<float>(const float*, uint64_t, double*, double*, hipStream_t);
template hipError_t launch_norm<double>(const double*, uint64_t, double*, double*, hipStream_t);
template hipError_t launch_probs<float>(const float*, uint64_t, double*, hipStream_t);
template hipError_t launch_probs<double>(const double*, uint64_t, double*, hipStream_t);
template hipError_t launch_gather<float>(const float*, const uint64_t*, uint64_t, Perm64, double*,
                                         hipStream_t);
template hipError_t launch_gather<double>(const double*, const uint64_t*, uint64_t, Perm64,
                                          double*, hipStream_t);

}  // namespace qs
