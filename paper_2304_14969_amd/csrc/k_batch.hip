// Batched block application: one launch applies one fused block to each of
// many independent kets stored in one arena (the many-small-circuits case).
//
// The work of a launch is a list of items (ket, block). Each item's groups
// (the 2^(n-k) assignments of the bits outside the block) are split into tiles
// of 256, one group per thread; a prefix of tile counts maps a workgroup's tile
// to its item, whose matrix is staged in LDS. Workgroups stride over tiles, so
// one launch covers the whole batch whatever its size.
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBlock = 256;

template <typename R> struct Cx { R r, i; };

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int pos) {
  const uint64_t lo = x & ((uint64_t(1) << pos) - 1);
  return lo | ((x ^ lo) << 1);
}

template <typename R, int K>
__global__ void __launch_bounds__(kBlock) k_batch_fused(R* __restrict__ arena,
                                                        const BatchItem* __restrict__ items,
                                                        int nitems, uint64_t tiles,
                                                        const R* __restrict__ mats) {
  constexpr int D = 1 << K;
  __shared__ Cx<R> M[D * D];
  __shared__ int item_of_tile;
  for (uint64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    if (threadIdx.x == 0) {
      int lo = 0, hi = nitems - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (items[mid].first_tile <= tile) lo = mid; else hi = mid - 1;
      }
      item_of_tile = lo;
    }
    __syncthreads();
    const BatchItem it = items[item_of_tile];
    const R* m = mats + 2 * it.mat_off;
    for (int e = threadIdx.x; e < D * D; e += kBlock) M[e] = {m[2 * e], m[2 * e + 1]};
    __syncthreads();
    const uint64_t g = (tile - it.first_tile) * kBlock + threadIdx.x;
    const uint64_t groups = uint64_t(1) << (it.n - K);
    if (g < groups) {
      uint64_t base = g;
#pragma unroll
      for (int j = 0; j < K; ++j) base = insert_zero(base, it.sorted[j]);
      R* a = arena + 2 * it.amp_off;
      uint64_t off[D];
      Cx<R> v[D];
#pragma unroll
      for (int c = 0; c < D; ++c) {
        uint64_t o = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) o |= uint64_t((c >> j) & 1) << it.q[j];
        off[c] = base | o;
        v[c] = {a[2 * off[c]], a[2 * off[c] + 1]};
      }
#pragma unroll
      for (int r = 0; r < D; ++r) {
        R yr = 0, yi = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const Cx<R> mm = M[r * D + c];
          yr += mm.r * v[c].r - mm.i * v[c].i;
          yi += mm.r * v[c].i + mm.i * v[c].r;
        }
        a[2 * off[r]] = yr;
        a[2 * off[r] + 1] = yi;
      }
    }
    __syncthreads();
  }
}

// zero the arena, then |0...0> in every ket
template <typename R>
__global__ void __launch_bounds__(kBlock) k_batch_zero(R* __restrict__ arena, uint64_t reals) {
  for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < reals;
       i += uint64_t(gridDim.x) * kBlock)
    arena[i] = R(0);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_batch_ones(R* __restrict__ arena,
                                                       const uint64_t* __restrict__ offs,
                                                       int count) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < count) arena[2 * offs[i]] = R(1);
}

unsigned grid_cap(uint64_t want) {
  const uint64_t cap = uint64_t(1) << 16;
  return unsigned(want < cap ? (want > 0 ? want : 1) : cap);
}

}  // namespace

template <typename R>
hipError_t launch_batch_fused(R* arena, const BatchItem* items, int nitems, uint64_t tiles,
                              int k, const R* mats, hipStream_t s) {
  const dim3 grid(grid_cap(tiles)), block(kBlock);
  switch (k) {
    case 1: hipLaunchKernelGGL((k_batch_fused<R, 1>), grid, block, 0, s, arena, items, nitems, tiles, mats); break;
    case 2: hipLaunchKernelGGL((k_batch_fused<R, 2>), grid, block, 0, s, arena, items, nitems, tiles, mats); break;
    case 3: hipLaunchKernelGGL((k_batch_fused<R, 3>), grid, block, 0, s, arena, items, nitems, tiles, mats); break;
    case 4: hipLaunchKernelGGL((k_batch_fused<R, 4>), grid, block, 0, s, arena, items, nitems, tiles, mats); break;
    case 5: hipLaunchKernelGGL((k_batch_fused<R, 5>), grid, block, 0, s, arena, items, nitems, tiles, mats); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_batch_reset(R* arena, uint64_t total_amps, const uint64_t* offs, int count,
                              hipStream_t s) {
  const uint64_t reals = 2 * total_amps;
  hipLaunchKernelGGL(k_batch_zero<R>, dim3(grid_cap((reals + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, arena, reals);
  hipLaunchKernelGGL(k_batch_ones<R>, dim3((count + kBlock - 1) / kBlock), dim3(kBlock), 0, s,
                     arena, offs, count);
  return hipGetLastError();
}

template hipError_t launch_batch_fused<float>(float*, const BatchItem*, int, uint64_t, int,
                                              const float*, hipStream_t);
template hipError_t launch_batch_fused<double>(double*, const BatchItem*, int, uint64_t, int,
                                               const double*, hipStream_t);
template hipError_t launch_batch_reset<float>(float*, uint64_t, const uint64_t*, int, hipStream_t);
template hipError_t launch_batch_reset<double>(double*, uint64_t, const uint64_t*, int,
                                               hipStream_t);

}  // namespace qs
