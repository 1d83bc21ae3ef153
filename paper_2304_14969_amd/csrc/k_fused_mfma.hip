// Dense k-qubit block (k = 4, 5) on the FP32 matrix cores (complex64 states).
//
// For every assignment of the n-k bits outside the block (a "group"), the 2^k
// amplitudes of the group are multiplied by the block's complex matrix U. Over
// a tile of groups this is a complex GEMM Y = U V with V = 2^k rows x groups.
// It runs as a real GEMM with the interleaved embedding
//   row 2r+q of the output (q = 0 real, 1 imaginary part of output row r),
//   column 2c+p of the input (p = 0 real, 1 imaginary part of input row c),
//   Uemb[2r][2c] = Re U, Uemb[2r][2c+1] = -Im U,
//   Uemb[2r+1][2c] = Im U, Uemb[2r+1][2c+1] = Re U,
// on v_mfma_f32_32x32x2f32: one K-step of 2 covers (Re, Im) of one input row,
// so a wavefront's B operand is 32 whole amplitudes read from LDS.
//
// Tile: the contiguous low bits [0, C) plus the block's bits at or above C.
// C is chosen so that the tile holds 128 groups; every tile row is 2^C >= 128
// contiguous amplitudes (>= 1 KiB), loaded and stored with 16-byte vectors.
// Each of the 4 wavefronts of a workgroup owns 32 of the 128 groups: it holds
// its rows of Uemb in VGPRs (the A operand, the same for every group), runs
// the 2^k K-steps per 32-row block of the output, and writes the results into
// its own LDS columns, which only it reads.
#include "qs_internal.h"

namespace qs {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kThreads = 256;  // 4 wavefronts
constexpr int kGroupBits = 7;  // 128 groups per tile

__device__ __forceinline__ uint64_t insert_zero64(uint64_t x, int pos) {
  const uint64_t lo = x & ((uint64_t(1) << pos) - 1);
  return lo | ((x ^ lo) << 1);
}
__device__ __forceinline__ int insert_zero32(int x, int pos) {
  const int lo = x & ((1 << pos) - 1);
  return lo | ((x ^ lo) << 1);
}

template <int K, bool NT>
__global__ void __launch_bounds__(kThreads) k_fused_mfma(float* __restrict__ a, FusedGeom g,
                                                         const float* __restrict__ mat) {
  constexpr int D = 1 << K;           // block dimension
  constexpr int MB = 2 * D / 32;      // 32-row blocks of the embedded output
  constexpr int TB = K + kGroupBits;  // tile bits
  __shared__ float2 sm[1 << TB];
  __shared__ int toff[D];             // tile offset of block row c
  const int C = g.C, h = g.h;

  // tile offsets of the block rows
  for (int c = threadIdx.x; c < D; c += kThreads) {
    int t = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) t |= ((c >> j) & 1) << g.tpos[j];
    toff[c] = t;
  }
  // global index of tile entry t: low C bits in place, tile bit C+i -> qhi[i],
  // the workgroup index fills the remaining bits
  uint64_t ob = uint64_t(blockIdx.x) << C;
  for (int i = 0; i < h; ++i) ob = insert_zero64(ob, g.qhi[i]);
  auto glob = [&](int t) {
    uint64_t x = ob | uint64_t(t & ((1 << C) - 1));
    for (int i = 0; i < h; ++i) x |= uint64_t((t >> (C + i)) & 1) << g.qhi[i];
    return x;
  };

  // load the tile: 2^h rows of 2^C amplitudes, two amplitudes per vector
  constexpr int NV = (1 << TB) / 2 / kThreads;
  float4 buf[NV];
  const int vrow = C - 1;  // log2 vectors per row
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int e = threadIdx.x + v * kThreads;
    const int t = ((e >> vrow) << C) | ((e & ((1 << vrow) - 1)) << 1);
    buf[v] = ld16<NT>(reinterpret_cast<const float4*>(a + 2 * glob(t)));
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int e = threadIdx.x + v * kThreads;
    const int t = ((e >> vrow) << C) | ((e & ((1 << vrow) - 1)) << 1);
    sm[t] = make_float2(buf[v].x, buf[v].y);
    sm[t + 1] = make_float2(buf[v].z, buf[v].w);
  }

  // A operand: lane holds Uemb[32 mb + lane%32][2 ks + lane/32]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int p = lane >> 5;
  float A[MB][D];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const int i = 32 * mb + (lane & 31);
    const int r = i >> 1, q = i & 1;
#pragma unroll
    for (int ks = 0; ks < D; ++ks) {
      const float ur = mat[2 * (r * D + ks)], ui = mat[2 * (r * D + ks) + 1];
      A[mb][ks] = q == 0 ? (p == 0 ? ur : -ui) : (p == 0 ? ui : ur);
    }
  }
  __syncthreads();

  // this lane's group: tile index of its base (zeros at the block's low bits)
  int tb = wave * 32 + (lane & 31);
  for (int i = 0; i < g.nlow; ++i) tb = insert_zero32(tb, g.lowblk[i]);

  f32x16 acc[MB];
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) acc[mb] = f32x16{};
#pragma unroll
  for (int ks = 0; ks < D; ++ks) {
    const float2 v = sm[tb | toff[ks]];
    const float b = p ? v.y : v.x;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
      acc[mb] = __builtin_amdgcn_mfma_f32_32x32x2f32(A[mb][ks], b, acc[mb], 0, 0, 0);
  }
  // D layout: lane, register e -> column lane%32, row 8*(e/4) + 4*(lane/32) + e%4;
  // registers e and e+1 (e even) are the real and imaginary part of one output row
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
    for (int e = 0; e < 16; e += 2) {
      const int i = 32 * mb + 8 * (e >> 2) + 4 * p + (e & 3);
      sm[tb | toff[i >> 1]] = make_float2(acc[mb][e], acc[mb][e + 1]);
    }
  }
  __syncthreads();

  // store the tile
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int e = threadIdx.x + v * kThreads;
    const int t = ((e >> vrow) << C) | ((e & ((1 << vrow) - 1)) << 1);
    const float2 x0 = sm[t], x1 = sm[t + 1];
    st16<NT>(reinterpret_cast<float4*>(a + 2 * glob(t)), make_float4(x0.x, x0.y, x1.x, x1.y));
  }
}

}  // namespace

// Tile geometry for a block on `qubits` (k of them) in an n-qubit state, or
// false if the state is too small for a 128-group tile.
bool fused_geometry(int n, const int* qubits, int k, FusedGeom* g) {
  // smallest C such that the block bits below C leave 7 free low bits
  int C = kGroupBits;
  for (;;) {
    int below = 0;
    for (int j = 0; j < k; ++j) below += qubits[j] < C;
    if (C - below >= kGroupBits) break;
    ++C;
  }
  if (C > n) return false;
  int hiq[6], nh = 0, lowq[6], nl = 0;
  for (int j = 0; j < k; ++j) (qubits[j] >= C ? hiq[nh++] : lowq[nl++]) = qubits[j];
  for (int i = 1; i < nh; ++i)
    for (int j = i; j > 0 && hiq[j - 1] > hiq[j]; --j) { const int t = hiq[j]; hiq[j] = hiq[j - 1]; hiq[j - 1] = t; }
  for (int i = 1; i < nl; ++i)
    for (int j = i; j > 0 && lowq[j - 1] > lowq[j]; --j) { const int t = lowq[j]; lowq[j] = lowq[j - 1]; lowq[j - 1] = t; }
  if (C + nh > n || C < 1) return false;
  g->k = k;
  g->C = C;
  g->h = nh;
  g->nlow = nl;
  for (int i = 0; i < nh; ++i) g->qhi[i] = hiq[i];
  for (int i = 0; i < nl; ++i) g->lowblk[i] = lowq[i];
  for (int j = 0; j < k; ++j) {
    if (qubits[j] < C) {
      g->tpos[j] = qubits[j];
    } else {
      int rank = 0;
      for (int i = 0; i < nh; ++i) rank += hiq[i] < qubits[j];
      g->tpos[j] = C + rank;
    }
  }
  return true;
}

hipError_t launch_fused_mfma(float* a, int n, const int* qubits, int k, const float* mat,
                             hipStream_t s) {
  FusedGeom g{};
  if ((k != 4 && k != 5) || !fused_geometry(n, qubits, k, &g)) return hipErrorNotSupported;
  const uint64_t tiles = uint64_t(1) << (n - g.C - g.h);
  if (tiles > 0x7fffffffu) return hipErrorNotSupported;
  const bool nt = stream_sweep(n, 8, g.C);  // rows of 2^C contiguous amplitudes
  auto kern = k == 4 ? (nt ? k_fused_mfma<4, true> : k_fused_mfma<4, false>)
                     : (nt ? k_fused_mfma<5, true> : k_fused_mfma<5, false>);
  hipLaunchKernelGGL(kern, dim3(unsigned(tiles)), dim3(kThreads), 0, s, a, g, mat);
  return hipGetLastError();
}

}  // namespace qs
