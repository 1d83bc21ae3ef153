// Tile passes of a planned circuit: one HBM read and write of the ket for all
// the gates of a pass.
//
// A tile is 2^(C+H) amplitudes: the contiguous low bits [0, C) (rows of 2^C
// amplitudes) and H = 7 row bits chosen by the planner (complex64: C = 5 by
// default, 256-byte rows and 32 KiB tiles, 4 or 6 by knob; complex128: C = 4,
// 256-byte rows, 32 KiB). The tile is staged
// in LDS (one complex of padding every 16 entries) and transformed round by
// round, each round acting on 4 tile bits. Complex64 rounds are dense 4-qubit
// blocks on the matrix cores (k_tile_mfma), each complex product as three
// real ones (Re U X_r, Im U X_i and (Re U + Im U)(X_r + X_i), 16 x 16 x 4
// MFMAs: 3/4 of the flops of the 32 x 32 real embedding); complex128 rounds
// (k_tile_pass) gather, per thread, the 16 amplitudes that differ in the round's bits and
// apply the round's one- and two-qubit gates in registers (the gate's bits
// inside the round select a compile-time form).
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kW = 4;
constexpr int kV = 1 << kW;  // amplitudes per thread in a round

template <typename R> struct Cx { R r, i; };
template <typename R> struct Vec16;
template <> struct Vec16<float> { using T = float4; static constexpr int AMPS = 2; };
template <> struct Vec16<double> { using T = double2; static constexpr int AMPS = 1; };

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int pos) {
  const uint64_t lo = x & ((uint64_t(1) << pos) - 1);
  return lo | ((x ^ lo) << 1);
}
__device__ __forceinline__ int lds_pos(int x) { return x + (x >> 4); }

template <typename R>
__device__ __forceinline__ Cx<R> cmac(Cx<R> acc, Cx<R> a, Cx<R> b) {
  return {fmadd(a.r, b.r, fmadd(-a.i, b.i, acc.r)), fmadd(a.r, b.i, fmadd(a.i, b.r, acc.i))};
}

// 2x2 matrix (row-major, interleaved) on round bit J.
template <typename R, int J>
__device__ __forceinline__ void apply1(Cx<R> (&v)[kV], const R* __restrict__ m) {
  const Cx<R> m00{m[0], m[1]}, m01{m[2], m[3]}, m10{m[4], m[5]}, m11{m[6], m[7]};
#pragma unroll
  for (int x = 0; x < kV; ++x) {
    if (x & (1 << J)) continue;
    const Cx<R> a = v[x], b = v[x | (1 << J)];
    v[x] = cmac(cmac(Cx<R>{0, 0}, m00, a), m01, b);
    v[x | (1 << J)] = cmac(cmac(Cx<R>{0, 0}, m10, a), m11, b);
  }
}

// 4x4 matrix: row/column bit 0 on round bit J1, bit 1 on round bit J2.
template <typename R, int J1, int J2>
__device__ __forceinline__ void apply2(Cx<R> (&v)[kV], const R* __restrict__ m) {
  Cx<R> M[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) M[e] = {m[2 * e], m[2 * e + 1]};
#pragma unroll
  for (int x = 0; x < kV; ++x) {
    if (x & ((1 << J1) | (1 << J2))) continue;
    int idx[4];
    Cx<R> in[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      idx[c] = x | ((c & 1) << J1) | ((c >> 1) << J2);
      in[c] = v[idx[c]];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Cx<R> y{0, 0};
#pragma unroll
      for (int c = 0; c < 4; ++c) y = cmac(y, M[4 * r + c], in[c]);
      v[idx[r]] = y;
    }
  }
}

template <typename R>
__device__ __forceinline__ void apply_gate(Cx<R> (&v)[kV], int code, const R* __restrict__ m) {
  const int kind = code & 15, j1 = (code >> 4) & 15, j2 = (code >> 8) & 15;
  if (kind == 1) {
    switch (j1) {
      case 0: apply1<R, 0>(v, m); break;
      case 1: apply1<R, 1>(v, m); break;
      case 2: apply1<R, 2>(v, m); break;
      default: apply1<R, 3>(v, m); break;
    }
    return;
  }
  switch (j1 * 4 + j2) {
    case 1: apply2<R, 0, 1>(v, m); break;
    case 2: apply2<R, 0, 2>(v, m); break;
    case 3: apply2<R, 0, 3>(v, m); break;
    case 4: apply2<R, 1, 0>(v, m); break;
    case 6: apply2<R, 1, 2>(v, m); break;
    case 7: apply2<R, 1, 3>(v, m); break;
    case 8: apply2<R, 2, 0>(v, m); break;
    case 9: apply2<R, 2, 1>(v, m); break;
    case 11: apply2<R, 2, 3>(v, m); break;
    case 12: apply2<R, 3, 0>(v, m); break;
    case 13: apply2<R, 3, 1>(v, m); break;
    default: apply2<R, 3, 2>(v, m); break;
  }
}

template <typename R, int C, int H, bool STREAM>
__global__ void __launch_bounds__(1 << (C + H - kW))
    k_tile_pass(R* __restrict__ a, TileRows rows, const int4* __restrict__ rounds, int nrounds,
                const int2* __restrict__ gates, const R* __restrict__ mats) {
  constexpr int TB = C + H;
  constexpr int NT = 1 << (TB - kW);
  using V = typename Vec16<R>::T;
  constexpr int AP = Vec16<R>::AMPS;
  constexpr int VPR = (1 << C) / AP;       // 16-byte vectors per row
  constexpr int NV = (1 << TB) / AP / NT;  // vectors per thread
  extern __shared__ unsigned char smraw[];
  Cx<R>* sm = reinterpret_cast<Cx<R>*>(smraw);
  // tile base: the workgroup index spread over the bits outside the tile
  uint64_t base = uint64_t(blockIdx.x) << C;
#pragma unroll
  for (int j = 0; j < H; ++j) base = insert_zero(base, rows.b[j]);
  auto glob = [&](int row, int col) {
    uint64_t g = base | uint64_t(col);
#pragma unroll
    for (int j = 0; j < H; ++j) g |= uint64_t((row >> j) & 1) << rows.b[j];
    return g;
  };
  V* p = reinterpret_cast<V*>(a);
  V buf[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int e = threadIdx.x + k * NT;
    buf[k] = ld16<STREAM>(p + glob(e / VPR, (e % VPR) * AP) / AP);
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int e = threadIdx.x + k * NT;
    const int x = ((e / VPR) << C) | (e % VPR) * AP;
    if constexpr (AP == 2) {
      sm[lds_pos(x)] = {buf[k].x, buf[k].y};
      sm[lds_pos(x + 1)] = {buf[k].z, buf[k].w};
    } else {
      sm[lds_pos(x)] = {buf[k].x, buf[k].y};
    }
  }
  __syncthreads();
  for (int r = 0; r < nrounds; ++r) {
    const int4 rd = rounds[r];
    const int b0 = rd.x & 255, b1 = (rd.x >> 8) & 255, b2 = (rd.x >> 16) & 255,
              b3 = (rd.x >> 24) & 255;
    int x0 = threadIdx.x;
    x0 = int(insert_zero(uint64_t(x0), b0));
    x0 = int(insert_zero(uint64_t(x0), b1));
    x0 = int(insert_zero(uint64_t(x0), b2));
    x0 = int(insert_zero(uint64_t(x0), b3));
    int pos[kV];
    Cx<R> v[kV];
#pragma unroll
    for (int m = 0; m < kV; ++m) {
      pos[m] = lds_pos(x0 | ((m & 1) << b0) | (((m >> 1) & 1) << b1) | (((m >> 2) & 1) << b2) |
                       (((m >> 3) & 1) << b3));
      v[m] = sm[pos[m]];
    }
    for (int g = rd.y; g < rd.y + rd.z; ++g) {
      const int2 gg = gates[g];
      apply_gate<R>(v, gg.x, mats + gg.y);
    }
#pragma unroll
    for (int m = 0; m < kV; ++m) sm[pos[m]] = v[m];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int e = threadIdx.x + k * NT;
    const int x = ((e / VPR) << C) | (e % VPR) * AP;
    V o;
    const Cx<R> v0 = sm[lds_pos(x)];
    if constexpr (AP == 2) {
      const Cx<R> v1 = sm[lds_pos(x + 1)];
      o = {v0.r, v0.i, v1.r, v1.i};
    } else {
      o = {v0.r, v0.i};
    }
    st16<STREAM>(p + glob(e / VPR, (e % VPR) * AP) / AP, o);
  }
}

// Complex64 passes whose rounds are dense 4-qubit blocks on the FP32 matrix
// cores. A round multiplies the 16 amplitudes of every group (the other 9
// tile bits) by the round's 16x16 complex matrix U, as a real GEMM on the
// interleaved embedding [[Re U, -Im U], [Im U, Re U]] with
// v_mfma_f32_32x32x2f32: a wavefront takes 32 groups at a time (lane % 32 =
// group, lane / 32 = real or imaginary part), one K-step per input amplitude.
// `amats` holds each round's embedding in lane order: entry ks * 64 + lane =
// Uemb[lane % 32][2 ks + lane / 32].
typedef float f32x4 __attribute__((ext_vector_type(4)));
// matrix-core operands of a round per lane: Re U, Im U, Re U + Im U for 4 K-steps
constexpr int kOps = 12;
static_assert(kOps * 64 == kRoundOperands, "round operand layout");

// One tile of a matrix-core pass: `base` is the global index of tile entry 0
// (zeros at the low bits and the row bits), `rows` the row bits.
template <int C, int H, bool STREAM>
__device__ __forceinline__ void tile_mfma_body(float* __restrict__ a, uint64_t base,
                                               const TileRows& rows,
                                               const int4* __restrict__ rounds, int nrounds,
                                               const float* __restrict__ amats) {
  constexpr int TB = C + H;
  constexpr int NT = 1 << (TB - kW);
  constexpr int VPR = (1 << C) / 2;        // float4 vectors per row
  constexpr int NV = (1 << TB) / 2 / NT;   // vectors per thread
  constexpr int CHUNKS = (1 << (TB - kW)) / 32 / (NT / 64);  // 32-group chunks per wave
  // vector e = tid + k NT lies in tile row tid / VPR + k RT: the low row bits
  // come from the thread, the others from k (uniform across the workgroup)
  constexpr int RT = NT / VPR;
  constexpr int RTB = __builtin_ctz(RT);
  static_assert(RT * VPR == NT && RTB <= H, "tile shape");
  extern __shared__ unsigned char smraw[];
  float2* sm = reinterpret_cast<float2*>(smraw);
  const int r0 = int(threadIdx.x) / VPR;
  uint64_t off_t = base | uint64_t((int(threadIdx.x) % VPR) * 2);
#pragma unroll
  for (int j = 0; j < RTB; ++j) off_t |= uint64_t((r0 >> j) & 1) << rows.b[j];
  auto glob_k = [&](int k) {  // global index of this thread's vector k (k known at compile time)
    uint64_t g = off_t;
#pragma unroll
    for (int j = RTB; j < H; ++j)
      if (((k * RT) >> j) & 1) g |= uint64_t(1) << rows.b[j];
    return g;
  };
  float4* p4 = reinterpret_cast<float4*>(a);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, col = lane & 15;
  // this lane's part of the first round's operands, issued before the tile so
  // that its latency hides behind the tile's (the scheduling barrier keeps
  // the compiler from sinking these loads to their first use)
  float A[kOps];
#pragma unroll
  for (int k = 0; k < kOps; ++k) A[k] = amats[rounds[0].y + k * 64 + lane];
  __builtin_amdgcn_sched_barrier(0);
  {
    float4 buf[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) buf[k] = ld16<STREAM>(p4 + glob_k(k) / 2);
    // an empty use of the matrix after the tile loads are issued: it anchors
    // the matrix loads ahead of them (they complete first, in order)
#pragma unroll
    for (int k = 0; k < kOps; ++k) asm volatile("" ::"v"(A[k]));
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = threadIdx.x + k * NT;
      const int x = ((e / VPR) << C) | (e % VPR) * 2;
      sm[lds_pos(x)] = make_float2(buf[k].x, buf[k].y);
      sm[lds_pos(x + 1)] = make_float2(buf[k].z, buf[k].w);
    }
  }
  __syncthreads();
  for (int r = 0; r < nrounds; ++r) {
    const int4 rd = rounds[r];
    const int b0 = rd.x & 255, b1 = (rd.x >> 8) & 255, b2 = (rd.x >> 16) & 255,
              b3 = (rd.x >> 24) & 255;
    // the next round's operands are loaded while this round computes (kept
    // here by the scheduling barrier; left to itself the compiler sinks the
    // loads to the end of the round and the next round waits for them)
    float An[kOps];
    const int offn = rounds[r + 1 < nrounds ? r + 1 : r].y;
#pragma unroll
    for (int k = 0; k < kOps; ++k) An[k] = amats[offn + k * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
    int dep[kV];  // LDS offset of round-local index m (the round bits and padding)
#pragma unroll
    for (int m = 0; m < kV; ++m)
      dep[m] = lds_pos(((m & 1) << b0) | (((m >> 1) & 1) << b1) | (((m >> 2) & 1) << b2) |
                       (((m >> 3) & 1) << b3));
    // lane (q, col) reads input index 4 s + q and writes output index 4 q + i;
    // lds_pos adds over disjoint bits, so these offsets are dep[4 s] + qin and
    // dep[i] + qout with per-lane qin = dep[q], qout = dep[4 q] (a
    // lane-dependent index into dep[] would compile to select chains)
    const int qin = ((q & 1) ? dep[1] : 0) + ((q & 2) ? dep[2] : 0);
    const int qout = ((q & 1) ? dep[4] : 0) + ((q & 2) ? dep[8] : 0);
#pragma unroll
    for (int ch = 0; ch < CHUNKS; ++ch) {
      int px[2];  // LDS offset of this lane's group in each 16-group block
#pragma unroll
      for (int bk = 0; bk < 2; ++bk) {
        int x0 = (wave * CHUNKS + ch) * 32 + 16 * bk + col;
        x0 = int(insert_zero(uint64_t(x0), b0));
        x0 = int(insert_zero(uint64_t(x0), b1));
        x0 = int(insert_zero(uint64_t(x0), b2));
        x0 = int(insert_zero(uint64_t(x0), b3));
        px[bk] = lds_pos(x0);
      }
      // three real 16 x 16 products per block: Re U X_r, Im U X_i,
      // (Re U + Im U)(X_r + X_i), K = 16 in 4 steps of 4
      f32x4 p1[2] = {f32x4{}, f32x4{}}, p2[2] = {f32x4{}, f32x4{}}, p3[2] = {f32x4{}, f32x4{}};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
        for (int bk = 0; bk < 2; ++bk) {
          const float2 v = sm[px[bk] + dep[4 * s4] + qin];
          p1[bk] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[3 * s4], v.x, p1[bk], 0, 0, 0);
          p2[bk] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[3 * s4 + 1], v.y, p2[bk], 0, 0, 0);
          p3[bk] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[3 * s4 + 2], v.x + v.y, p3[bk], 0, 0,
                                                         0);
        }
      }
      // D layout: register i -> output row 4 q + i of group col;
      // Y = (p1 - p2) + i (p3 - p1 - p2)
#pragma unroll
      for (int bk = 0; bk < 2; ++bk)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          sm[px[bk] + dep[i] + qout] =
              make_float2(p1[bk][i] - p2[bk][i], p3[bk][i] - (p1[bk][i] + p2[bk][i]));
    }
#pragma unroll
    for (int k = 0; k < kOps; ++k) A[k] = An[k];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int e = threadIdx.x + k * NT;
    const int x = ((e / VPR) << C) | (e % VPR) * 2;
    const float2 v0 = sm[lds_pos(x)], v1 = sm[lds_pos(x + 1)];
    st16<STREAM>(p4 + glob_k(k) / 2, make_float4(v0.x, v0.y, v1.x, v1.y));
  }
}

template <int C, int H, bool STREAM>
__global__ void __launch_bounds__(1 << (C + H - kW))
    k_tile_mfma(float* __restrict__ a, TileRows rows, const int4* __restrict__ rounds,
                int nrounds, const float* __restrict__ amats) {
  // tile base: the workgroup index spread over the bits outside the tile
  uint64_t base = uint64_t(blockIdx.x) << C;
#pragma unroll
  for (int j = 0; j < H; ++j) base = insert_zero(base, rows.b[j]);
  tile_mfma_body<C, H, STREAM>(a, base, rows, rounds, nrounds, amats);
}

// Many kets at once: workgroup -> item by binary search over the items'
// first tiles; each item is one pass of one ket of the arena.
template <int C, int H>
__global__ void __launch_bounds__(1 << (C + H - kW))
    k_tile_mfma_batch(float* __restrict__ arena, const TileItem* __restrict__ items, int nitems,
                      const int4* __restrict__ rounds, const float* __restrict__ amats) {
  int lo = 0, hi = nitems - 1;
  const uint64_t b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].first_tile <= b) lo = mid;
    else hi = mid - 1;
  }
  const TileItem& it = items[lo];
  uint64_t base = (b - it.first_tile) << C;
#pragma unroll
  for (int j = 0; j < H; ++j) base = insert_zero(base, it.rows.b[j]);
  tile_mfma_body<C, H, false>(arena + 2 * it.amp_off, base, it.rows, rounds + it.r0, it.nr,
                              amats);
}

}  // namespace

namespace {
template <int C>
hipError_t launch_mfma_c(float* a, int n, const TileRows& rows, const void* rounds, int nrounds,
                         const float* amats, hipStream_t s) {
  constexpr int H = kTileRowBits, TB = C + H;
  if (n < TB || nrounds < 1) return hipErrorInvalidValue;
  for (int j = 0; j < H; ++j)
    if (rows.b[j] < C || rows.b[j] >= n || (j > 0 && rows.b[j] <= rows.b[j - 1]))
      return hipErrorInvalidValue;
  const size_t bytes = size_t((1 << TB) + ((1 << TB) >> 4)) * sizeof(float2);
  const uint64_t tiles = uint64_t(1) << (n - TB);
  auto kern = stream_sweep(n, 8, C) ? k_tile_mfma<C, H, true> : k_tile_mfma<C, H, false>;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  hipLaunchKernelGGL(kern, dim3(unsigned(tiles)), dim3(1 << (TB - kW)), bytes, s, a, rows,
                     static_cast<const int4*>(rounds), nrounds, amats);
  return hipGetLastError();
}
}  // namespace


hipError_t launch_tile_mfma(float* a, int n, int low_bits, const TileRows& rows,
                            const void* rounds, int nrounds, const float* amats, hipStream_t s) {
  switch (low_bits) {
    case 4: return launch_mfma_c<4>(a, n, rows, rounds, nrounds, amats, s);
    case 5: return launch_mfma_c<5>(a, n, rows, rounds, nrounds, amats, s);
    case 6: return launch_mfma_c<6>(a, n, rows, rounds, nrounds, amats, s);
    default: return hipErrorInvalidValue;
  }
}

// complex64 (dtype 1): rows of 2^g_tile_low_c64 amplitudes (4: 128 bytes, 5:
// 256 bytes, 6: 512 bytes); complex128: 16 (256 bytes). Rows of 32 complex64
// amplitudes measured fastest for 10-layer random circuits (a 32 KiB tile
// leaves room for four workgroups per CU, against two 64 KiB ones); for
// complex128, rows of 16 (32 KiB tiles) took 4% less time per circuit than
// rows of 32 (64 KiB), one more pass at 7% less time each.
int g_tile_low_c64 = 5;
int tile_low_bits(int dtype) { return dtype == 1 ? g_tile_low_c64 : 4; }

namespace {
template <typename R, int C>
hipError_t launch_pass_c(R* a, int n, const TileRows& rows, const void* rounds, int nrounds,
                         const void* gates, const R* mats, hipStream_t s) {
  constexpr int H = kTileRowBits;
  constexpr int TB = C + H;
  if (n < TB) return hipErrorInvalidValue;
  for (int j = 0; j < H; ++j)
    if (rows.b[j] < C || rows.b[j] >= n || (j > 0 && rows.b[j] <= rows.b[j - 1]))
      return hipErrorInvalidValue;
  const size_t bytes = size_t((1 << TB) + ((1 << TB) >> 4)) * 2 * sizeof(R);
  auto kern = stream_sweep(n, 2 * sizeof(R), C) ? k_tile_pass<R, C, H, true>
                                                : k_tile_pass<R, C, H, false>;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  const unsigned grid = unsigned(uint64_t(1) << (n - TB));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(1 << (TB - kW)), bytes, s, a, rows,
                     static_cast<const int4*>(rounds), nrounds, static_cast<const int2*>(gates),
                     mats);
  return hipGetLastError();
}
}  // namespace

template <typename R>
hipError_t launch_tile_pass(R* a, int n, int low_bits, const TileRows& rows, const void* rounds,
                            int nrounds, const void* gates, const R* mats, hipStream_t s) {
  if (low_bits == 4) return launch_pass_c<R, 4>(a, n, rows, rounds, nrounds, gates, mats, s);
  if (low_bits == 5) return launch_pass_c<R, 5>(a, n, rows, rounds, nrounds, gates, mats, s);
  if constexpr (sizeof(R) == 4)
    if (low_bits == 6) return launch_pass_c<R, 6>(a, n, rows, rounds, nrounds, gates, mats, s);
  return hipErrorInvalidValue;
}

hipError_t launch_tile_mfma_batch(float* arena, const TileItem* items, int nitems, uint64_t tiles,
                                  const void* rounds, const float* amats, hipStream_t s) {
  constexpr int C = kBatchTileLow, H = kTileRowBits, TB = C + H;
  if (nitems < 1 || tiles < 1 || tiles > 0x7fffffffu) return hipErrorInvalidValue;
  const size_t bytes = size_t((1 << TB) + ((1 << TB) >> 4)) * sizeof(float2);
  auto kern = k_tile_mfma_batch<C, H>;
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                            hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  hipLaunchKernelGGL(kern, dim3(unsigned(tiles)), dim3(1 << (TB - kW)), bytes, s, arena, items,
                     nitems, static_cast<const int4*>(rounds), amats);
  return hipGetLastError();
}

template hipError_t launch_tile_pass<float>(float*, int, int, const TileRows&, const void*, int,
                                            const void*, const float*, hipStream_t);
template hipError_t launch_tile_pass<double>(double*, int, int, const TileRows&, const void*, int,
                                             const void*, const double*, hipStream_t);

}  // namespace qs
