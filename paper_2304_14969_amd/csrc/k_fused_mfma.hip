// Dense k-qubit block (k = 4, 5) on the FP32 matrix cores (complex64 states).
//
// For every assignment of the n-k bits outside the block (a "group"), the 2^k
// amplitudes of the group are multiplied by the block's complex matrix U. Over
// a tile of groups this is a complex product Y = U X with X = 2^k rows x
// groups, computed as three real products on v_mfma_f32_16x16x4f32:
//   P1 = Re U X_r,  P2 = Im U X_i,  P3 = (Re U + Im U)(X_r + X_i),
//   Re Y = P1 - P2,  Im Y = P3 - P1 - P2
// (3/4 of the matrix flops of the real embedding [[Re U, -Im U], [Im U,
// Re U]]). One instruction multiplies 16 output rows by 4 input rows for 16
// groups: lane (q, col) = (lane / 16, lane % 16) supplies U[16 rb + col][4 s +
// q] as the A operand and input row 4 s + q of group col as the B operand,
// one 8-byte LDS read per input amplitude feeding all three products, and
// gets output rows 16 rb + 4 q + i (i < 4) of group col back.
//
// Tile: the contiguous low bits [0, C) plus the block's bits at or above C.
// C is chosen so that the tile holds 128 groups; every tile row is 2^C >= 128
// contiguous amplitudes (>= 1 KiB), loaded and stored with 16-byte vectors.
// Each of the 4 wavefronts of a workgroup owns 32 of the 128 groups, in two
// blocks of 16, and writes its results into the LDS entries of its own groups,
// which only it reads. The matrix is staged in LDS of its own (8 KiB at
// k = 5, XOR-swizzled rows), from which each lane picks its operands.
//
// Which LDS banks a wavefront's 64 input reads hit depends on where the
// block's bits fall in the tile (with the block on bits 0-4 all 16 groups of a
// read share one bank pair). For such 5-qubit blocks the SWZ form keeps tile
// index x at LDS entry x ^ ((x >> swz) & 15), a bijection (swz >= 4) that is
// linear over XOR, so a lane's entry is its own part XOR a uniform part; the
// host picks swz (fused_geometry) and keeps the plain layout wherever it
// already spreads the reads (the extra index work costs more than spreading
// the output writes, which nothing waits for, saves).
#include <algorithm>

#include "qs_internal.h"

namespace qs {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

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

template <int K, bool NT, bool SWZ>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_fused_mfma(float* __restrict__ a, FusedGeom g,
                                                         const float* __restrict__ mat) {
  constexpr int D = 1 << K;           // block dimension
  constexpr int RB = D / 16;          // 16-row blocks of the output
  constexpr int S4 = D / 4;           // K-steps of 4 input rows
  constexpr int BKT = RB == 1 ? 2 : 1;  // 16-group blocks in flight per wave
  constexpr int TB = K + kGroupBits;  // tile bits
  // 32 KiB tile + 8 KiB matrix for k = 5: four workgroups fill a CU's LDS
  __shared__ __align__(16) float2 sm[1 << TB];
  __shared__ float2 smat[D * D];
  const int C = g.C, h = g.h, swz = g.swz;
  auto lp = [&](int x) { return SWZ ? x ^ ((x >> swz) & 15) : x; };
  // tile offset of block row c (block bit j at tile bit tpos[j]); block rows
  // with disjoint bit sets have OR-able offsets
  auto toff = [&](int c) {
    int t = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) t |= ((c >> j) & 1) << g.tpos[j];
    return t;
  };
  // matrix entry (r, c) lives at r D + (c ^ 4 (r mod D/4)): the 16 rows x 4
  // columns an operand read touches fall in distinct LDS banks
  auto mpos = [](int r, int c) { return r * D + (c ^ (4 * (r & (D / 4 - 1)))); };

  // global index of tile entry t: low C bits in place, tile bit C+i -> qhi[i],
  // the workgroup index fills the remaining bits
  uint64_t ob = uint64_t(blockIdx.x) << C;
  for (int i = 0; i < h; ++i) ob = insert_zero64(ob, g.qhi[i]);
  auto glob = [&](int t) {
    uint64_t x = ob | uint64_t(t & ((1 << C) - 1));
    for (int i = 0; i < h; ++i) x |= uint64_t((t >> (C + i)) & 1) << g.qhi[i];
    return x;
  };

  // the matrix first, then the tile: 2^h rows of 2^C amplitudes, two
  // amplitudes per vector (the matrix loads complete first)
  constexpr int NM = (D * D + kThreads - 1) / kThreads;
  float2 mreg[NM];
#pragma unroll
  for (int v = 0; v < NM; ++v) {
    const int e = threadIdx.x + v * kThreads;
    if (e < D * D) mreg[v] = reinterpret_cast<const float2*>(mat)[e];
  }
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
  for (int v = 0; v < NM; ++v) {
    const int e = threadIdx.x + v * kThreads;
    if (e < D * D) smat[mpos(e / D, e % D)] = mreg[v];
  }
  // entries t and t + 1 (t even) land at lp(t) and lp(t) ^ 1: one 16-byte
  // write, its halves swapped when lp(t) is odd
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int e = threadIdx.x + v * kThreads;
    const int t = lp(((e >> vrow) << C) | ((e & ((1 << vrow) - 1)) << 1));
    const float4 x = buf[v];
    reinterpret_cast<float4*>(sm)[t >> 1] = (t & 1) ? make_float4(x.z, x.w, x.x, x.y) : x;
  }
  __syncthreads();

  // this lane's operands: W_c[16 rb + col][4 s + q] for W_0 = Re U,
  // W_1 = Im U, W_2 = Re U + Im U
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, col = lane & 15;
  float A[3][RB][S4];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int s = 0; s < S4; ++s) {
      const float2 u = smat[mpos(16 * rb + col, 4 * s + q)];
      A[0][rb][s] = u.x;
      A[1][rb][s] = u.y;
      A[2][rb][s] = u.x + u.y;
    }
  const int qin = toff(q), qout = toff(4 * q);

#pragma unroll
  for (int b0 = 0; b0 < 2; b0 += BKT) {
    // LDS entries of this lane's input row q and output row 4 q of its group
    // in each block (the group's tile index has zeros at the block's bits)
    int pin[BKT], pout[BKT];
#pragma unroll
    for (int j = 0; j < BKT; ++j) {
      int tb = wave * 32 + 16 * (b0 + j) + col;
      for (int i = 0; i < g.nlow; ++i) tb = insert_zero32(tb, g.lowblk[i]);
      pin[j] = lp(tb | qin);
      pout[j] = lp(tb | qout);
    }
    f32x4 p1[BKT][RB], p2[BKT][RB], p3[BKT][RB];
#pragma unroll
    for (int j = 0; j < BKT; ++j)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) p1[j][rb] = p2[j][rb] = p3[j][rb] = f32x4{};
#pragma unroll
    for (int s = 0; s < S4; ++s) {
      const int ks = lp(toff(4 * s));
#pragma unroll
      for (int j = 0; j < BKT; ++j) {
        const float2 v = sm[pin[j] ^ ks];
        const float vs = v.x + v.y;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          p1[j][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[0][rb][s], v.x, p1[j][rb], 0, 0, 0);
          p2[j][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[1][rb][s], v.y, p2[j][rb], 0, 0, 0);
          p3[j][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[2][rb][s], vs, p3[j][rb], 0, 0, 0);
        }
      }
    }
    // D layout: register i -> output row 16 rb + 4 q + i of group col
#pragma unroll
    for (int j = 0; j < BKT; ++j)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const f32x4 x1 = p1[j][rb], x2 = p2[j][rb], x3 = p3[j][rb];
          sm[pout[j] ^ lp(toff(16 * rb + i))] =
              make_float2(x1[i] - x2[i], x3[i] - (x1[i] + x2[i]));
        }
  }
  __syncthreads();

  // store the tile
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int e = threadIdx.x + v * kThreads;
    const int t = ((e >> vrow) << C) | ((e & ((1 << vrow) - 1)) << 1);
    const int l = lp(t);
    const float4 x = reinterpret_cast<const float4*>(sm)[l >> 1];
    st16<NT>(reinterpret_cast<float4*>(a + 2 * glob(t)), (l & 1) ? make_float4(x.z, x.w, x.x, x.y) : x);
  }
}

}  // namespace

namespace {
// Cost of one wavefront LDS access of 8-byte entries: 32 banks of 4 bytes,
// so entry x occupies bank pair x mod 16; distinct entries on one pair are
// served one after another (the wavefront takes at least 4 such steps).
int lds_steps(const int* entry) {
  int cnt[16] = {}, seen[64], ns = 0;
  int worst = 0;
  for (int l = 0; l < 64; ++l) {
    bool dup = false;
    for (int i = 0; i < ns && !dup; ++i) dup = seen[i] == entry[l];
    if (dup) continue;
    seen[ns++] = entry[l];
    worst = std::max(worst, ++cnt[entry[l] & 15]);
  }
  return worst;
}

// The swizzle shift for a block's tile (16: none): among none and 4..11, the
// one whose input reads take the fewest bank steps, then whose output writes
// do; none whenever it reads as well as the best. Uniform bits (wavefront,
// group block, K-step, output row) XOR every lane's entry with the same
// value, which permutes the bank pairs, so one read and one write of
// wavefront 0 decide. 4-qubit blocks keep the plain layout: eight of their
// workgroups share a CU and hide the conflicts (swizzling measured slower).
int lds_swizzle(const FusedGeom& g) {
  if (g.k != 5) return 16;
  auto toff = [&](int c) {
    int t = 0;
    for (int j = 0; j < g.k; ++j) t |= ((c >> j) & 1) << g.tpos[j];
    return t;
  };
  int best = 16, best_cost = 1 << 30, plain_reads = 0;
  for (int sw : {16, 4, 5, 6, 7, 8, 9, 10, 11}) {
    int rd[64], wr[64];
    for (int lane = 0; lane < 64; ++lane) {
      const int q = lane >> 4, col = lane & 15;
      int tb = col;
      for (int i = 0; i < g.nlow; ++i) {
        const int lo = tb & ((1 << g.lowblk[i]) - 1);
        tb = lo | ((tb ^ lo) << 1);
      }
      const int xr = tb | toff(q), xw = tb | toff(4 * q);
      rd[lane] = xr ^ ((xr >> sw) & 15);
      wr[lane] = xw ^ ((xw >> sw) & 15);
    }
    const int reads = lds_steps(rd), cost = 64 * reads + lds_steps(wr);
    if (sw == 16) plain_reads = reads;
    if (cost < best_cost) best = sw, best_cost = cost;
  }
  return best_cost / 64 == plain_reads ? 16 : best;
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
  g->swz = lds_swizzle(*g);
  return true;
}

hipError_t launch_fused_mfma(float* a, int n, const int* qubits, int k, const float* mat,
                             hipStream_t s) {
  FusedGeom g{};
  if ((k != 4 && k != 5) || !fused_geometry(n, qubits, k, &g)) return hipErrorNotSupported;
  const uint64_t tiles = uint64_t(1) << (n - g.C - g.h);
  if (tiles > 0x7fffffffu) return hipErrorNotSupported;
  const bool nt = stream_sweep(n, 8, g.C);  // rows of 2^C contiguous amplitudes
  const bool sw = g.swz < 16;
  decltype(&k_fused_mfma<4, true, true>) kern;
  if (k == 4)
    kern = nt ? k_fused_mfma<4, true, false> : k_fused_mfma<4, false, false>;
  else
    kern = nt ? (sw ? k_fused_mfma<5, true, true> : k_fused_mfma<5, true, false>)
              : (sw ? k_fused_mfma<5, false, true> : k_fused_mfma<5, false, false>);
  hipLaunchKernelGGL(kern, dim3(unsigned(tiles)), dim3(kThreads), 0, s, a, g, mat);
  return hipGetLastError();
}

}  // namespace qs
