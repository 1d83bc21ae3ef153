// Dense k-qubit block (k = 4, 5) on the matrix cores: complex64 states on the
// FP32 ones, complex128 states on the FP64 ones.
//
// For every assignment of the n-k bits outside the block (a "group"), the 2^k
// amplitudes of the group are multiplied by the block's complex matrix U. Over
// a tile of groups this is a complex product Y = U X with X = 2^k rows x
// groups, computed as three real products on v_mfma_f32_16x16x4f32 (or
// v_mfma_f64_16x16x4f64):
//   P1 = Re U X_r,  P2 = Im U X_i,  P3 = (Re U + Im U)(X_r + X_i),
//   Re Y = P1 - P2,  Im Y = P3 - P1 - P2
// (3/4 of the matrix flops of the real embedding [[Re U, -Im U], [Im U,
// Re U]]). One instruction multiplies 16 output rows by 4 input rows for 16
// groups: lane (q, col) = (lane / 16, lane % 16) supplies U[16 rb + col][4 s +
// q] as the A operand and input row 4 s + q of group col as the B operand,
// one LDS read per input amplitude feeding all three products, and gets
// four output rows of group col back in its result registers i < 4: rows
// 16 rb + 4 q + i from the FP32 instruction, 16 rb + q + 4 i from the FP64
// one.
//
// Tile: the contiguous low bits [0, C) plus the block's bits at or above C.
// C is chosen so that the tile holds 128 groups (complex64) or 64 groups
// (complex128); every tile row is >= 1 KiB of contiguous amplitudes, loaded
// and stored with 16-byte vectors. Each of the 4 wavefronts of a workgroup
// owns a quarter of the groups, in blocks of 16, and writes its results into
// the LDS entries of its own groups, which only it reads. The matrix is
// staged in LDS of its own (8 KiB at k = 5 in complex64, 16 KiB in
// complex128, XOR-swizzled rows), from which each lane picks its operands.
//
// Which LDS banks a wavefront's 64 input reads hit depends on where the
// block's bits fall in the tile (with the block on bits 0-4 all 16 groups of a
// read share one bank pair). For such complex64 5-qubit blocks the SWZ form
// keeps tile index x at LDS entry x ^ ((x >> swz) & 15), a bijection (swz >=
// 4) that is linear over XOR, so a lane's entry is its own part XOR a
// uniform part; the host picks swz (fused_geometry) and keeps the plain
// layout wherever it already spreads the reads (the extra index work costs
// more than spreading the output writes, which nothing waits for, saves).
#include <algorithm>

#include "qs_internal.h"

namespace qs {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;  // 4 wavefronts

__device__ __forceinline__ uint64_t insert_zero64(uint64_t x, int pos) {
  const uint64_t lo = x & ((uint64_t(1) << pos) - 1);
  return lo | ((x ^ lo) << 1);
}
__device__ __forceinline__ int insert_zero32(int x, int pos) {
  const int lo = x & ((1 << pos) - 1);
  return lo | ((x ^ lo) << 1);
}

// Per precision: complex entry, 16-byte vector (amplitudes per vector AP),
// accumulator, group bits of the tile, waves per SIMD the registers allow,
// and the result layout (register i of lane group q holds output row
// QS q + IS i of the 16-row block).
template <typename R> struct Prec;
template <> struct Prec<float> {
  using Cx = float2;
  using V = float4;
  using Acc = f32x4;
  static constexpr int AP = 2, GB = 7, WPE = 4, QS = 4, IS = 1;
};
template <> struct Prec<double> {
  using Cx = double2;
  using V = double2;
  using Acc = f64x4;
  static constexpr int AP = 1, GB = 6, WPE = 3, QS = 1, IS = 4;
};
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename R, int K, bool NT, bool SWZ>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(Prec<R>::WPE)))
k_fused_mfma(R* __restrict__ a, FusedGeom g, const R* __restrict__ mat) {
  using P = Prec<R>;
  using Cx = typename P::Cx;
  using V = typename P::V;
  using Acc = typename P::Acc;
  constexpr int D = 1 << K;           // block dimension
  constexpr int RB = D / 16;          // 16-row blocks of the output
  constexpr int S4 = D / 4;           // K-steps of 4 input rows
  constexpr int NB = (1 << P::GB) / 64;  // 16-group blocks per wave
  constexpr int BKT = RB == 1 && NB >= 2 ? 2 : 1;  // blocks in flight per wave
  constexpr int TB = K + P::GB;       // tile bits
  constexpr int LAP = P::AP == 2 ? 1 : 0;
  // k = 5: 32 KiB tile + 8 KiB matrix (complex64, four workgroups fill a
  // CU's LDS) or 32 + 16 KiB (complex128, three)
  __shared__ __align__(16) Cx sm[1 << TB];
  __shared__ Cx smat[D * D];
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
  // tile entry of this thread's vector e: 2^h rows of 2^C amplitudes, AP
  // amplitudes per vector
  const int vrow = C - LAP;  // log2 vectors per row
  auto tent = [&](int e) { return ((e >> vrow) << C) | ((e & ((1 << vrow) - 1)) << LAP); };

  // the matrix first, then the tile (the matrix loads complete first)
  constexpr int NM = D * D / kThreads;
  static_assert(NM * kThreads == D * D, "matrix entries per thread");
  Cx mreg[NM];
#pragma unroll
  for (int v = 0; v < NM; ++v) mreg[v] = reinterpret_cast<const Cx*>(mat)[threadIdx.x + v * kThreads];
  constexpr int NV = (1 << TB) / P::AP / kThreads;
  V buf[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    buf[v] = ld16<NT>(reinterpret_cast<const V*>(a + 2 * glob(tent(threadIdx.x + v * kThreads))));
#pragma unroll
  for (int v = 0; v < NM; ++v) {
    const int e = threadIdx.x + v * kThreads;
    smat[mpos(e / D, e % D)] = mreg[v];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int t = lp(tent(threadIdx.x + v * kThreads));
    if constexpr (P::AP == 2) {
      // entries t and t + 1 (t even) land at lp(t) and lp(t) ^ 1: one
      // 16-byte write, its halves swapped when lp(t) is odd
      const V x = buf[v];
      reinterpret_cast<V*>(sm)[t >> 1] = (t & 1) ? V{x.z, x.w, x.x, x.y} : x;
    } else {
      sm[t] = buf[v];
    }
  }
  __syncthreads();

  // this lane's operands: W_c[16 rb + col][4 s + q] for W_0 = Re U,
  // W_1 = Im U, W_2 = Re U + Im U
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = lane >> 4, col = lane & 15;
  R A[3][RB][S4];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int s = 0; s < S4; ++s) {
      const Cx u = smat[mpos(16 * rb + col, 4 * s + q)];
      A[0][rb][s] = u.x;
      A[1][rb][s] = u.y;
      A[2][rb][s] = u.x + u.y;
    }
  const int qin = toff(q), qout = toff(P::QS * q);

#pragma unroll
  for (int b0 = 0; b0 < NB; b0 += BKT) {
    // LDS entries of this lane's input row q and first output row of its
    // group in each block (the group's tile index has zeros at the block's
    // bits)
    int pin[BKT], pout[BKT];
#pragma unroll
    for (int j = 0; j < BKT; ++j) {
      int tb = wave * (16 * NB) + 16 * (b0 + j) + col;
      for (int i = 0; i < g.nlow; ++i) tb = insert_zero32(tb, g.lowblk[i]);
      pin[j] = lp(tb | qin);
      pout[j] = lp(tb | qout);
    }
    Acc p1[BKT][RB], p2[BKT][RB], p3[BKT][RB];
#pragma unroll
    for (int j = 0; j < BKT; ++j)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) p1[j][rb] = p2[j][rb] = p3[j][rb] = Acc{};
#pragma unroll
    for (int s = 0; s < S4; ++s) {
      const int ks = lp(toff(4 * s));
#pragma unroll
      for (int j = 0; j < BKT; ++j) {
        const Cx v = sm[pin[j] ^ ks];
        const R vs = v.x + v.y;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          p1[j][rb] = mfma16(A[0][rb][s], v.x, p1[j][rb]);
          p2[j][rb] = mfma16(A[1][rb][s], v.y, p2[j][rb]);
          p3[j][rb] = mfma16(A[2][rb][s], vs, p3[j][rb]);
        }
      }
    }
    // result register i -> output row 16 rb + QS q + IS i of group col
#pragma unroll
    for (int j = 0; j < BKT; ++j)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const Acc x1 = p1[j][rb], x2 = p2[j][rb], x3 = p3[j][rb];
          sm[pout[j] ^ lp(toff(16 * rb + P::IS * i))] = Cx{x1[i] - x2[i], x3[i] - (x1[i] + x2[i])};
        }
  }
  __syncthreads();

  // store the tile
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int t = tent(threadIdx.x + v * kThreads);
    const int l = lp(t);
    V* dst = reinterpret_cast<V*>(a + 2 * glob(t));
    if constexpr (P::AP == 2) {
      const V x = reinterpret_cast<const V*>(sm)[l >> 1];
      st16<NT>(dst, (l & 1) ? V{x.z, x.w, x.x, x.y} : x);
    } else {
      st16<NT>(dst, sm[l]);
    }
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

// Tile geometry for a block on `qubits` (k of them) in an n-qubit state of
// amp_bytes-byte amplitudes, or false if the state is too small for a tile of
// 128 (complex64) or 64 (complex128) groups.
bool fused_geometry(int n, const int* qubits, int k, FusedGeom* g, int amp_bytes) {
  const int group_bits = amp_bytes == 8 ? Prec<float>::GB : Prec<double>::GB;
  // smallest C such that the block bits below C leave group_bits free low bits
  int C = group_bits;
  for (;;) {
    int below = 0;
    for (int j = 0; j < k; ++j) below += qubits[j] < C;
    if (C - below >= group_bits) break;
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
  g->swz = amp_bytes == 8 ? lds_swizzle(*g) : 16;
  return true;
}

namespace {
template <typename R>
hipError_t launch_mfma_block(R* a, int n, const int* qubits, int k, const R* mat, hipStream_t s) {
  FusedGeom g{};
  if ((k != 4 && k != 5) || !fused_geometry(n, qubits, k, &g, int(2 * sizeof(R))))
    return hipErrorNotSupported;
  const uint64_t tiles = uint64_t(1) << (n - g.C - g.h);
  if (tiles > 0x7fffffffu) return hipErrorNotSupported;
  const bool nt = stream_sweep(n, 2 * sizeof(R), g.C);  // rows of 2^C contiguous amplitudes
  const bool sw = g.swz < 16;
  decltype(&k_fused_mfma<R, 4, true, true>) kern;
  if (k == 4)
    kern = nt ? k_fused_mfma<R, 4, true, false> : k_fused_mfma<R, 4, false, false>;
  else if constexpr (sizeof(R) == 8)
    kern = nt ? k_fused_mfma<R, 5, true, false> : k_fused_mfma<R, 5, false, false>;
  else
    kern = nt ? (sw ? k_fused_mfma<R, 5, true, true> : k_fused_mfma<R, 5, true, false>)
              : (sw ? k_fused_mfma<R, 5, false, true> : k_fused_mfma<R, 5, false, false>);
  hipLaunchKernelGGL(kern, dim3(unsigned(tiles)), dim3(kThreads), 0, s, a, g, mat);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_fused_mfma(float* a, int n, const int* qubits, int k, const float* mat,
                             hipStream_t s) {
  return launch_mfma_block(a, n, qubits, k, mat, s);
}
hipError_t launch_fused_mfma(double* a, int n, const int* qubits, int k, const double* mat,
                             hipStream_t s) {
  return launch_mfma_block(a, n, qubits, k, mat, s);
}

}  // namespace qs
