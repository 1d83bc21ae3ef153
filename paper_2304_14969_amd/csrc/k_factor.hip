// Kernels of the factorized (approximate) mode, Sec. III.
//
//   compose    c[iA + 2^nA iB] = a[iA] b[iB]      (merge of two subsystems)
//   bloch      s = sum conj(a0) a1, z0 = sum |a0|^2, z1 = sum |a1|^2 over the
//              pairs (a0, a1) that differ in bit t, accumulated in float64 in a
//              fixed order (the reduced state of one qubit, Sec. III-A step 1)
//   decompose  b[u] = (conj(phi0) a[i0(u)] + conj(phi1) a[i1(u)]) * scale,
//              i0/i1 = u with a 0/1 inserted at bit t (projection of the qubit
//              on phi and removal of its bit, Sec. III-A steps 2-4)
//   inner      sum conj(a) b in float64 (fidelity of Eq. fid_exact)
//   gather_mul out[j] *= a[local index of x_j] (readout of a product state)
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBlock = 256;
constexpr int kRedBlocks = 1024;
constexpr int kMaxMulti = 5;  // qubits per multi-qubit Bloch sweep

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int pos) {
  const uint64_t lo = x & ((uint64_t(1) << pos) - 1);
  return lo | ((x ^ lo) << 1);
}

template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N], double* sh) {
  // sh holds N * kBlock doubles; fixed tree order
#pragma unroll
  for (int k = 0; k < N; ++k) sh[k * kBlock + threadIdx.x] = v[k];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < N; ++k) sh[k * kBlock + threadIdx.x] += sh[k * kBlock + threadIdx.x + w];
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = sh[k * kBlock];
}

// Amplitude i of a (x) b, a's qubits at the low na bits.
template <typename R>
__device__ __forceinline__ void compose_at(const R* __restrict__ a, int na,
                                           const R* __restrict__ b, uint64_t i, R& re, R& im) {
  const uint64_t ia = i & ((uint64_t(1) << na) - 1), ib = i >> na;
  const R ar = a[2 * ia], ai = a[2 * ia + 1], br = b[2 * ib], bi = b[2 * ib + 1];
  re = ar * br - ai * bi;
  im = ar * bi + ai * br;
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_compose(R* __restrict__ c, const R* __restrict__ a,
                                                    int na, const R* __restrict__ b,
                                                    uint64_t total) {
  for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < total;
       i += uint64_t(gridDim.x) * kBlock)
    compose_at(a, na, b, i, c[2 * i], c[2 * i + 1]);
}

// Output u of the projection of the qubit at bit t on phi (with the kept
// branch's scale).
template <typename R>
__device__ __forceinline__ void decompose_at(R* __restrict__ b, const R* __restrict__ a,
                                             uint64_t u, int t, double p0r, double p0i,
                                             double p1r, double p1i, double scale) {
  const uint64_t i0 = insert_zero(u, t), i1 = i0 | (uint64_t(1) << t);
  const double x0 = a[2 * i0], y0 = a[2 * i0 + 1], x1 = a[2 * i1], y1 = a[2 * i1 + 1];
  // conj(phi0) a0 + conj(phi1) a1
  const double re = p0r * x0 + p0i * y0 + p1r * x1 + p1i * y1;
  const double im = p0r * y0 - p0i * x0 + p1r * y1 - p1i * x1;
  b[2 * u] = static_cast<R>(re * scale);
  b[2 * u + 1] = static_cast<R>(im * scale);
}

// partial[k * kRedBlocks + block], k = 0..3: Re s, Im s, z0, z1
template <typename R>
__global__ void __launch_bounds__(kBlock) k_bloch_partial(const R* __restrict__ a, uint64_t pairs,
                                                          int t, double* __restrict__ partial) {
  __shared__ double sh[4 * kBlock];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  const uint64_t bit = uint64_t(1) << t;
  for (uint64_t u = uint64_t(blockIdx.x) * kBlock + threadIdx.x; u < pairs; u += stride) {
    const uint64_t i0 = insert_zero(u, t), i1 = i0 | bit;
    const double x0 = a[2 * i0], y0 = a[2 * i0 + 1], x1 = a[2 * i1], y1 = a[2 * i1 + 1];
    v[0] += x0 * x1 + y0 * y1;  // Re conj(a0) a1
    v[1] += x0 * y1 - y0 * x1;  // Im conj(a0) a1
    v[2] += x0 * x0 + y0 * y0;
    v[3] += x1 * x1 + y1 * y1;
  }
  block_sum<4>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) partial[k * gridDim.x + blockIdx.x] = v[k];
}

// The whole reduction in one workgroup (small subsystems): the same sums in
// a fixed order, written straight to `out`.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_bloch_small(const R* __restrict__ a, uint64_t pairs,
                                                        int t, double* __restrict__ out) {
  __shared__ double sh[4 * kBlock];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  const uint64_t bit = uint64_t(1) << t;
  for (uint64_t u = threadIdx.x; u < pairs; u += kBlock) {
    const uint64_t i0 = insert_zero(u, t), i1 = i0 | bit;
    const double x0 = a[2 * i0], y0 = a[2 * i0 + 1], x1 = a[2 * i1], y1 = a[2 * i1 + 1];
    v[0] += x0 * x1 + y0 * y1;
    v[1] += x0 * y1 - y0 * x1;
    v[2] += x0 * x0 + y0 * y0;
    v[3] += x1 * x1 + y1 * y1;
  }
  block_sum<4>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) out[k] = v[k];
}

// The Bloch sums of G qubits of one subsystem in one sweep. Each thread
// gathers the 2^G amplitudes that differ only in the target bits (ascending
// in `bits`) and adds, for every target j, the pairs that differ in bit j.
// Output row 4j+k (k = Re s, Im s, z0, z1) of `partial` per workgroup, or of
// `out` directly when the launch has one workgroup.
struct Bits8 {
  int b[8];
};
struct PairPhi {
  double v[8];  // phi_m, m = 0..3, interleaved
};

// Adds, for every thread-owned group g = first, first + stride, ... < groups,
// the 2^G amplitudes that differ only in the target bits (ascending in
// `bits`): for every target j, the pairs that differ in bit j go to row 4j+k
// of v (k = Re s, Im s, z0, z1).
template <typename R, int G>
__device__ __forceinline__ void bloch_accumulate(const R* __restrict__ a, uint64_t groups,
                                                 const Bits8& bits, uint64_t first,
                                                 uint64_t stride, double (&v)[4 * G]) {
  constexpr int D = 1 << G;
  for (uint64_t g = first; g < groups; g += stride) {
    uint64_t base = g;
#pragma unroll
    for (int j = 0; j < G; ++j) base = insert_zero(base, bits.b[j]);
    R x[D], y[D];
#pragma unroll
    for (int m = 0; m < D; ++m) {
      uint64_t o = base;
#pragma unroll
      for (int j = 0; j < G; ++j) o |= uint64_t((m >> j) & 1) << bits.b[j];
      x[m] = a[2 * o];
      y[m] = a[2 * o + 1];
    }
#pragma unroll
    for (int j = 0; j < G; ++j)
#pragma unroll
      for (int m = 0; m < D; ++m) {
        if (m & (1 << j)) continue;
        const int m1 = m | (1 << j);
        const double x0 = x[m], y0 = y[m], x1 = x[m1], y1 = y[m1];
        v[4 * j + 0] += x0 * x1 + y0 * y1;
        v[4 * j + 1] += x0 * y1 - y0 * x1;
        v[4 * j + 2] += x0 * x0 + y0 * y0;
        v[4 * j + 3] += x1 * x1 + y1 * y1;
      }
  }
}

template <typename R, int G>
__global__ void __launch_bounds__(kBlock) k_bloch_multi(const R* __restrict__ a, uint64_t groups,
                                                        Bits8 bits, double* __restrict__ partial,
                                                        double* __restrict__ out) {
  __shared__ double sh[4 * G * kBlock];
  double v[4 * G];
#pragma unroll
  for (int k = 0; k < 4 * G; ++k) v[k] = 0.0;
  bloch_accumulate<R, G>(a, groups, bits, uint64_t(blockIdx.x) * kBlock + threadIdx.x,
                         uint64_t(gridDim.x) * kBlock, v);
  block_sum<4 * G>(v, sh);
  if (threadIdx.x == 0) {
    if (gridDim.x == 1) {
      for (int k = 0; k < 4 * G; ++k) out[k] = v[k];
    } else {
      for (int k = 0; k < 4 * G; ++k) partial[k * gridDim.x + blockIdx.x] = v[k];
    }
  }
}

// One workgroup per item (a subsystem of at most 2^15 amplitudes and its G
// target bits): the sums of a one-workgroup k_bloch_multi (k_bloch_small for
// G = 1, the same order), written to out[item.out + 4j + k].
template <typename R, int G>
__device__ __forceinline__ void bloch_item(const BlochItem<R>& it, double* sh,
                                           double* __restrict__ out) {
  Bits8 bits{};
#pragma unroll
  for (int j = 0; j < G; ++j) bits.b[j] = it.bits[j];
  double v[4 * G];
#pragma unroll
  for (int k = 0; k < 4 * G; ++k) v[k] = 0.0;
  bloch_accumulate<R, G>(it.amps, uint64_t(1) << (it.nq - G), bits, threadIdx.x, kBlock, v);
  block_sum<4 * G>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4 * G; ++k) out[it.out + k] = v[k];
}

template <typename R>
__device__ __forceinline__ void bloch_dispatch(const BlochItem<R>& it, double* sh,
                                               double* __restrict__ out) {
  switch (it.G) {
    case 1: bloch_item<R, 1>(it, sh, out); break;
    case 2: bloch_item<R, 2>(it, sh, out); break;
    case 3: bloch_item<R, 3>(it, sh, out); break;
    case 4: bloch_item<R, 4>(it, sh, out); break;
    default: bloch_item<R, 5>(it, sh, out); break;
  }
}

// Completion signal of a batched launch (sig.counter == nullptr: none): every
// workgroup's thread 0, after writing its sums, makes them visible to the host
// and counts itself on a device counter; the workgroup that brings the count
// to sig.target stores sig.seq into the host-mapped flag (plain vector stores
// and a vector atomic on device memory).
struct DoneSignal {
  unsigned* counter;
  unsigned* flag;
  unsigned target, seq;
};

__device__ __forceinline__ void signal_done(const DoneSignal& sig) {
  if (sig.counter == nullptr || threadIdx.x != 0) return;
  __threadfence_system();
  const unsigned old = atomicAdd(sig.counter, 1u);
  if (old + 1u == sig.target) {
    __threadfence_system();
    *reinterpret_cast<volatile unsigned*>(sig.flag) = sig.seq;
  }
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_bloch_batch(const BlochItem<R>* __restrict__ items,
                                                        double* __restrict__ out, DoneSignal sig) {
  __shared__ double sh[4 * kMaxMulti * kBlock];
  const BlochItem<R> it = items[blockIdx.x];
  bloch_dispatch(it, sh, out);
  signal_done(sig);
}

// The same with the item table in the kernel arguments (no table reads from
// host memory over the bus).
template <typename R>
struct BlochArgs {
  BlochItem<R> it[kBlochArgItems];
};
template <typename R>
__global__ void __launch_bounds__(kBlock) k_bloch_batch_arg(BlochArgs<R> args,
                                                            double* __restrict__ out,
                                                            DoneSignal sig) {
  __shared__ double sh[4 * kMaxMulti * kBlock];
  const BlochItem<R> it = args.it[blockIdx.x];
  bloch_dispatch(it, sh, out);
  signal_done(sig);
}

// One workgroup per item: the item's subsystem (at most 2^12 amplitudes) is
// staged in LDS, its gates are applied there in order, and it is stored back.
template <typename R, typename GateAt>
__device__ __forceinline__ void fact_1q_item(const Fact1qItem<R>& it, GateAt gate_at, R* sh) {
  const uint32_t words = uint32_t(2) << it.nq, pairs = uint32_t(1) << (it.nq - 1);
  for (uint32_t i = threadIdx.x; i < words; i += kBlock) sh[i] = it.amps[i];
  __syncthreads();
  for (int g = it.g0; g < it.g0 + it.ng; ++g) {
    const Fact1qGate<R> gt = gate_at(g);
    const uint32_t bit = uint32_t(1) << gt.t, low = bit - 1;
    for (uint32_t u = threadIdx.x; u < pairs; u += kBlock) {
      const uint32_t i0 = ((u & ~low) << 1) | (u & low), i1 = i0 | bit;
      const R x0 = sh[2 * i0], y0 = sh[2 * i0 + 1];
      const R x1 = sh[2 * i1], y1 = sh[2 * i1 + 1];
      sh[2 * i0] = gt.m[0] * x0 - gt.m[1] * y0 + gt.m[2] * x1 - gt.m[3] * y1;
      sh[2 * i0 + 1] = gt.m[0] * y0 + gt.m[1] * x0 + gt.m[2] * y1 + gt.m[3] * x1;
      sh[2 * i1] = gt.m[4] * x0 - gt.m[5] * y0 + gt.m[6] * x1 - gt.m[7] * y1;
      sh[2 * i1 + 1] = gt.m[4] * y0 + gt.m[5] * x0 + gt.m[6] * y1 + gt.m[7] * x1;
    }
    __syncthreads();  // the next gate reads what this one wrote
  }
  for (uint32_t i = threadIdx.x; i < words; i += kBlock) it.amps[i] = sh[i];
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_fact_1q_batch(const Fact1qItem<R>* __restrict__ items,
                                                          const Fact1qGate<R>* __restrict__ gates) {
  extern __shared__ __align__(16) char fact_lds[];
  const Fact1qItem<R> it = items[blockIdx.x];
  fact_1q_item(it, [gates](int g) { return gates[g]; }, reinterpret_cast<R*>(fact_lds));
}

// The same with both tables in the kernel arguments.
template <typename R>
struct Fact1qArgs {
  Fact1qItem<R> items[kFact1qArgItems];
  Fact1qGate<R> gates[fact1q_arg_gates<R>()];
};
template <typename R>
__global__ void __launch_bounds__(kBlock) k_fact_1q_batch_arg(Fact1qArgs<R> args) {
  extern __shared__ __align__(16) char fact_lds[];
  const Fact1qItem<R> it = args.items[blockIdx.x];
  fact_1q_item(it, [&args](int g) { return args.gates[g]; }, reinterpret_cast<R*>(fact_lds));
}

template <typename R>
__global__ void k_store_single(R* __restrict__ dst, R a0r, R a0i, R a1r, R a1i) {
  if (threadIdx.x == 0) {
    dst[0] = a0r;
    dst[1] = a0i;
    dst[2] = a1r;
    dst[3] = a1i;
  }
}

template <int N>
__global__ void __launch_bounds__(kBlock) k_sum_rows(const double* __restrict__ partial, int count,
                                                     double* __restrict__ out) {
  __shared__ double sh[N * kBlock];
  double v[N];
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = 0.0;
  for (int i = threadIdx.x; i < count; i += kBlock)
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] += partial[k * count + i];
  block_sum<N>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < N; ++k) out[k] = v[k];
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_decompose(R* __restrict__ b, const R* __restrict__ a,
                                                      uint64_t count, int t, double p0r, double p0i,
                                                      double p1r, double p1i, double scale) {
  for (uint64_t u = uint64_t(blockIdx.x) * kBlock + threadIdx.x; u < count;
       u += uint64_t(gridDim.x) * kBlock)
    decompose_at(b, a, u, t, p0r, p0i, p1r, p1i, scale);
}

// Group g of the merge-and-gate operation: the four amplitudes that differ in
// local bits t0 and t1 of a (x) b (or of a alone when nb = 0), composed as
// k_compose does, times the 4x4 matrix m in the order of the two-qubit
// argument-matrix kernel, written to c.
template <typename R>
__device__ __forceinline__ void merge_gate_group(const R* a, int na, const R* __restrict__ b,
                                                 int nb, R* c, int t0, int t1,
                                                 const R* __restrict__ m, uint64_t g) {
  const int lo = min(t0, t1), hi = max(t0, t1);
  const uint64_t base = insert_zero(insert_zero(g, lo), hi);
  uint64_t off[4];
  R vr[4], vi[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    off[k] = base | (uint64_t(k & 1) << t0) | (uint64_t(k >> 1) << t1);
    if (nb > 0) {
      compose_at(a, na, b, off[k], vr[k], vi[k]);
    } else {
      vr[k] = a[2 * off[k]];
      vi[k] = a[2 * off[k] + 1];
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    R yr = 0, yi = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const R mr = m[2 * (r * 4 + k)], mi = m[2 * (r * 4 + k) + 1];
      yr += mr * vr[k] - mi * vi[k];
      yi += mr * vi[k] + mi * vr[k];
    }
    c[2 * off[r]] = yr;
    c[2 * off[r] + 1] = yi;
  }
}

template <typename R>
struct MatArg4 {
  R v[32];
};

// The 4x4 reduced density matrix of the qubits at bits t1 != t2, unnormalized:
// over the groups g of amplitudes that differ only in those bits (a_m, m =
// bit t1 + 2 bit t2), sums of a_m conj(a_m') in float64. Row k of the output:
// k < 4: rho_kk; then (Re, Im) of rho_01, rho_02, rho_03, rho_12, rho_13,
// rho_23. Per workgroup in `partial` (rows of gridDim.x), or straight to
// `out` when the launch has one workgroup.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_pair_rho(const R* __restrict__ a, uint64_t groups,
                                                     int t1, int t2, double* __restrict__ partial,
                                                     double* __restrict__ out, DoneSignal sig) {
  __shared__ double sh[16 * kBlock];
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = 0.0;
  const int lo = min(t1, t2), hi = max(t1, t2);
  for (uint64_t g = uint64_t(blockIdx.x) * kBlock + threadIdx.x; g < groups;
       g += uint64_t(gridDim.x) * kBlock) {
    const uint64_t base = insert_zero(insert_zero(g, lo), hi);
    double xr[4], xi[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint64_t o = base | (uint64_t(m & 1) << t1) | (uint64_t(m >> 1) << t2);
      xr[m] = a[2 * o];
      xi[m] = a[2 * o + 1];
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) v[m] += xr[m] * xr[m] + xi[m] * xi[m];
    int k = 4;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int mp = m + 1; mp < 4; ++mp) {
        // a_m conj(a_mp)
        v[k++] += xr[m] * xr[mp] + xi[m] * xi[mp];
        v[k++] += xi[m] * xr[mp] - xr[m] * xi[mp];
      }
  }
  block_sum<16>(v, sh);
  if (threadIdx.x == 0) {
    if (gridDim.x == 1) {
      for (int k = 0; k < 16; ++k) out[k] = v[k];
    } else {
      for (int k = 0; k < 16; ++k) partial[k * gridDim.x + blockIdx.x] = v[k];
    }
  }
  if (gridDim.x == 1) signal_done(sig);  // (launches of several workgroups pass no signal)
}

// b[u] = scale * sum_m conj(phi_m) a[u with bits t1, t2 set to m] (m = bit t1
// + 2 bit t2), u over the indices with the two bits removed; and the pair's
// own subsystem `pair` = phi (4 amplitudes, bit 0 = t1's qubit).
template <typename R>
__global__ void __launch_bounds__(kBlock) k_decompose_pair(R* __restrict__ b,
                                                           const R* __restrict__ a,
                                                           uint64_t count, int t1, int t2,
                                                           PairPhi phi, double scale,
                                                           R* __restrict__ pair) {
  const int lo = min(t1, t2), hi = max(t1, t2);
  for (uint64_t u = uint64_t(blockIdx.x) * kBlock + threadIdx.x; u < count;
       u += uint64_t(gridDim.x) * kBlock) {
    const uint64_t base = insert_zero(insert_zero(u, lo), hi);
    double re = 0.0, im = 0.0;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const uint64_t o = base | (uint64_t(m & 1) << t1) | (uint64_t(m >> 1) << t2);
      const double x = a[2 * o], y = a[2 * o + 1];
      const double pr = phi.v[2 * m], pi = phi.v[2 * m + 1];
      re += pr * x + pi * y;  // conj(phi_m) a
      im += pr * y - pi * x;
    }
    b[2 * u] = static_cast<R>(re * scale);
    b[2 * u + 1] = static_cast<R>(im * scale);
  }
  if (blockIdx.x == 0 && threadIdx.x < 8) pair[threadIdx.x] = static_cast<R>(phi.v[threadIdx.x]);
}

// One workgroup per operation (see FactOp). The merge-and-gate form computes
// the composed amplitudes as k_compose does and the 4x4 product as the
// two-qubit argument-matrix kernel does, in the same order.
template <typename R>
__device__ __forceinline__ void fact_op(const FactOp<R>& op) {
  if (op.kind == 1) {
    const uint64_t count = uint64_t(1) << (op.na - 1);
    for (uint64_t u = threadIdx.x; u < count; u += kBlock)
      decompose_at(op.c, op.a, u, op.t0, op.phi[0], op.phi[1], op.phi[2], op.phi[3], op.scale);
    if (threadIdx.x == 0) {
      op.single[0] = static_cast<R>(op.phi[0]);
      op.single[1] = static_cast<R>(op.phi[1]);
      op.single[2] = static_cast<R>(op.phi[2]);
      op.single[3] = static_cast<R>(op.phi[3]);
    }
    return;
  }
  const uint64_t groups = uint64_t(1) << (op.na + op.nb - 2);
  for (uint64_t g = threadIdx.x; g < groups; g += kBlock)
    merge_gate_group(op.a, op.na, op.b, op.nb, op.c, op.t0, op.t1, op.m, g);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_fact_ops(const FactOp<R>* __restrict__ ops) {
  const FactOp<R> op = ops[blockIdx.x];  // the table may be in host memory: read it once
  fact_op(op);
}

// The same with the operations in the kernel arguments.
template <typename R>
struct OpsArgs {
  FactOp<R> op[fact_arg_ops<R>()];
};
template <typename R>
__global__ void __launch_bounds__(kBlock) k_fact_ops_arg(OpsArgs<R> args) {
  const FactOp<R> op = args.op[blockIdx.x];
  fact_op(op);
}

// The merge-and-gate operation over a grid (large subsystems).
template <typename R>
__global__ void __launch_bounds__(kBlock) k_merge_gate(const R* a, int na,
                                                       const R* __restrict__ b, int nb, R* c,
                                                       int t0, int t1, MatArg4<R> m) {
  const uint64_t groups = uint64_t(1) << (na + nb - 2);
  for (uint64_t g = uint64_t(blockIdx.x) * kBlock + threadIdx.x; g < groups;
       g += uint64_t(gridDim.x) * kBlock)
    merge_gate_group(a, na, b, nb, c, t0, t1, m.v, g);
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_inner_partial(const R* __restrict__ a,
                                                          const R* __restrict__ b, uint64_t count,
                                                          double* __restrict__ partial) {
  __shared__ double sh[2 * kBlock];
  double v[2] = {0.0, 0.0};
  const uint64_t stride = uint64_t(gridDim.x) * kBlock;
  for (uint64_t i = uint64_t(blockIdx.x) * kBlock + threadIdx.x; i < count; i += stride) {
    const double ar = a[2 * i], ai = a[2 * i + 1], br = b[2 * i], bi = b[2 * i + 1];
    v[0] += ar * br + ai * bi;
    v[1] += ar * bi - ai * br;
  }
  block_sum<2>(v, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 2; ++k) partial[k * gridDim.x + blockIdx.x] = v[k];
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_gather_mul(const R* __restrict__ a,
                                                       const uint64_t* __restrict__ idx, uint64_t m,
                                                       Perm64 bits, double* __restrict__ out) {
  for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < m;
       j += uint64_t(gridDim.x) * kBlock) {
    const uint64_t x = idx[j];
    uint64_t loc = 0;
    for (int t = 0; t < bits.n; ++t) loc |= ((x >> bits.p[t]) & 1) << t;
    const double ar = a[2 * loc], ai = a[2 * loc + 1];
    const double orr = out[2 * j], oi = out[2 * j + 1];
    out[2 * j] = orr * ar - oi * ai;
    out[2 * j + 1] = orr * ai + oi * ar;
  }
}

// grid of an elementwise kernel; the kernels stride, so the grid is capped
unsigned blocks_for(uint64_t n) {
  const uint64_t b = (n + kBlock - 1) / kBlock;
  const uint64_t cap = uint64_t(1) << 20;
  return unsigned(b < cap ? (b > 0 ? b : 1) : cap);
}
unsigned red_blocks(uint64_t n) {
  const uint64_t b = (n + kBlock - 1) / kBlock;
  return unsigned(b < kRedBlocks ? (b > 0 ? b : 1) : kRedBlocks);
}

}  // namespace

int factor_scratch_doubles() { return 4 * kMaxMulti * kRedBlocks + 8; }

template <typename R>
hipError_t launch_compose(R* c, const R* a, int na, const R* b, int nb, hipStream_t s) {
  const uint64_t total = uint64_t(1) << (na + nb);
  hipLaunchKernelGGL(k_compose<R>, dim3(blocks_for(total)), dim3(kBlock), 0, s, c, a, na, b, total);
  return hipGetLastError();
}

// Subsystems of up to 2^14 pairs are reduced by one workgroup in one launch.
constexpr uint64_t kSmallPairs = uint64_t(1) << 14;

template <typename R>
hipError_t launch_bloch(const R* a, int nq, int t, double* scratch, double* out, hipStream_t s) {
  const uint64_t pairs = uint64_t(1) << (nq - 1);
  if (pairs <= kSmallPairs) {
    hipLaunchKernelGGL(k_bloch_small<R>, dim3(1), dim3(kBlock), 0, s, a, pairs, t, out);
    return hipGetLastError();
  }
  const unsigned nb = red_blocks(pairs);
  hipLaunchKernelGGL(k_bloch_partial<R>, dim3(nb), dim3(kBlock), 0, s, a, pairs, t, scratch + 8);
  hipLaunchKernelGGL(k_sum_rows<4>, dim3(1), dim3(kBlock), 0, s, scratch + 8, int(nb), out);
  return hipGetLastError();
}

template <typename R, int G>
hipError_t launch_multi_g(const R* a, int nq, const int* bits, double* scratch, double* out,
                          hipStream_t s) {
  Bits8 b{};
  for (int j = 0; j < G; ++j) b.b[j] = bits[j];
  const uint64_t groups = uint64_t(1) << (nq - G);
  // one workgroup for small subsystems (same bound in amplitudes as the
  // one-qubit path), else the partial sums of up to kRedBlocks workgroups
  if ((groups << G) <= 2 * kSmallPairs) {
    hipLaunchKernelGGL((k_bloch_multi<R, G>), dim3(1), dim3(kBlock), 0, s, a, groups, b, nullptr,
                       out);
    return hipGetLastError();
  }
  const unsigned nb = red_blocks(groups);
  hipLaunchKernelGGL((k_bloch_multi<R, G>), dim3(nb), dim3(kBlock), 0, s, a, groups, b,
                     scratch + 8, nullptr);
  hipLaunchKernelGGL(k_sum_rows<4 * G>, dim3(1), dim3(kBlock), 0, s, scratch + 8, int(nb), out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bloch_multi(const R* a, int nq, const int* bits, int G, double* scratch,
                              double* out, hipStream_t s) {
  switch (G) {
    case 2: return launch_multi_g<R, 2>(a, nq, bits, scratch, out, s);
    case 3: return launch_multi_g<R, 3>(a, nq, bits, scratch, out, s);
    case 4: return launch_multi_g<R, 4>(a, nq, bits, scratch, out, s);
    case 5: return launch_multi_g<R, 5>(a, nq, bits, scratch, out, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename R>
hipError_t launch_fact_1q_batch(const Fact1qItem<R>* host_items, const Fact1qItem<R>* items,
                                int nitems, const Fact1qGate<R>* host_gates,
                                const Fact1qGate<R>* gates, int ngates, int max_nq,
                                hipStream_t s) {
  if (nitems < 1) return hipSuccess;
  if (max_nq < 1 || max_nq > kFact1qMaxQubits) return hipErrorInvalidValue;
  const size_t lds = (size_t(2) << max_nq) * sizeof(R);
  if (g_kernarg_tables && nitems <= kFact1qArgItems && ngates <= fact1q_arg_gates<R>()) {
    Fact1qArgs<R> args;
    for (int i = 0; i < nitems; ++i) args.items[i] = host_items[i];
    for (int i = 0; i < ngates; ++i) args.gates[i] = host_gates[i];
    hipLaunchKernelGGL(k_fact_1q_batch_arg<R>, dim3(nitems), dim3(kBlock), lds, s, args);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_fact_1q_batch<R>, dim3(nitems), dim3(kBlock), lds, s, items, gates);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_pair_rho(const R* a, int nq, int t1, int t2, double* scratch, double* out,
                           unsigned* counter, unsigned* flag, unsigned target, unsigned seq,
                           hipStream_t s) {
  if (nq < 2 || t1 == t2 || t1 < 0 || t2 < 0 || t1 >= nq || t2 >= nq) return hipErrorInvalidValue;
  const uint64_t groups = uint64_t(1) << (nq - 2);
  if ((groups << 2) <= 2 * kSmallPairs) {
    hipLaunchKernelGGL(k_pair_rho<R>, dim3(1), dim3(kBlock), 0, s, a, groups, t1, t2, nullptr,
                       out, DoneSignal{counter, flag, target, seq});
    return hipGetLastError();
  }
  if (counter) return hipErrorInvalidValue;  // no signal from a multi-workgroup reduction
  const unsigned nb = red_blocks(groups);
  hipLaunchKernelGGL(k_pair_rho<R>, dim3(nb), dim3(kBlock), 0, s, a, groups, t1, t2, scratch + 8,
                     nullptr, DoneSignal{nullptr, nullptr, 0, 0});
  hipLaunchKernelGGL(k_sum_rows<16>, dim3(1), dim3(kBlock), 0, s, scratch + 8, int(nb), out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_decompose_pair(R* b, const R* a, int nq, int t1, int t2, const double phi[8],
                                 double scale, R* pair, hipStream_t s) {
  if (nq < 3 || t1 == t2 || t1 < 0 || t2 < 0 || t1 >= nq || t2 >= nq) return hipErrorInvalidValue;
  PairPhi ph;
  for (int i = 0; i < 8; ++i) ph.v[i] = phi[i];
  const uint64_t count = uint64_t(1) << (nq - 2);
  hipLaunchKernelGGL(k_decompose_pair<R>, dim3(blocks_for(count)), dim3(kBlock), 0, s, b, a,
                     count, t1, t2, ph, scale, pair);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_merge_gate(R* c, const R* a, int na, const R* b, int nb, int t0, int t1,
                             const double m[32], hipStream_t s) {
  if (na < 1 || nb < 0 || na + nb < 2 || t0 == t1 || t0 < 0 || t1 < 0 || t0 >= na + nb ||
      t1 >= na + nb)
    return hipErrorInvalidValue;
  MatArg4<R> mat;
  for (int i = 0; i < 32; ++i) mat.v[i] = static_cast<R>(m[i]);
  const uint64_t groups = uint64_t(1) << (na + nb - 2);
  hipLaunchKernelGGL(k_merge_gate<R>, dim3(blocks_for(groups)), dim3(kBlock), 0, s, a, na, b, nb,
                     c, t0, t1, mat);
  return hipGetLastError();
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_ops_bloch(const BlochItem<R>* __restrict__ items,
                                                      const FactOp<R>* __restrict__ ops,
                                                      double* __restrict__ out, DoneSignal sig) {
  __shared__ double sh[4 * kMaxMulti * kBlock];
  const BlochItem<R> it = items[blockIdx.x];
  if (it.op >= 0) {
    const FactOp<R> op = ops[it.op];
    fact_op(op);
    __syncthreads();  // the sweep reads what the operation wrote
  }
  bloch_dispatch(it, sh, out);
  signal_done(sig);
}

template <typename R>
struct OpsBlochArgs {
  BlochItem<R> it[kFusedItems];
  FactOp<R> op[fused_arg_ops<R>()];
};
template <typename R>
__global__ void __launch_bounds__(kBlock) k_ops_bloch_arg(OpsBlochArgs<R> args,
                                                          double* __restrict__ out,
                                                          DoneSignal sig) {
  __shared__ double sh[4 * kMaxMulti * kBlock];
  const BlochItem<R> it = args.it[blockIdx.x];
  if (it.op >= 0) {
    const FactOp<R> op = args.op[it.op];
    fact_op(op);
    __syncthreads();  // the sweep reads what the operation wrote
  }
  bloch_dispatch(it, sh, out);
  signal_done(sig);
}

template <typename R>
hipError_t launch_ops_bloch(const BlochItem<R>* host_items, const BlochItem<R>* items, int nitems,
                            const FactOp<R>* host_ops, const FactOp<R>* ops, int nops,
                            double* out, unsigned* counter, unsigned* flag, unsigned target,
                            unsigned seq, hipStream_t s) {
  if (nitems < 1) return hipSuccess;
  const DoneSignal sig{counter, flag, target, seq};
  if (g_kernarg_tables && nitems <= kFusedItems && nops <= fused_arg_ops<R>()) {
    OpsBlochArgs<R> args;
    for (int i = 0; i < nitems; ++i) args.it[i] = host_items[i];
    for (int i = 0; i < nops; ++i) args.op[i] = host_ops[i];
    hipLaunchKernelGGL(k_ops_bloch_arg<R>, dim3(nitems), dim3(kBlock), 0, s, args, out, sig);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_ops_bloch<R>, dim3(nitems), dim3(kBlock), 0, s, items, ops, out, sig);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fact_ops(const FactOp<R>* host_ops, const FactOp<R>* ops, int nops,
                           hipStream_t s) {
  if (nops < 1) return hipSuccess;
  if (g_kernarg_tables && nops <= fact_arg_ops<R>()) {
    OpsArgs<R> args;
    for (int i = 0; i < nops; ++i) args.op[i] = host_ops[i];
    hipLaunchKernelGGL(k_fact_ops_arg<R>, dim3(nops), dim3(kBlock), 0, s, args);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_fact_ops<R>, dim3(nops), dim3(kBlock), 0, s, ops);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bloch_batch(const BlochItem<R>* host_items, const BlochItem<R>* items,
                              int nitems, double* out, unsigned* counter, unsigned* flag,
                              unsigned target, unsigned seq, hipStream_t s) {
  if (nitems < 1) return hipSuccess;
  const DoneSignal sig{counter, flag, target, seq};
  if (g_kernarg_tables && nitems <= kBlochArgItems) {
    BlochArgs<R> args;
    for (int i = 0; i < nitems; ++i) args.it[i] = host_items[i];
    hipLaunchKernelGGL(k_bloch_batch_arg<R>, dim3(nitems), dim3(kBlock), 0, s, args, out, sig);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_bloch_batch<R>, dim3(nitems), dim3(kBlock), 0, s, items, out, sig);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_store_single(R* dst, const double amp[4], hipStream_t s) {
  hipLaunchKernelGGL(k_store_single<R>, dim3(1), dim3(64), 0, s, dst, R(amp[0]), R(amp[1]),
                     R(amp[2]), R(amp[3]));
  return hipGetLastError();
}

template <typename R>
hipError_t launch_decompose(R* b, const R* a, int nq, int t, const double phi[4], double scale,
                            hipStream_t s) {
  const uint64_t count = uint64_t(1) << (nq - 1);
  hipLaunchKernelGGL(k_decompose<R>, dim3(blocks_for(count)), dim3(kBlock), 0, s, b, a, count, t,
                     phi[0], phi[1], phi[2], phi[3], scale);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_inner(const R* a, const R* b, uint64_t count, double* scratch, hipStream_t s) {
  const unsigned nb = red_blocks(count);
  hipLaunchKernelGGL(k_inner_partial<R>, dim3(nb), dim3(kBlock), 0, s, a, b, count, scratch + 8);
  hipLaunchKernelGGL(k_sum_rows<2>, dim3(1), dim3(kBlock), 0, s, scratch + 8, int(nb), scratch);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_gather_mul(const R* a, const uint64_t* idx, uint64_t m, Perm64 bits, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_gather_mul<R>, dim3(blocks_for(m)), dim3(kBlock), 0, s, a, idx, m, bits, out);
  return hipGetLastError();
}

#define QS_INST(R)                                                                          \
  template hipError_t launch_compose<R>(R*, const R*, int, const R*, int, hipStream_t);     \
  template hipError_t launch_bloch<R>(const R*, int, int, double*, double*, hipStream_t);   \
  template hipError_t launch_store_single<R>(R*, const double*, hipStream_t);               \
  template hipError_t launch_bloch_batch<R>(const BlochItem<R>*, const BlochItem<R>*, int,   \
                                            double*, unsigned*, unsigned*, unsigned,        \
                                            unsigned, hipStream_t);                         \
  template hipError_t launch_fact_ops<R>(const FactOp<R>*, const FactOp<R>*, int, hipStream_t); \
  template hipError_t launch_ops_bloch<R>(const BlochItem<R>*, const BlochItem<R>*, int,     \
                                          const FactOp<R>*, const FactOp<R>*, int, double*,  \
                                          unsigned*, unsigned*, unsigned, unsigned,          \
                                          hipStream_t);                                      \
  template hipError_t launch_pair_rho<R>(const R*, int, int, int, double*, double*,         \
                                         unsigned*, unsigned*, unsigned, unsigned,          \
                                         hipStream_t);                                      \
  template hipError_t launch_decompose_pair<R>(R*, const R*, int, int, int, const double*,  \
                                               double, R*, hipStream_t);                    \
  template hipError_t launch_merge_gate<R>(R*, const R*, int, const R*, int, int, int,      \
                                           const double*, hipStream_t);                     \
  template hipError_t launch_fact_1q_batch<R>(const Fact1qItem<R>*, const Fact1qItem<R>*, int, \
                                              const Fact1qGate<R>*, const Fact1qGate<R>*, int, \
                                              int, hipStream_t);                            \
  template hipError_t launch_bloch_multi<R>(const R*, int, const int*, int, double*, double*, \
                                            hipStream_t);                                   \
  template hipError_t launch_decompose<R>(R*, const R*, int, int, const double*, double,    \
                                          hipStream_t);                                     \
  template hipError_t launch_inner<R>(const R*, const R*, uint64_t, double*, hipStream_t);  \
  template hipError_t launch_gather_mul<R>(const R*, const uint64_t*, uint64_t, Perm64,     \
                                           double*, hipStream_t);
QS_INST(float)
QS_INST(double)
#undef QS_INST

}  // namespace qs
