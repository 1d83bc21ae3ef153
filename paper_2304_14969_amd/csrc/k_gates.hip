// Per-gate sweeps over the dense ket (gfx950).
//
// Layout: amplitudes interleaved (re, im); qubit q is bit q of the index.
// Every kernel moves 16-byte vectors (one c128 amplitude or two adjacent c64
// amplitudes) so each wavefront touches whole 64-byte segments; the pair
// partner at distance 2^t sits in the same thread, so each byte is read and
// written once per gate. Grids are capped and threads stride through the
// work, so a launch never exceeds the 2^32 threads of one grid dimension.
#include "qs_internal.h"

namespace qs {
namespace {

template <typename R> struct Vec16;
template <> struct Vec16<float> { using T = float4; static constexpr int AMPS = 2; };
template <> struct Vec16<double> { using T = double2; static constexpr int AMPS = 1; };

constexpr int kBlock = 256;
constexpr uint64_t kMaxGrid = uint64_t(1) << 20;

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int pos) {
  const uint64_t lo = x & ((uint64_t(1) << pos) - 1);
  return lo | ((x ^ lo) << 1);
}

__device__ __forceinline__ uint64_t insert_zeros(uint64_t x, const BitSet16& b) {
  for (int k = 0; k < b.n; ++k) x = insert_zero(x, b.pos[k]);
  return x;
}

// y = m x on one amplitude pair, as a fixed chain of fused multiply-adds
template <typename R>
__device__ __forceinline__ void mat2_apply(const Mat2<R>& m, R& x0r, R& x0i, R& x1r, R& x1i) {
  const R y0r = fmadd(m.re[0], x0r, fmadd(-m.im[0], x0i, fmadd(m.re[1], x1r, -m.im[1] * x1i)));
  const R y0i = fmadd(m.re[0], x0i, fmadd(m.im[0], x0r, fmadd(m.re[1], x1i, m.im[1] * x1r)));
  const R y1r = fmadd(m.re[2], x0r, fmadd(-m.im[2], x0i, fmadd(m.re[3], x1r, -m.im[3] * x1i)));
  const R y1i = fmadd(m.re[2], x0i, fmadd(m.im[2], x0r, fmadd(m.re[3], x1i, m.im[3] * x1r)));
  x0r = y0r; x0i = y0i; x1r = y1r; x1i = y1i;
}

inline unsigned grid_for(uint64_t units) {
  const uint64_t b = (units + kBlock - 1) / kBlock;
  return static_cast<unsigned>(b < kMaxGrid ? (b > 0 ? b : 1) : kMaxGrid);
}

#define QS_STRIDE_LOOP(u, units)                                               \
  for (uint64_t u = uint64_t(blockIdx.x) * kBlock + threadIdx.x; u < (units); \
       u += uint64_t(gridDim.x) * kBlock)

// ------------------------------------------------------------------ 1q
// c64, target bit t >= 1: a unit is two adjacent pairs (i, i+1) x (bit t).
// CTRL: a singly controlled gate swept densely (every pair read and written,
// the matrix applied where index & cmask == cval), for controls whose bit
// leaves runs too short for the sparse sweep.
template <bool NT, bool CTRL = false>
__global__ void __launch_bounds__(kBlock) k_1q_f_vec(float* __restrict__ a, uint64_t units,
                                                     int t, Mat2<float> m, uint64_t cmask,
                                                     uint64_t cval) {
  QS_STRIDE_LOOP(u, units) {
    const uint64_t i0 = insert_zero(u << 1, t);
    float4* p0 = reinterpret_cast<float4*>(a + 2 * i0);
    float4* p1 = reinterpret_cast<float4*>(a + 2 * (i0 + (uint64_t(1) << t)));
    float4 x = ld16<NT>(p0), y = ld16<NT>(p1);
    if (!CTRL || (i0 & cmask) == cval) mat2_apply(m, x.x, x.y, y.x, y.y);
    if (!CTRL || ((i0 + 1) & cmask) == cval) mat2_apply(m, x.z, x.w, y.z, y.w);
    st16<NT>(p0, x);
    st16<NT>(p1, y);
  }
}

// c64, target bit 0: both amplitudes of a pair are in one 16-byte vector.
template <bool NT, bool CTRL = false>
__global__ void __launch_bounds__(kBlock) k_1q_f_bit0(float* __restrict__ a, uint64_t units,
                                                      Mat2<float> m, uint64_t cmask,
                                                      uint64_t cval) {
  QS_STRIDE_LOOP(u, units) {
    float4* p = reinterpret_cast<float4*>(a + 4 * u);
    float4 x = ld16<NT>(p);
    if (!CTRL || ((2 * u) & cmask) == cval) mat2_apply(m, x.x, x.y, x.z, x.w);
    st16<NT>(p, x);
  }
}

// c64, target bit 1 <= t <= 6 with wavefront shuffles: a unit is one 16-byte
// vector (amplitudes 2u, 2u + 1), so every wave instruction covers 1 KiB
// contiguously; the amplitudes with bit t flipped sit 2^(t-1) lanes away in
// the same wave and come over with cross-lane shuffles. Each lane computes
// the rows of its own amplitudes (the same fused multiply-adds as
// mat2_apply). Needs units a multiple of 2^t (all partners in the launch).
template <bool NT, bool CTRL = false>
__global__ void __launch_bounds__(kBlock) k_1q_f_shfl(float* __restrict__ a, uint64_t units,
                                                      int t, Mat2<float> m, uint64_t cmask,
                                                      uint64_t cval) {
  const int d = 1 << (t - 1);
  QS_STRIDE_LOOP(u, units) {
    float4* p = reinterpret_cast<float4*>(a) + u;
    const float4 x = ld16<NT>(p);
    float4 y;
    y.x = __shfl_xor(x.x, d);
    y.y = __shfl_xor(x.y, d);
    y.z = __shfl_xor(x.z, d);
    y.w = __shfl_xor(x.w, d);
    float4 o;
    if ((u >> (t - 1)) & 1) {  // bit t set: rows 1, partner holds the bit-0 amplitudes
      float r0 = y.x, i0 = y.y, r1 = x.x, i1 = x.y;
      mat2_apply(m, r0, i0, r1, i1);
      o.x = r1; o.y = i1;
      r0 = y.z; i0 = y.w; r1 = x.z; i1 = x.w;
      mat2_apply(m, r0, i0, r1, i1);
      o.z = r1; o.w = i1;
    } else {
      float r0 = x.x, i0 = x.y, r1 = y.x, i1 = y.y;
      mat2_apply(m, r0, i0, r1, i1);
      o.x = r0; o.y = i0;
      r0 = x.z; i0 = x.w; r1 = y.z; i1 = y.w;
      mat2_apply(m, r0, i0, r1, i1);
      o.z = r0; o.w = i0;
    }
    if (CTRL) {  // amplitudes 2u, 2u + 1 keep their value where the control does not match
      if (((2 * u) & cmask) != cval) { o.x = x.x; o.y = x.y; }
      if (((2 * u + 1) & cmask) != cval) { o.z = x.z; o.w = x.w; }
    }
    st16<NT>(p, o);
  }
}

// c128: a unit is one pair.
template <bool NT>
__global__ void __launch_bounds__(kBlock) k_1q_d(double* __restrict__ a, uint64_t units, int t,
                                                 Mat2<double> m) {
  QS_STRIDE_LOOP(u, units) {
    const uint64_t i0 = insert_zero(u, t);
    double2* p0 = reinterpret_cast<double2*>(a + 2 * i0);
    double2* p1 = reinterpret_cast<double2*>(a + 2 * (i0 + (uint64_t(1) << t)));
    double2 x = ld16<NT>(p0), y = ld16<NT>(p1);
    mat2_apply(m, x.x, x.y, y.x, y.y);
    st16<NT>(p0, x);
    st16<NT>(p1, y);
  }
}

// ------------------------------------------------------------------ controlled
// Vector path (no fixed bit below the vector width): one unit = Vec16 amps.
template <typename R, bool NT>
__global__ void __launch_bounds__(kBlock) k_ctrl_vec(R* __restrict__ a, uint64_t units,
                                                     BitSet16 fixed, uint64_t set_mask, int tbit,
                                                     Mat2<R> m) {
  using V = typename Vec16<R>::T;
  constexpr int AP = Vec16<R>::AMPS;
  QS_STRIDE_LOOP(u, units) {
    const uint64_t i0 = insert_zeros(u * AP, fixed) | set_mask;
    V* p0 = reinterpret_cast<V*>(a + 2 * i0);
    V* p1 = reinterpret_cast<V*>(a + 2 * (i0 | (uint64_t(1) << tbit)));
    V x = ld16<NT>(p0), y = ld16<NT>(p1);
    if constexpr (AP == 2) {
      mat2_apply(m, x.x, x.y, y.x, y.y);
      mat2_apply(m, x.z, x.w, y.z, y.w);
    } else {
      mat2_apply(m, x.x, x.y, y.x, y.y);
    }
    st16<NT>(p0, x);
    st16<NT>(p1, y);
  }
}

// Scalar path (a fixed bit is bit 0): one pair per thread.
template <typename R, bool NT>
__global__ void __launch_bounds__(kBlock) k_ctrl_scalar(R* __restrict__ a, uint64_t units,
                                                        BitSet16 fixed, uint64_t set_mask,
                                                        int tbit, Mat2<R> m) {
  QS_STRIDE_LOOP(u, units) {
    const uint64_t i0 = insert_zeros(u, fixed) | set_mask;
    const uint64_t i1 = i0 | (uint64_t(1) << tbit);
    R x0r, x0i, x1r, x1i;
    ld_amp<NT>(a + 2 * i0, &x0r, &x0i);
    ld_amp<NT>(a + 2 * i1, &x1r, &x1i);
    mat2_apply(m, x0r, x0i, x1r, x1i);
    st_amp<NT>(a + 2 * i0, x0r, x0i);
    st_amp<NT>(a + 2 * i1, x1r, x1i);
  }
}

// ------------------------------------------------------------------ phase
template <typename R, bool NT>
__global__ void __launch_bounds__(kBlock) k_cphase_vec(R* __restrict__ a, uint64_t units,
                                                       BitSet16 fixed, uint64_t set_mask, R cr,
                                                       R ci) {
  using V = typename Vec16<R>::T;
  constexpr int AP = Vec16<R>::AMPS;
  QS_STRIDE_LOOP(u, units) {
    const uint64_t i = insert_zeros(u * AP, fixed) | set_mask;
    V* p = reinterpret_cast<V*>(a + 2 * i);
    V x = ld16<NT>(p);
    R t;
    t = fmadd(x.x, cr, -x.y * ci); x.y = fmadd(x.x, ci, x.y * cr); x.x = t;
    if constexpr (AP == 2) { t = fmadd(x.z, cr, -x.w * ci); x.w = fmadd(x.z, ci, x.w * cr); x.z = t; }
    st16<NT>(p, x);
  }
}

template <typename R, bool NT>
__global__ void __launch_bounds__(kBlock) k_cphase_scalar(R* __restrict__ a, uint64_t units,
                                                          BitSet16 fixed, uint64_t set_mask,
                                                          R cr, R ci) {
  QS_STRIDE_LOOP(u, units) {
    const uint64_t i = insert_zeros(u, fixed) | set_mask;
    R xr, xi;
    ld_amp<NT>(a + 2 * i, &xr, &xi);
    st_amp<NT>(a + 2 * i, fmadd(xr, cr, -xi * ci), fmadd(xr, ci, xi * cr));
  }
}

// ------------------------------------------------------------------ bit swap
// Exchange the amplitudes at base|2^lo and base|2^hi (bits lo < hi).
template <typename R, bool NT>
__global__ void __launch_bounds__(kBlock) k_bitswap_vec(R* __restrict__ a, uint64_t units,
                                                        BitSet16 fixed, int lo, int hi) {
  using V = typename Vec16<R>::T;
  constexpr int AP = Vec16<R>::AMPS;
  QS_STRIDE_LOOP(u, units) {
    const uint64_t b = insert_zeros(u * AP, fixed);
    V* p0 = reinterpret_cast<V*>(a + 2 * (b | (uint64_t(1) << lo)));
    V* p1 = reinterpret_cast<V*>(a + 2 * (b | (uint64_t(1) << hi)));
    const V x = ld16<NT>(p0), y = ld16<NT>(p1);
    st16<NT>(p0, y);
    st16<NT>(p1, x);
  }
}

template <typename R, bool NT>
__global__ void __launch_bounds__(kBlock) k_bitswap_scalar(R* __restrict__ a, uint64_t units,
                                                           BitSet16 fixed, int lo, int hi) {
  QS_STRIDE_LOOP(u, units) {
    const uint64_t b = insert_zeros(u, fixed);
    const uint64_t i0 = b | (uint64_t(1) << lo), i1 = b | (uint64_t(1) << hi);
    R xr, xi, yr, yi;
    ld_amp<NT>(a + 2 * i0, &xr, &xi);
    ld_amp<NT>(a + 2 * i1, &yr, &yi);
    st_amp<NT>(a + 2 * i0, yr, yi);
    st_amp<NT>(a + 2 * i1, xr, xi);
  }
}

// ------------------------------------------------------------------ setup
template <typename R>
__global__ void __launch_bounds__(kBlock) k_set_basis(R* __restrict__ a, uint64_t units,
                                                      uint64_t x) {
  using V = typename Vec16<R>::T;
  constexpr int AP = Vec16<R>::AMPS;
  QS_STRIDE_LOOP(u, units) {
    V v{};
    if (x / AP == u) {
      if constexpr (AP == 2) {
        if (x % 2 == 0) v.x = R(1); else v.z = R(1);
      } else {
        v.x = R(1);
      }
    }
    reinterpret_cast<V*>(a)[u] = v;
  }
}

template <typename Rd, typename Rs>
__global__ void __launch_bounds__(kBlock) k_convert(Rd* __restrict__ d, const Rs* __restrict__ s,
                                                    uint64_t count) {
  QS_STRIDE_LOOP(u, count) {
    d[2 * u] = static_cast<Rd>(s[2 * u]);
    d[2 * u + 1] = static_cast<Rd>(s[2 * u + 1]);
  }
}

BitSet16 sorted_bits(std::initializer_list<int> bits) {
  BitSet16 b{};
  for (int v : bits) b.pos[b.n++] = v;
  for (int i = 1; i < b.n; ++i)
    for (int j = i; j > 0 && b.pos[j - 1] > b.pos[j]; --j) {
      const int t = b.pos[j];
      b.pos[j] = b.pos[j - 1];
      b.pos[j - 1] = t;
    }
  return b;
}

template <typename R>
constexpr int log_amps() { return Vec16<R>::AMPS == 2 ? 1 : 0; }

}  // namespace

// sweep.stream: 0 streaming accesses for states above the last-level cache,
// 1 always, 2 never
int g_sweep_stream = 0;
// gate.shuffle_bits: complex64 one-qubit gates on bits 1 .. this (at most 6)
// exchange partner amplitudes by wavefront shuffles (0: never). At 30 qubits
// they run at the rate of a gate on bit 0 (6.3-6.4 TB/s) where strided pairs
// reach 5.5-5.6 (bits 1-3) and 6.0 TB/s (bits 4-6).
int g_shuffle_bits = 6;
// gate.dense_ctrl: singly controlled complex64 gates with the control below
// bit 3 swept densely (1) or sparsely (0)
int g_dense_ctrl = 1;

// ------------------------------------------------------------------ launchers
namespace {
// Every sweep streams its state when stream_sweep says so (states above the
// last-level cache): kt is the streaming instantiation, kf the plain one.
template <typename KT, typename KF, typename... Args>
void launch_nt(bool nt, KT kt, KF kf, unsigned grid, hipStream_t s, Args... args) {
  if (nt)
    hipLaunchKernelGGL(kt, dim3(grid), dim3(kBlock), 0, s, args...);
  else
    hipLaunchKernelGGL(kf, dim3(grid), dim3(kBlock), 0, s, args...);
}
}  // namespace

template <>
hipError_t launch_apply_1q<float>(float* a, int n, int t, const Mat2<float>& m, hipStream_t s) {
  if (t >= 1 && t <= g_shuffle_bits && n >= 7) {
    // contiguous vectors, partners by shuffle: streams like bit 0
    const uint64_t units = uint64_t(1) << (n - 1);
    launch_nt(stream_sweep(n, 8, 6), k_1q_f_shfl<true>, k_1q_f_shfl<false>, grid_for(units), s,
              a, units, t, m, uint64_t(0), uint64_t(0));
    return hipGetLastError();
  }
  const bool nt = stream_sweep(n, 8, t == 0 ? 6 : t);
  if (t == 0) {
    const uint64_t units = uint64_t(1) << (n - 1);
    launch_nt(nt, k_1q_f_bit0<true>, k_1q_f_bit0<false>, grid_for(units), s, a, units, m,
              uint64_t(0), uint64_t(0));
  } else {
    const uint64_t units = uint64_t(1) << (n - 2);
    launch_nt(nt, k_1q_f_vec<true>, k_1q_f_vec<false>, grid_for(units), s, a, units, t, m,
              uint64_t(0), uint64_t(0));
  }
  return hipGetLastError();
}

template <>
hipError_t launch_apply_1q<double>(double* a, int n, int t, const Mat2<double>& m,
                                   hipStream_t s) {
  const uint64_t units = uint64_t(1) << (n - 1);
  launch_nt(stream_sweep(n, 16, t), k_1q_d<true>, k_1q_d<false>, grid_for(units), s, a, units,
            t, m);
  return hipGetLastError();
}

// A singly controlled complex64 gate whose control bit is below 3: the sparse
// sweep would touch 16-32-byte pieces of the half it changes, and the memory
// system move whole segments around them anyway, so the whole state is swept
// as for a one-qubit gate on the target (contiguous, streaming) with the
// matrix applied where the control matches. At 30 qubits: control 0-2,
// target 22: 3.1 against 3.4 ms; control 1, target 0: 2.7 against 3.3 ms.
// With the control at bit 3 or above the sparse sweep reads the changed half
// in long runs whatever the target (control 22, target 0-2: 1.5 against
// 2.7 ms dense) and is kept.
bool ctrl_dense(float* a, int n, const BitSet16& fixed, uint64_t set_mask, int tbit,
                const Mat2<float>& m, hipStream_t s) {
  if (!g_dense_ctrl || fixed.n != 2 || n < 7) return false;
  const int cbit = fixed.pos[0] == tbit ? fixed.pos[1] : fixed.pos[0];
  if (cbit >= 3) return false;
  const uint64_t cmask = uint64_t(1) << cbit, cval = set_mask & cmask;
  const bool nt = stream_sweep(n, 8, 6);
  if (tbit == 0) {
    const uint64_t units = uint64_t(1) << (n - 1);
    launch_nt(nt, k_1q_f_bit0<true, true>, k_1q_f_bit0<false, true>, grid_for(units), s, a,
              units, m, cmask, cval);
  } else if (tbit <= g_shuffle_bits) {
    const uint64_t units = uint64_t(1) << (n - 1);
    launch_nt(nt, k_1q_f_shfl<true, true>, k_1q_f_shfl<false, true>, grid_for(units), s, a,
              units, tbit, m, cmask, cval);
  } else {
    const uint64_t units = uint64_t(1) << (n - 2);
    launch_nt(nt, k_1q_f_vec<true, true>, k_1q_f_vec<false, true>, grid_for(units), s, a,
              units, tbit, m, cmask, cval);
  }
  return true;
}

template <typename R>
hipError_t launch_apply_ctrl(R* a, int n, const BitSet16& fixed, uint64_t set_mask, int tbit,
                             const Mat2<R>& m, hipStream_t s) {
  if constexpr (sizeof(R) == 4)
    if (ctrl_dense(a, n, fixed, set_mask, tbit, m, s)) return hipGetLastError();
  const int free_bits = n - fixed.n;
  const bool nt = stream_sweep(n, 2 * sizeof(R), fixed.pos[0]);
  if (fixed.pos[0] >= log_amps<R>() && free_bits >= log_amps<R>()) {
    const uint64_t units = (uint64_t(1) << free_bits) / Vec16<R>::AMPS;
    launch_nt(nt, k_ctrl_vec<R, true>, k_ctrl_vec<R, false>, grid_for(units), s,
              a, units, fixed, set_mask, tbit, m);
  } else {
    const uint64_t units = uint64_t(1) << free_bits;
    launch_nt(nt, k_ctrl_scalar<R, true>, k_ctrl_scalar<R, false>, grid_for(units), s,
              a, units, fixed, set_mask, tbit, m);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_cphase(R* a, int n, int qa, int qb, R cr, R ci, hipStream_t s) {
  const BitSet16 fixed = sorted_bits({qa, qb});
  const uint64_t set_mask = (uint64_t(1) << qa) | (uint64_t(1) << qb);
  const int free_bits = n - 2;
  const bool nt = stream_sweep(n, 2 * sizeof(R), fixed.pos[0]);
  if (fixed.pos[0] >= log_amps<R>() && free_bits >= log_amps<R>()) {
    const uint64_t units = (uint64_t(1) << free_bits) / Vec16<R>::AMPS;
    launch_nt(nt, k_cphase_vec<R, true>, k_cphase_vec<R, false>, grid_for(units), s,
              a, units, fixed, set_mask, cr, ci);
  } else {
    const uint64_t units = uint64_t(1) << free_bits;
    launch_nt(nt, k_cphase_scalar<R, true>, k_cphase_scalar<R, false>, grid_for(units), s,
              a, units, fixed, set_mask, cr, ci);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_bitswap(R* a, int n, int qa, int qb, hipStream_t s) {
  const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
  const BitSet16 fixed = sorted_bits({lo, hi});
  const int free_bits = n - 2;
  const bool nt = stream_sweep(n, 2 * sizeof(R), lo);
  if (lo >= log_amps<R>() && free_bits >= log_amps<R>()) {
    const uint64_t units = (uint64_t(1) << free_bits) / Vec16<R>::AMPS;
    launch_nt(nt, k_bitswap_vec<R, true>, k_bitswap_vec<R, false>, grid_for(units), s,
              a, units, fixed, lo, hi);
  } else {
    const uint64_t units = uint64_t(1) << free_bits;
    launch_nt(nt, k_bitswap_scalar<R, true>, k_bitswap_scalar<R, false>, grid_for(units), s,
              a, units, fixed, lo, hi);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t launch_set_basis(R* a, int n, uint64_t x, hipStream_t s) {
  const uint64_t units = ((uint64_t(1) << n) + Vec16<R>::AMPS - 1) / Vec16<R>::AMPS;
  hipLaunchKernelGGL(k_set_basis<R>, dim3(grid_for(units)), dim3(kBlock), 0, s, a, units, x);
  return hipGetLastError();
}

template <typename Rd, typename Rs>
hipError_t launch_convert(Rd* d, const Rs* src, uint64_t count, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<Rd, Rs>), dim3(grid_for(count)), dim3(kBlock), 0, s, d, src,
                     count);
  return hipGetLastError();
}

template hipError_t launch_apply_ctrl<float>(float*, int, const BitSet16&, uint64_t, int,
                                             const Mat2<float>&, hipStream_t);
template hipError_t launch_apply_ctrl<double>(double*, int, const BitSet16&, uint64_t, int,
                                              const Mat2<double>&, hipStream_t);
template hipError_t launch_cphase<float>(float*, int, int, int, float, float, hipStream_t);
template hipError_t launch_cphase<double>(double*, int, int, int, double, double, hipStream_t);
template hipError_t launch_bitswap<float>(float*, int, int, int, hipStream_t);
template hipError_t launch_bitswap<double>(double*, int, int, int, hipStream_t);
template hipError_t launch_set_basis<float>(float*, int, uint64_t, hipStream_t);
template hipError_t launch_set_basis<double>(double*, int, uint64_t, hipStream_t);
template hipError_t launch_convert<float, double>(float*, const double*, uint64_t, hipStream_t);
template hipError_t launch_convert<double, double>(double*, const double*, uint64_t, hipStream_t);
template hipError_t launch_convert<float, float>(float*, const float*, uint64_t, hipStream_t);
template hipError_t launch_convert<double, float>(double*, const float*, uint64_t, hipStream_t);

}  // namespace qs
