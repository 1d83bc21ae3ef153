// Quantum Fourier transform as multi-stage passes over the dense ket.
//
// The QFT circuit (Sec. II-E) is, for each qubit j of the range from the top
// down, H on j followed by controlled phases pi/2^(j-m) from every lower qubit
// m of the range, and a final bit reversal. The phases of stage j together
// multiply every amplitude whose bit j is set by e^{i pi u / 2^(j-start)},
// u = the range bits below j. A stage is therefore a butterfly on one bit plus
// a diagonal twiddle, and consecutive stages can run on data held on-chip:
//
//  * register pass (bits at or above the LDS tile): each thread holds the 2^G
//    amplitudes that differ in bits [lo, lo+G) and performs G stages in
//    registers; lanes run along the low index bits, so each wavefront
//    load/store covers contiguous memory.
//  * LDS pass (bits below T): a workgroup loads a contiguous 2^T tile,
//    performs every stage of those bits in LDS, in register rounds of up to 4
//    bits, and writes the tile back.
//
// Orientation. The final bit reversal is a relabelling, so the range arrives
// either in natural order or bit-reversed (after a previous transform). In
// natural order the stages run from the top bit down and the twiddle of a
// stage depends on the bits below it. Bit-reversed, logical qubit j lives at
// physical bit start+len-1-(j-start): the stages run from the bottom bit up
// and the twiddle of the stage at bit a is e^{i pi sum_{d>=1} bit(a+d)/2^d},
// a binary fraction of the bits above it. Both cost one sweep per pass, so
// back-to-back transforms never move data for the relabelling.
//
// Twiddles. Inside a pass the twiddle of the stage at bit lo+jj factors into
// a root of unity fixed by the pass-local bits (a 32-entry table computed in
// float64 on the host) times a per-thread factor of the bits outside the pass,
// computed once per thread and stage with sincospi on an exactly
// representable argument below 1.
//
// Scaling. The butterflies are unscaled (x+y, x-y); each pass multiplies by an
// exact power of two so that the passes together scale by 2^(-len/2) (one
// rounded 1/sqrt(2) when len is odd). Rounding 1/sqrt(2) in every butterfly
// would shrink the norm by ~3.4e-8 per stage in float32.
//
// The inverse transform is the complex conjugate of the forward one (the DFT
// matrix is symmetric), so it runs the same passes with conjugated twiddles.
#include "qs_internal.h"

namespace qs {
namespace {

constexpr int kBlock = 256;

template <typename R>
struct Roots32 {
  R re[32];
  R im[32];
};

template <typename R> struct Cx { R r, i; };
template <typename R> struct Vec8;
template <> struct Vec8<float> { using T = float2; };
template <> struct Vec8<double> { using T = double2; };

__device__ __forceinline__ void sc_pi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ __forceinline__ void sc_pi(double x, double* s, double* c) { sincospi(x, s, c); }

template <typename R>
__device__ __forceinline__ Cx<R> cmul(Cx<R> a, Cx<R> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}

constexpr int rev_bits(int x, int k) {
  int r = 0;
  for (int i = 0; i < k; ++i) r |= ((x >> i) & 1) << (k - 1 - i);
  return r;
}

// Natural order: stages jj = G-1 .. 0 on v[0 .. 2^G) held by one thread.
// ls = (index bits below lo) >> start, e0 = lo - start.
template <typename R, int G>
__device__ __forceinline__ void stages_fwd(Cx<R> (&v)[1 << G], uint64_t ls, int e0, int sign,
                                           const Roots32<R>& rt) {
  const R lsr = R(ls);
  Cx<R> tw[G > 1 ? (1 << (G - 1)) : 1];
#pragma unroll
  for (int jj = G - 1; jj >= 0; --jj) {
    R s, c;
    sc_pi(lsr * R(sign) * ldexp(R(1), -(e0 + jj)), &s, &c);
    const Cx<R> w{c, s};
#pragma unroll
    for (int k = 0; k < (1 << jj); ++k) {
      const int idx = k << (5 - jj);
      tw[k] = cmul(Cx<R>{rt.re[idx], R(sign) * rt.im[idx]}, w);
    }
#pragma unroll
    for (int m = 0; m < (1 << G); ++m) {
      if (m & (1 << jj)) continue;
      const int m1 = m | (1 << jj);
      const Cx<R> x = v[m], y = v[m1];
      v[m] = {x.r + y.r, x.i + y.i};
      v[m1] = cmul(Cx<R>{x.r - y.r, x.i - y.i}, tw[m & ((1 << jj) - 1)]);
    }
  }
}

// Bit-reversed order: stages jj = 0 .. G-1. hx = the range bits above the
// pass, bit-reversed (H of them).
template <typename R, int G>
__device__ __forceinline__ void stages_rev(Cx<R> (&v)[1 << G], uint64_t hx, int H, int sign,
                                           const Roots32<R>& rt) {
  const R hxr = R(hx);
  Cx<R> tw[G > 1 ? (1 << (G - 1)) : 1];
#pragma unroll
  for (int jj = 0; jj < G; ++jj) {
    R s = 0, c = 1;
    if (H > 0) sc_pi(hxr * R(sign) * ldexp(R(1), -(H - 1 + G - jj)), &s, &c);
    const Cx<R> w{c, s};
    const int kb = G - 1 - jj;  // pass bits above jj
#pragma unroll
    for (int k = 0; k < (1 << kb); ++k) {
      const int idx = kb > 0 ? (rev_bits(k, kb) << (5 - kb)) : 0;
      tw[k] = cmul(Cx<R>{rt.re[idx], R(sign) * rt.im[idx]}, w);
    }
#pragma unroll
    for (int m = 0; m < (1 << G); ++m) {
      if (m & (1 << jj)) continue;
      const int m1 = m | (1 << jj);
      const Cx<R> x = v[m], y = v[m1];
      v[m] = {x.r + y.r, x.i + y.i};
      v[m1] = cmul(Cx<R>{x.r - y.r, x.i - y.i}, tw[m >> (jj + 1)]);
    }
  }
}

// Stages of the bits [lo, lo+G) for the amplitudes of one thread; xg is the
// global index of its element 0.
template <typename R, int G, bool REV>
__device__ __forceinline__ void pass_stages(Cx<R> (&v)[1 << G], uint64_t xg, int start, int len,
                                            int lo, int sign, const Roots32<R>& rt) {
  if constexpr (REV) {
    const int H = start + len - lo - G;
    uint64_t hx = 0;
    if (H > 0) {
      const uint64_t hf = (xg >> (lo + G)) & ((uint64_t(1) << H) - 1);
      hx = __builtin_bitreverse64(hf) >> (64 - H);
    }
    stages_rev<R, G>(v, hx, H, sign, rt);
  } else {
    const uint64_t ls = (xg & ((uint64_t(1) << lo) - 1)) >> start;
    stages_fwd<R, G>(v, ls, lo - start, sign, rt);
  }
}

// ------------------------------------------------------------------ register pass
template <typename R, int G, bool REV>
__global__ void __launch_bounds__(kBlock) k_qft_reg(R* __restrict__ a, int n, int start, int len,
                                                    int lo, int sign, R scale, Roots32<R> rt) {
  using V = typename Vec8<R>::T;
  const uint64_t r = uint64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (r >= (uint64_t(1) << (n - G))) return;
  const uint64_t l = r & ((uint64_t(1) << lo) - 1);
  const uint64_t base = ((r >> lo) << (lo + G)) | l;
  V* p = reinterpret_cast<V*>(a) + base;
  const uint64_t stride = uint64_t(1) << lo;
  Cx<R> v[1 << G];
#pragma unroll
  for (int m = 0; m < (1 << G); ++m) {
    const V t = p[m * stride];
    v[m] = {t.x, t.y};
  }
  pass_stages<R, G, REV>(v, base, start, len, lo, sign, rt);
#pragma unroll
  for (int m = 0; m < (1 << G); ++m) {
    V t;
    t.x = v[m].r * scale;
    t.y = v[m].i * scale;
    p[m * stride] = t;
  }
}

// ------------------------------------------------------------------ LDS pass
// LDS position of tile index x: one complex of padding every 16 keeps strided
// column reads spread over the banks.
__device__ __forceinline__ int lds_pos(int x) { return x + (x >> 4); }

template <typename R, int W, bool REV>
__device__ __forceinline__ void lds_group(Cx<R>* sm, uint64_t tile_base, int T, int start,
                                          int len, int g0, int sign, const Roots32<R>& rt) {
  const int g1 = g0 + W;
  const int cols = 1 << (T - W);
  for (int c = threadIdx.x; c < cols; c += kBlock) {
    const int cl = c & ((1 << g0) - 1);
    const int ch = c >> g0;
    const int xb = (ch << g1) | cl;
    Cx<R> v[1 << W];
#pragma unroll
    for (int m = 0; m < (1 << W); ++m) v[m] = sm[lds_pos(xb | (m << g0))];
    pass_stages<R, W, REV>(v, tile_base | uint64_t(xb), start, len, g0, sign, rt);
#pragma unroll
    for (int m = 0; m < (1 << W); ++m) sm[lds_pos(xb | (m << g0))] = v[m];
  }
}

template <typename R, bool REV>
__device__ __forceinline__ void lds_round(Cx<R>* sm, uint64_t tile_base, int T, int start,
                                          int len, int g0, int w, int sign,
                                          const Roots32<R>& rt) {
  switch (w) {
    case 1: lds_group<R, 1, REV>(sm, tile_base, T, start, len, g0, sign, rt); break;
    case 2: lds_group<R, 2, REV>(sm, tile_base, T, start, len, g0, sign, rt); break;
    case 3: lds_group<R, 3, REV>(sm, tile_base, T, start, len, g0, sign, rt); break;
    default: lds_group<R, 4, REV>(sm, tile_base, T, start, len, g0, sign, rt); break;
  }
}

// Stages of the bits [start, hi) on a 2^T tile; hi <= T.
template <typename R, bool REV>
__global__ void __launch_bounds__(kBlock) k_qft_lds(R* __restrict__ a, int T, int start, int len,
                                                    int hi, int sign, R scale, Roots32<R> rt) {
  extern __shared__ unsigned char smraw[];
  Cx<R>* sm = reinterpret_cast<Cx<R>*>(smraw);
  using V = typename Vec8<R>::T;
  const uint64_t tile_base = uint64_t(blockIdx.x) << T;
  V* p = reinterpret_cast<V*>(a) + tile_base;
  const int tile = 1 << T;
  for (int x = threadIdx.x; x < tile; x += kBlock) {
    const V t = p[x];
    sm[lds_pos(x)] = {t.x, t.y};
  }
  __syncthreads();
  if constexpr (REV) {
    // bottom-up rounds: the lowest round takes the remainder of (hi-start)/4
    int g0 = start;
    int first = (hi - start) % 4;
    if (first == 0) first = 4;
    for (int w = first; g0 < hi; g0 += w, w = 4) {
      lds_round<R, REV>(sm, tile_base, T, start, len, g0, w, sign, rt);
      __syncthreads();
    }
  } else {
    for (int g1 = hi; g1 > start;) {
      const int w = (g1 - start) < 4 ? (g1 - start) : 4;
      const int g0 = g1 - w;
      lds_round<R, REV>(sm, tile_base, T, start, len, g0, w, sign, rt);
      __syncthreads();
      g1 = g0;
    }
  }
  for (int x = threadIdx.x; x < tile; x += kBlock) {
    const Cx<R> v = sm[lds_pos(x)];
    V t;
    t.x = v.r * scale;
    t.y = v.i * scale;
    p[x] = t;
  }
}

template <typename R>
Roots32<R> make_roots() {
  Roots32<R> rt;
  for (int k = 0; k < 32; ++k) {
    // e^{i pi k / 32}, evaluated in float64 and rounded once
    const double ang = 3.14159265358979323846 * double(k) / 32.0;
    rt.re[k] = static_cast<R>(cos(ang));
    rt.im[k] = static_cast<R>(sin(ang));
  }
  return rt;
}

template <typename R> constexpr int tile_bits() { return sizeof(R) == 4 ? 12 : 11; }
constexpr int kRegMax = 5;

template <typename R, int G, bool REV>
hipError_t launch_reg(R* a, int n, int start, int len, int lo, int sign, R scale,
                      const Roots32<R>& rt, hipStream_t s) {
  const uint64_t threads = uint64_t(1) << (n - G);
  const unsigned grid = static_cast<unsigned>((threads + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_qft_reg<R, G, REV>), dim3(grid), dim3(kBlock), 0, s, a, n, start, len, lo,
                     sign, scale, rt);
  return hipGetLastError();
}

template <typename R, bool REV>
hipError_t launch_pass(R* a, int n, int start, int len, int lo, int hi, int sign, R scale,
                       hipStream_t s) {
  const Roots32<R> rt = make_roots<R>();
  const int T = n < tile_bits<R>() ? n : tile_bits<R>();
  if (hi <= T) {
    if (lo != start) return hipErrorInvalidValue;
    const size_t shmem = size_t((1 << T) + ((1 << T) >> 4)) * 2 * sizeof(R);
    const unsigned grid = static_cast<unsigned>(uint64_t(1) << (n - T));
    hipLaunchKernelGGL((k_qft_lds<R, REV>), dim3(grid), dim3(kBlock), shmem, s, a, T, start, len,
                       hi, sign, scale, rt);
    return hipGetLastError();
  }
  if (lo < T) return hipErrorInvalidValue;
  switch (hi - lo) {
    case 1: return launch_reg<R, 1, REV>(a, n, start, len, lo, sign, scale, rt, s);
    case 2: return launch_reg<R, 2, REV>(a, n, start, len, lo, sign, scale, rt, s);
    case 3: return launch_reg<R, 3, REV>(a, n, start, len, lo, sign, scale, rt, s);
    case 4: return launch_reg<R, 4, REV>(a, n, start, len, lo, sign, scale, rt, s);
    case 5: return launch_reg<R, 5, REV>(a, n, start, len, lo, sign, scale, rt, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

template <typename R>
hipError_t launch_qft_pass(R* a, int n, int start, int len, int lo, int hi, int sign, bool rev,
                           double scale, hipStream_t s) {
  return rev ? launch_pass<R, true>(a, n, start, len, lo, hi, sign, R(scale), s)
             : launch_pass<R, false>(a, n, start, len, lo, hi, sign, R(scale), s);
}

template hipError_t launch_qft_pass<float>(float*, int, int, int, int, int, int, bool, double,
                                           hipStream_t);
template hipError_t launch_qft_pass<double>(double*, int, int, int, int, int, int, bool, double,
                                            hipStream_t);

// Pass plan of a QFT on [start, start+len): register passes of near-equal
// width over the bits at or above the LDS tile and one LDS pass over the bits
// below it; top-down in natural order, bottom-up when bit-reversed. Each pass
// gets an exact power-of-two scale, the last one also 1/sqrt(2) if len is odd.
template <typename R>
int qft_plan(int n, int start, int len, bool rev, QftPass* out, int max_passes) {
  const int T = n < tile_bits<R>() ? n : tile_bits<R>();
  const int top = start + len;
  const int reg_lo = start > T ? start : T;
  int np = 0;
  if (top > reg_lo) {
    const int width = top - reg_lo;
    const int passes = (width + kRegMax - 1) / kRegMax;
    int cur = top;
    for (int k = 0; k < passes; ++k) {
      const int left = passes - k;
      const int w = (cur - reg_lo + left - 1) / left;
      if (np >= max_passes) return -1;
      out[np].lo = cur - w;
      out[np].hi = cur;
      ++np;
      cur -= w;
    }
  }
  if (start < T) {
    if (np >= max_passes) return -1;
    out[np].lo = start;
    out[np].hi = top < T ? top : T;
    ++np;
  }
  if (rev)
    for (int i = 0; i < np / 2; ++i) {
      const QftPass t = out[i];
      out[i] = out[np - 1 - i];
      out[np - 1 - i] = t;
    }
  int acc = 0;
  for (int i = 0; i < np; ++i) {
    const int g = out[i].hi - out[i].lo;
    const int e = (acc + g) / 2 - acc / 2;
    acc += g;
    out[i].scale = ldexp(1.0, -e);
    if (i == np - 1 && (len & 1)) out[i].scale *= 0.70710678118654752440;
  }
  return np;
}

template int qft_plan<float>(int, int, int, bool, QftPass*, int);
template int qft_plan<double>(int, int, int, bool, QftPass*, int);

}  // namespace qs
