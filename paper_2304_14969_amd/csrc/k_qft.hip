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
// Twiddles. Inside a round of W consecutive bits, the twiddle of each stage
// factors into a root of unity fixed by the round's own bits and a factor of
// the bits outside the round. The roots are compile-time constants once the
// butterfly loops are unrolled (nothing for a zero angle, a swap for pi/2, a
// product with literal cosines otherwise). The outside factors commute with
// the round's later butterflies, so they are applied once after them: the
// amplitude at round index m gets w^e(m) (e(m) = m bit-reversed in natural
// order, m in bit-reversed order), w from one sincospi of an argument in
// [0, 1), an integer of the range bits outside the round times a power of
// two, and its powers by squaring. The argument is exact while that integer
// has at most 24 significant bits (in float32; 53 in float64); in longer
// float32 ranges it is rounded once, a phase error below pi * 2^-24
// (1.9e-7 rad), the size of the rounding of the sine and cosine themselves;
// the powers add at most 2W roundings.
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

// cos(pi j / 32), j = 0 .. 16 (float64 literals, rounded once to R where used)
__device__ constexpr double kCos32[17] = {
    1.0, 0.99518472667219693, 0.98078528040323043, 0.95694033573220882,
    0.92387953251128674, 0.88192126434835505, 0.83146961230254524, 0.77301045336273699,
    0.70710678118654757, 0.63439328416364549, 0.55557023301960229, 0.47139673682599781,
    0.38268343236508984, 0.29028467725446233, 0.19509032201612833, 0.09801714032956077,
    0.0};

// x * e^{i pi SIGN k / 2^b} for 0 <= k < 2^b <= 32, with k and b known at
// compile time once the butterfly loops are unrolled: nothing for k = 0, a
// swap for pi/2, a complex product with literal constants otherwise.
template <typename R, int SIGN>
__device__ __forceinline__ Cx<R> rot(Cx<R> x, int k, int b) {
  if (k == 0) return x;
  const int a = k << (5 - b);  // angle in units of pi/32, in (0, 32)
  if (a == 16) return SIGN > 0 ? Cx<R>{-x.i, x.r} : Cx<R>{x.i, -x.r};
  const R c = R(a < 16 ? kCos32[a] : -kCos32[32 - a]);
  const R s = R(SIGN) * R(a < 16 ? kCos32[16 - a] : kCos32[a - 16]);
  return {x.r * c - x.i * s, x.r * s + x.i * c};
}

// The butterflies of G consecutive stages on the 2^G amplitudes of one thread
// with the twiddles of the bits inside the group only (constants).
// Natural order: stages jj = G-1 .. 0; stage jj is the butterfly on bit jj,
// then e^{i pi u / 2^jj} on the amplitudes with bit jj set, u = bits below jj.
// Bit-reversed order: stages jj = 0 .. G-1; the twiddle is
// e^{i pi sum_{d>=1} bit(jj+d) / 2^d} over the bits above jj.
template <typename R, int G, bool REV, int SIGN>
__device__ __forceinline__ void local_stages(Cx<R> (&v)[1 << G]) {
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const int jj = REV ? t : G - 1 - t;
#pragma unroll
    for (int m = 0; m < (1 << G); ++m) {
      if (m & (1 << jj)) continue;
      const int m1 = m | (1 << jj);
      const Cx<R> x = v[m], y = v[m1];
      v[m] = {x.r + y.r, x.i + y.i};
      const Cx<R> d{x.r - y.r, x.i - y.i};
      if (REV) {
        const int kb = G - 1 - jj;  // bits above jj
        v[m1] = rot<R, SIGN>(d, rev_bits(m >> (jj + 1), kb), kb);
      } else {
        v[m1] = rot<R, SIGN>(d, m & ((1 << jj) - 1), jj);
      }
    }
  }
}

// The twiddles of the bits outside the group. Each stage's factor from those
// bits multiplies the amplitudes with the stage's own bit set and commutes
// with the group's later butterflies (they act on other bits), so all of them
// are applied after the butterflies: amplitude m gets w^e(m), with
// e(m) = m bit-reversed (natural order) or m (bit-reversed order), and
// w = e^{i pi SIGN f} from one sincospi of an exact argument f. The powers
// are built by squaring and by one more factor w (at most 2 G products).
template <typename R, int G, bool REV>
__device__ __forceinline__ void outer_twiddles(Cx<R> (&v)[1 << G], R f) {
  R s, c;
  sc_pi(f, &s, &c);
  Cx<R> pw[1 << G];
  pw[1] = {c, s};
#pragma unroll
  for (int k = 2; k < (1 << G); ++k)
    pw[k] = (k & 1) ? cmul(pw[k - 1], pw[1]) : cmul(pw[k >> 1], pw[k >> 1]);
#pragma unroll
  for (int m = 1; m < (1 << G); ++m) v[m] = cmul(v[m], pw[REV ? m : rev_bits(m, G)]);
}

// Stages of the bits [lo, lo+G) for the amplitudes of one thread; xg is the
// global index of its element 0.
template <typename R, int G, bool REV, int SIGN>
__device__ __forceinline__ void pass_stages_s(Cx<R> (&v)[1 << G], uint64_t xg, int start,
                                              int len, int lo) {
  local_stages<R, G, REV, SIGN>(v);
  if constexpr (REV) {
    // bits above the group, bit-reversed: hx / 2^H is their binary fraction
    const int H = start + len - lo - G;
    if (H > 0) {
      const uint64_t hf = (xg >> (lo + G)) & ((uint64_t(1) << H) - 1);
      const uint64_t hx = __builtin_bitreverse64(hf) >> (64 - H);
      outer_twiddles<R, G, REV>(v, R(SIGN) * R(hx) * ldexp(R(1), -(H + G - 1)));
    }
  } else {
    // range bits below the group: ls / 2^(lo-start) is their binary fraction
    const int e0 = lo - start;
    if (e0 > 0) {
      const uint64_t ls = (xg & ((uint64_t(1) << lo) - 1)) >> start;
      outer_twiddles<R, G, REV>(v, R(SIGN) * R(ls) * ldexp(R(1), -(e0 + G - 1)));
    }
  }
}

template <typename R, int G, bool REV>
__device__ __forceinline__ void pass_stages(Cx<R> (&v)[1 << G], uint64_t xg, int start, int len,
                                            int lo, int sign) {
  if (sign > 0)
    pass_stages_s<R, G, REV, 1>(v, xg, start, len, lo);
  else
    pass_stages_s<R, G, REV, -1>(v, xg, start, len, lo);
}

// ------------------------------------------------------------------ register pass
template <typename R, int G, bool REV>
__global__ void __launch_bounds__(kBlock) k_qft_reg(R* __restrict__ a, int n, int start, int len,
                                                    int lo, int sign, R scale) {
  using V = typename Vec8<R>::T;
  const uint64_t total = uint64_t(1) << (n - G);
  for (uint64_t r = uint64_t(blockIdx.x) * kBlock + threadIdx.x; r < total;
       r += uint64_t(gridDim.x) * kBlock) {
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
    pass_stages<R, G, REV>(v, base, start, len, lo, sign);
#pragma unroll
    for (int m = 0; m < (1 << G); ++m) {
      V t;
      t.x = v[m].r * scale;
      t.y = v[m].i * scale;
      p[m * stride] = t;
    }
  }
}

// ------------------------------------------------------------------ LDS tiles
// Both LDS kernels stage a tile of 2^TB amplitudes, run the pass's stages in
// register rounds of up to 5 bits (each thread takes the 2^W amplitudes of
// one column of the round), and write the tile back scaled. Global loads are
// issued as a batch of 16-byte vectors before any LDS write.

template <typename R> struct Vec16;
template <> struct Vec16<float> { using T = float4; static constexpr int AMPS = 2; };
template <> struct Vec16<double> { using T = double2; static constexpr int AMPS = 1; };

// Streaming 16-byte global accesses: each pass reads and writes every byte
// once, so both are non-temporal. In whole-state sweeps of the passes' tile
// shapes this moves 7% more bytes per second than plain accesses (top 8-bit
// strided tiles 5.15 -> 5.54 TB/s, contiguous 64 KiB tiles 5.43 -> 5.80).
// Buffer instructions with stores at device or system scope did better still
// in those sweeps, but not inside the passes (1-3% slower: each access then
// needs its wave's base address in scalar registers). States that fit the
// 256 MiB last-level cache keep plain accesses: back-to-back passes find part
// of the state there, and streaming made the QFT at 22-25 qubits 4-7% slower.
// The kernels take the choice as a (uniform) argument.

// LDS position of tile index x; one complex of padding every 16 entries keeps
// the strided columns of the lowest rounds on distinct banks.
template <bool PAD>
__device__ __forceinline__ int lds_pos(int x) { return PAD ? x + (x >> 4) : x; }

// Round over the tile bits [b0, b0+W): column q owns the 2^W entries that
// differ in those bits. Entry (tile index) -> global index via `glob`.
template <typename R, int W, bool REV, bool PAD, int NT, typename Glob>
__device__ __forceinline__ void tile_round(Cx<R>* sm, int TB, int b0, int start, int len,
                                           int glo, int sign, Glob glob) {
  const int cols = 1 << (TB - W);
  for (int q = threadIdx.x; q < cols; q += NT) {
    const int x0 = (q & ((1 << b0) - 1)) | ((q >> b0) << (b0 + W));
    Cx<R> v[1 << W];
#pragma unroll
    for (int m = 0; m < (1 << W); ++m) v[m] = sm[lds_pos<PAD>(x0 | (m << b0))];
    pass_stages<R, W, REV>(v, glob(x0), start, len, glo, sign);
#pragma unroll
    for (int m = 0; m < (1 << W); ++m) sm[lds_pos<PAD>(x0 | (m << b0))] = v[m];
  }
}

// Round count for `bits` tile bits with rounds of at most WMAX bits.
__host__ __device__ constexpr int round_count(int bits, int wmax) {
  return bits <= 0 ? 0 : (bits + wmax - 1) / wmax;
}
// Widest round of that split (the rounds are balanced).
__host__ __device__ constexpr int round_width(int bits, int wmax) {
  return bits <= 0 ? 0 : (bits + round_count(bits, wmax) - 1) / round_count(bits, wmax);
}

// Runs the rounds covering tile bits [b_lo, b_hi) (global bits glo_base +
// (b - b_lo)): balanced widths <= WMAX, top-down in natural order, bottom-up
// when bit-reversed.
template <typename R, bool REV, bool PAD, int NT, int WMAX, typename Glob>
__device__ __forceinline__ void tile_rounds(Cx<R>* sm, int TB, int b_lo, int b_hi, int glo_base,
                                            int start, int len, int sign,
                                            Glob glob) {
  const int bits = b_hi - b_lo;
  const int rounds = round_count(bits, WMAX);
  for (int k = 0; k < rounds; ++k) {
    // widths: the first (bits % rounds) rounds, counted from the top, get one more
    const int base_w = bits / rounds, extra = bits % rounds;
    const int kk = REV ? rounds - 1 - k : k;   // index from the top
    int top = b_hi;
    for (int i = 0; i < kk; ++i) top -= base_w + (i < extra ? 1 : 0);
    const int w = base_w + (kk < extra ? 1 : 0);
    const int b0 = top - w;
    const int glo = glo_base + (b0 - b_lo);
    switch (w) {
      case 1: tile_round<R, 1, REV, PAD, NT>(sm, TB, b0, start, len, glo, sign, glob); break;
      case 2: tile_round<R, 2, REV, PAD, NT>(sm, TB, b0, start, len, glo, sign, glob); break;
      case 3: tile_round<R, 3, REV, PAD, NT>(sm, TB, b0, start, len, glo, sign, glob); break;
      case 4: tile_round<R, 4, REV, PAD, NT>(sm, TB, b0, start, len, glo, sign, glob); break;
      default:
        if constexpr (WMAX >= 5)
          tile_round<R, 5, REV, PAD, NT>(sm, TB, b0, start, len, glo, sign, glob);
        break;
    }
    __syncthreads();
  }
}

// Contiguous tile [0, T): stages of the bits [lo, hi), hi <= T.
// Two workgroups of a complex64 tile (2 x 68 KiB) share a CU; the bound of
// two waves per SIMD (at most 256 VGPRs) keeps both resident.
template <typename R, int T, bool REV, int NT, int WMAX>
__global__ void __launch_bounds__(NT, sizeof(R) == 4 ? 2 : 1)
    k_qft_lds(R* __restrict__ a, int start, int len, int lo, int hi, int sign, R scale,
              int stream) {
  extern __shared__ unsigned char smraw[];
  Cx<R>* sm = reinterpret_cast<Cx<R>*>(smraw);
  using V = typename Vec16<R>::T;
  constexpr int AP = Vec16<R>::AMPS;
  constexpr int NV = (1 << T) / AP / NT;  // vectors per thread
  static_assert(NV >= 1, "tile smaller than the block");
  const uint64_t tile_base = uint64_t(blockIdx.x) << T;
  V* p = reinterpret_cast<V*>(a + 2 * tile_base);
  V buf[NV];
  if (stream) {
#pragma unroll
    for (int k = 0; k < NV; ++k) buf[k] = ld16<true>(p + threadIdx.x + k * NT);
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) buf[k] = p[threadIdx.x + k * NT];
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int x = (threadIdx.x + k * NT) * AP;
    if constexpr (AP == 2) {
      sm[lds_pos<true>(x)] = {buf[k].x, buf[k].y};
      sm[lds_pos<true>(x + 1)] = {buf[k].z, buf[k].w};
    } else {
      sm[lds_pos<true>(x)] = {buf[k].x, buf[k].y};
    }
  }
  __syncthreads();
  tile_rounds<R, REV, true, NT, WMAX>(sm, T, lo, hi, lo, start, len, sign,
                                      [tile_base](int x) { return tile_base | uint64_t(x); });
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int x = (threadIdx.x + k * NT) * AP;
    const Cx<R> v0 = sm[lds_pos<true>(x)];
    if constexpr (AP == 2) {
      const Cx<R> v1 = sm[lds_pos<true>(x + 1)];
      buf[k] = {v0.r * scale, v0.i * scale, v1.r * scale, v1.i * scale};
    } else {
      buf[k] = {v0.r * scale, v0.i * scale};
    }
  }
  if (stream) {
#pragma unroll
    for (int k = 0; k < NV; ++k) st16<true>(p + threadIdx.x + k * NT, buf[k]);
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) p[threadIdx.x + k * NT] = buf[k];
  }
}

// Strided tile: 2^G rows (global bits [lo, lo+G)) x 2^C contiguous columns
// (global bits [0, C)), C <= lo. Tile index = row * 2^C + column.
template <typename R, int G, int C, bool REV, int NT, int WMAX>
__global__ void __launch_bounds__(NT) k_qft_col(R* __restrict__ a, int start, int len, int lo,
                                                int sign, R scale, int stream) {
  extern __shared__ unsigned char smraw[];
  Cx<R>* sm = reinterpret_cast<Cx<R>*>(smraw);
  using V = typename Vec16<R>::T;
  constexpr int AP = Vec16<R>::AMPS;
  constexpr int TB = G + C;
  constexpr int VPR = (1 << C) / AP;        // vectors per row
  constexpr int NV = (1 << TB) / AP / NT;   // vectors per thread
  static_assert(NV >= 1 && VPR >= 1, "tile shape");
  const uint64_t b = blockIdx.x;
  const uint64_t mid = b & ((uint64_t(1) << (lo - C)) - 1);
  const uint64_t hi = b >> (lo - C);
  const uint64_t base = (hi << (lo + G)) | (mid << C);
  auto glob = [base, lo](int x) {
    return base | (uint64_t(x >> C) << lo) | uint64_t(x & ((1 << C) - 1));
  };
  V* p = reinterpret_cast<V*>(a);
  V buf[NV];
  if (stream) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = threadIdx.x + k * NT;
      buf[k] = ld16<true>(p + glob((e / VPR) << C | (e % VPR) * AP) / AP);
    }
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = threadIdx.x + k * NT;
      buf[k] = p[glob((e / VPR) << C | (e % VPR) * AP) / AP];
    }
  }
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int e = threadIdx.x + k * NT;
    const int x = ((e / VPR) << C) | (e % VPR) * AP;
    if constexpr (AP == 2) {
      sm[x] = {buf[k].x, buf[k].y};
      sm[x + 1] = {buf[k].z, buf[k].w};
    } else {
      sm[x] = {buf[k].x, buf[k].y};
    }
  }
  __syncthreads();
  tile_rounds<R, REV, false, NT, WMAX>(sm, TB, C, TB, lo, start, len, sign, glob);
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    const int e = threadIdx.x + k * NT;
    const int x = ((e / VPR) << C) | (e % VPR) * AP;
    const Cx<R> v0 = sm[x];
    if constexpr (AP == 2) {
      const Cx<R> v1 = sm[x + 1];
      buf[k] = {v0.r * scale, v0.i * scale, v1.r * scale, v1.i * scale};
    } else {
      buf[k] = {v0.r * scale, v0.i * scale};
    }
  }
  if (stream) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = threadIdx.x + k * NT;
      st16<true>(p + glob((e / VPR) << C | (e % VPR) * AP) / AP, buf[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = threadIdx.x + k * NT;
      p[glob((e / VPR) << C | (e % VPR) * AP) / AP] = buf[k];
    }
  }
}


// Tile shapes: the contiguous tile has 2^13 complex64 / 2^12 complex128
// entries (64 KiB plus padding); the strided tile 2^7 rows x 64 (complex64)
// or 32 (complex128) columns (64 KiB).
template <typename R> constexpr int lds_bits() { return sizeof(R) == 4 ? 13 : 12; }
template <typename R> constexpr int col_bits() { return sizeof(R) == 4 ? 6 : 5; }
constexpr int kColMax = 7;   // strided pass bits with 512-byte rows
constexpr int kColMax8 = 8;  // with 256-byte rows (knob qft.col_max)
constexpr int kRegMax = 5;

// Threads of a tile launch: at most `cap`, at most one per 16-byte vector of
// the tile, and at most the column count of the widest round, so that no
// thread idles in a round.
__host__ __device__ constexpr int tile_threads(int tile_bits, int vec_per_tile, int round_bits,
                                               int cap) {
  int nt = cap;
  if (nt > vec_per_tile) nt = vec_per_tile;
  if (nt > (1 << (tile_bits - round_bits))) nt = 1 << (tile_bits - round_bits);
  return nt < 1 ? 1 : nt;
}

template <typename K>
void allow_lds(K kernel, size_t bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

template <typename R, int G, bool REV>
hipError_t launch_reg(R* a, int n, int start, int len, int lo, int sign, R scale,
                      hipStream_t s) {
  const uint64_t threads = uint64_t(1) << (n - G);
  const uint64_t want = (threads + kBlock - 1) / kBlock, cap = uint64_t(1) << 20;
  const unsigned grid = static_cast<unsigned>(want < cap ? want : cap);
  hipLaunchKernelGGL((k_qft_reg<R, G, REV>), dim3(grid), dim3(kBlock), 0, s, a, n, start, len, lo,
                     sign, scale);
  return hipGetLastError();
}

// Streaming accesses (qft.stream: 0 when the state exceeds the last-level
// cache, 1 always, 2 never).
template <typename R>
int stream_policy(int n, const QftTuning& tune) {
  if (tune.stream == 1) return 1;
  if (tune.stream == 2) return 0;
  return (uint64_t(2 * sizeof(R)) << n) > (uint64_t(256) << 20) ? 1 : 0;
}

template <typename R, int G, int C, bool REV, int CAP, int WMAX>
hipError_t launch_col_cfg(R* a, int n, int start, int len, int lo, int sign, R scale,
                          int stream, hipStream_t s) {
  if (lo < C || n < lo + G) return hipErrorInvalidValue;
  constexpr int NT =
      tile_threads(G + C, (1 << (G + C)) / Vec16<R>::AMPS, round_width(G, WMAX), CAP);
  const size_t bytes = (size_t(1) << (G + C)) * 2 * sizeof(R);
  auto kern = k_qft_col<R, G, C, REV, NT, WMAX>;
  allow_lds(kern, bytes);
  const unsigned grid = static_cast<unsigned>(uint64_t(1) << (n - G - C));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), bytes, s, a, start, len, lo, sign, scale, stream);
  return hipGetLastError();
}

template <typename R, int T, bool REV, int CAP, int WMAX>
hipError_t launch_lds_cfg(R* a, int n, int start, int len, int lo, int hi, int sign, R scale,
                          int stream, hipStream_t s) {
  constexpr int VEC = (1 << T) / Vec16<R>::AMPS > 0 ? (1 << T) / Vec16<R>::AMPS : 1;
  constexpr int NT = tile_threads(T, VEC, round_width(T, WMAX), CAP);
  const size_t bytes = size_t((1 << T) + ((1 << T) >> 4)) * 2 * sizeof(R);
  auto kern = k_qft_lds<R, T, REV, NT, WMAX>;
  allow_lds(kern, bytes);
  const unsigned grid = static_cast<unsigned>(uint64_t(1) << (n - T));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(NT), bytes, s, a, start, len, lo, hi, sign, scale,
                     stream);
  return hipGetLastError();
}

// Launch configurations selectable by the tuning knobs: thread cap 256 or
// 512, round width 4 or 5 (tiles of at least 2^11 entries / 2^5 rows); smaller
// tiles always use cap 256 and rounds of 4.
template <typename R, int G, int C, bool REV>
hipError_t launch_col_c(R* a, int n, int start, int len, int lo, int sign, R scale,
                        const QftTuning& tune, hipStream_t s) {
  // thread cap: the knob, or (0) 512 for passes of 8 bits and 256 otherwise
  const int cap = tune.threads > 0 ? tune.threads : (G == 8 ? 512 : 256);
  const int st = stream_policy<R>(n, tune);
  if (G < 5 || (cap < 512 && tune.round_bits < 5))
    return launch_col_cfg<R, G, C, REV, 256, 4>(a, n, start, len, lo, sign, scale, st, s);
  if (cap >= 512 && tune.round_bits >= 5)
    return launch_col_cfg<R, G, C, REV, 512, 5>(a, n, start, len, lo, sign, scale, st, s);
  if (cap >= 512)
    return launch_col_cfg<R, G, C, REV, 512, 4>(a, n, start, len, lo, sign, scale, st, s);
  return launch_col_cfg<R, G, C, REV, 256, 5>(a, n, start, len, lo, sign, scale, st, s);
}

// Strided tiles of 2^G rows x 2^C columns: 512-byte rows (64 KiB at G = 7),
// or 256-byte rows for G = 8 (64 KiB) and, for complex128 or with
// qft.col_rows >= 1, for G = 7 (32 KiB, more workgroups per CU: a complex128
// 7-bit pass at 30 qubits 7.06 against 8.33 ms); qft.col_rows = 2 also gives
// complex64 passes of 8 bits 128-byte rows (32 KiB).
template <typename R, int G, bool REV>
hipError_t launch_col(R* a, int n, int start, int len, int lo, int sign, R scale,
                      const QftTuning& tune, hipStream_t s) {
  constexpr int CB = col_bits<R>();
  if constexpr (G == 8) {
    if constexpr (sizeof(R) == 4)
      if (tune.col_rows == 2)  // 128-byte rows, 32 KiB tiles
        return launch_col_c<R, G, CB - 2, REV>(a, n, start, len, lo, sign, scale, tune, s);
    return launch_col_c<R, G, CB - 1, REV>(a, n, start, len, lo, sign, scale, tune, s);
  }
  if constexpr (G == 7)
    if (sizeof(R) == 8 || tune.col_rows >= 1)
      return launch_col_c<R, G, CB - 1, REV>(a, n, start, len, lo, sign, scale, tune, s);
  return launch_col_c<R, G, CB, REV>(a, n, start, len, lo, sign, scale, tune, s);
}

template <typename R, int T, bool REV>
hipError_t launch_lds_t(R* a, int n, int start, int len, int lo, int hi, int sign, R scale,
                        const QftTuning& tune, hipStream_t s) {
  // complex128 stays at rounds of 4 bits: 32 double-precision amplitudes per
  // thread would leave one wave per SIMD
  const int cap = tune.threads > 0 ? tune.threads : 256;
  const int st = stream_policy<R>(n, tune);
  if (T < 11 || sizeof(R) == 8 || (cap < 512 && tune.round_bits < 5))
    return launch_lds_cfg<R, T, REV, 256, 4>(a, n, start, len, lo, hi, sign, scale, st, s);
  if (cap >= 512 && tune.round_bits >= 5)
    return launch_lds_cfg<R, T, REV, 512, 5>(a, n, start, len, lo, hi, sign, scale, st, s);
  if (cap >= 512)
    return launch_lds_cfg<R, T, REV, 512, 4>(a, n, start, len, lo, hi, sign, scale, st, s);
  return launch_lds_cfg<R, T, REV, 256, 5>(a, n, start, len, lo, hi, sign, scale, st, s);
}

template <typename R, bool REV>
hipError_t launch_lds(R* a, int n, int T, int start, int len, int lo, int hi, int sign, R scale,
                      const QftTuning& tune, hipStream_t s) {
  switch (T) {
#define QS_LDS_CASE(t) \
  case t: return launch_lds_t<R, t, REV>(a, n, start, len, lo, hi, sign, scale, tune, s);
    QS_LDS_CASE(1) QS_LDS_CASE(2) QS_LDS_CASE(3) QS_LDS_CASE(4) QS_LDS_CASE(5) QS_LDS_CASE(6)
    QS_LDS_CASE(7) QS_LDS_CASE(8) QS_LDS_CASE(9) QS_LDS_CASE(10) QS_LDS_CASE(11)
    QS_LDS_CASE(12)
#undef QS_LDS_CASE
    case 13:
      if constexpr (sizeof(R) == 4)
        return launch_lds_t<R, 13, REV>(a, n, start, len, lo, hi, sign, scale, tune, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <typename R, bool REV>
hipError_t launch_pass(R* a, int n, int start, int len, const QftPass& ps, int sign,
                       const QftTuning& tune, hipStream_t s) {
  const R scale = R(ps.scale);
  const int G = ps.hi - ps.lo;
  switch (ps.kind) {
    case QftPass::LDS:
      return launch_lds<R, REV>(a, n, ps.tile, start, len, ps.lo, ps.hi, sign, scale, tune, s);
    case QftPass::COL:
      switch (G) {
        case 1: return launch_col<R, 1, REV>(a, n, start, len, ps.lo, sign, scale, tune, s);
        case 2: return launch_col<R, 2, REV>(a, n, start, len, ps.lo, sign, scale, tune, s);
        case 3: return launch_col<R, 3, REV>(a, n, start, len, ps.lo, sign, scale, tune, s);
        case 4: return launch_col<R, 4, REV>(a, n, start, len, ps.lo, sign, scale, tune, s);
        case 5: return launch_col<R, 5, REV>(a, n, start, len, ps.lo, sign, scale, tune, s);
        case 6: return launch_col<R, 6, REV>(a, n, start, len, ps.lo, sign, scale, tune, s);
        case 7: return launch_col<R, 7, REV>(a, n, start, len, ps.lo, sign, scale, tune, s);
        case 8: return launch_col<R, 8, REV>(a, n, start, len, ps.lo, sign, scale, tune, s);
        default: return hipErrorInvalidValue;
      }
    case QftPass::REG:
      switch (G) {
        case 1: return launch_reg<R, 1, REV>(a, n, start, len, ps.lo, sign, scale, s);
        case 2: return launch_reg<R, 2, REV>(a, n, start, len, ps.lo, sign, scale, s);
        case 3: return launch_reg<R, 3, REV>(a, n, start, len, ps.lo, sign, scale, s);
        case 4: return launch_reg<R, 4, REV>(a, n, start, len, ps.lo, sign, scale, s);
        case 5: return launch_reg<R, 5, REV>(a, n, start, len, ps.lo, sign, scale, s);
        default: return hipErrorInvalidValue;
      }
  }
  return hipErrorInvalidValue;
}

}  // namespace

template <typename R>
hipError_t launch_qft_pass(R* a, int n, int start, int len, const QftPass& ps, int sign, bool rev,
                           const QftTuning& tune, hipStream_t s) {
  return rev ? launch_pass<R, true>(a, n, start, len, ps, sign, tune, s)
             : launch_pass<R, false>(a, n, start, len, ps, sign, tune, s);
}

template hipError_t launch_qft_pass<float>(float*, int, int, int, const QftPass&, int, bool,
                                           const QftTuning&, hipStream_t);
template hipError_t launch_qft_pass<double>(double*, int, int, int, const QftPass&, int, bool,
                                            const QftTuning&, hipStream_t);

// Pass plan of a QFT on [start, start+len): one contiguous-tile pass over the
// range bits below T, then passes of near-equal width (at most kColMax, or
// kRegMax for register passes) over the bits at or above T; top-down in
// natural order, bottom-up when bit-reversed. Each pass gets an exact
// power-of-two scale, the last one also 1/sqrt(2) if len is odd.
template <typename R>
int qft_plan(int n, int start, int len, bool rev, const QftTuning& tune, QftPass* out,
             int max_passes) {
  const bool use_reg = tune.high_kind == 1;
  const int wmax = use_reg ? kRegMax : (tune.col_max == 8 ? kColMax8 : kColMax);
  const int top = start + len;
  // passes of the plan with a contiguous tile of t bits
  auto pass_count = [&](int t) {
    int lo = start > t ? start : t;
    if (!use_reg && lo < col_bits<R>()) lo = col_bits<R>();
    return (top > lo ? (top - lo + wmax - 1) / wmax : 0) + (start < lo ? 1 : 0);
  };
  // contiguous tile bits: the knob, or (0) 12; complex64 states larger than
  // the last-level cache take 11 when that adds no pass (the 11-bit tile runs
  // more workgroups per CU: 6.2 against 5.8 TB/s at 27 qubits), complex128
  // ones always (the 12-bit complex128 tile, 64 KiB, ran at 4.0, the 11-bit
  // one at 5.0 TB/s at 29 qubits; a 26-qubit transform 1.18 instead of
  // 1.57 ms, a 29-qubit one 12.5 instead of 13.5)
  const bool big = (uint64_t(2 * sizeof(R)) << n) > (uint64_t(256) << 20);
  int T = tune.lds_bits > 0 ? tune.lds_bits : 12;
  if (T > lds_bits<R>()) T = lds_bits<R>();
  if (tune.lds_bits == 0 && big && (sizeof(R) == 8 || pass_count(11) <= pass_count(12))) T = 11;
  if (T > n) T = n;
  int reg_lo = start > T ? start : T;
  if (!use_reg && reg_lo < col_bits<R>()) reg_lo = col_bits<R>();
  int np = 0;
  if (top > reg_lo) {
    const int width = top - reg_lo;
    const int passes = (width + wmax - 1) / wmax;
    int cur = top;
    for (int k = 0; k < passes; ++k) {
      const int left = passes - k;
      const int w = (cur - reg_lo + left - 1) / left;
      if (np >= max_passes) return -1;
      out[np] = {use_reg ? QftPass::REG : QftPass::COL, cur - w, cur, 0, 1.0};
      ++np;
      cur -= w;
    }
  }
  if (start < reg_lo) {
    // the bits [start, reg_lo) lie in the contiguous tile [0, T')
    const int hi = top < reg_lo ? top : reg_lo;
    int Tt = hi > T ? hi : T;
    if (np >= max_passes) return -1;
    out[np] = {QftPass::LDS, start, hi, Tt, 1.0};
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

template int qft_plan<float>(int, int, int, bool, const QftTuning&, QftPass*, int);
template int qft_plan<double>(int, int, int, bool, const QftTuning&, QftPass*, int);

}  // namespace qs
