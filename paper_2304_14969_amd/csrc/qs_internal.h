// Internal declarations shared by the C-ABI layer and the HIP kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace qs {

// A 2x2 complex matrix in the state's precision, row-major.
template <typename R>
struct Mat2 {
  R re[4];
  R im[4];
};

// Up to 16 sorted bit positions at which zero bits are inserted into a
// compact counter to enumerate the index set of a gate.
struct BitSet16 {
  int n;
  int pos[16];
};

// ---------------------------------------------------------------- streaming accesses
// Whole-state sweeps read and write every byte once. For states larger than
// the 256 MiB last-level cache, non-temporal (streaming) loads and stores move
// 3-9% more bytes per second in sweeps whose waves touch contiguous runs of
// at least 64 bytes (30 qubits: a one-qubit gate on bit 0 6.36 against 5.91
// TB/s). With shorter runs (a gate bit below 64 bytes of amplitudes) the
// partial-line streaming writes cost more than they save (a controlled phase
// on bits 2 and 17: 2.13 against 1.63 ms), and smaller states keep plain
// accesses, since back-to-back sweeps then find part of the state in that
// cache (streaming made the QFT at 22-25 qubits 4-7% slower).
extern int g_sweep_stream;  // knob sweep.stream: 0 by size and run length, 1 always, 2 never
extern int g_shuffle_bits;  // knob gate.shuffle_bits: one-qubit gates on bits 1 .. this by shuffles
extern int g_dense_ctrl;    // knob gate.dense_ctrl: low-bit singly controlled gates swept densely
// n-qubit state of amp_bytes per amplitude, the lowest bit the sweep's
// indexing fixes at low_bit (runs of amp_bytes << low_bit contiguous bytes)
inline bool stream_sweep(int n, size_t amp_bytes, int low_bit) {
  if (g_sweep_stream == 1) return true;
  if (g_sweep_stream == 2) return false;
  return (uint64_t(amp_bytes) << n) > (uint64_t(256) << 20) &&
         (low_bit >= 6 || (uint64_t(amp_bytes) << low_bit) >= 64);
}

// Fused multiply-add, written out where a sweep's results must not depend on
// which products the compiler chooses to contract (so that its streaming
// and plain forms agree bit for bit).
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

typedef float qs_f32x2 __attribute__((ext_vector_type(2)));
typedef float qs_f32x4 __attribute__((ext_vector_type(4)));
typedef double qs_f64x2 __attribute__((ext_vector_type(2)));

// 16-byte loads and stores, non-temporal when NT
template <bool NT>
__device__ __forceinline__ float4 ld16(const float4* p) {
  if constexpr (NT) {
    const qs_f32x4 t = __builtin_nontemporal_load(reinterpret_cast<const qs_f32x4*>(p));
    return {t.x, t.y, t.z, t.w};
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ double2 ld16(const double2* p) {
  if constexpr (NT) {
    const qs_f64x2 t = __builtin_nontemporal_load(reinterpret_cast<const qs_f64x2*>(p));
    return {t.x, t.y};
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ void st16(float4* p, float4 v) {
  if constexpr (NT) {
    const qs_f32x4 t = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(t, reinterpret_cast<qs_f32x4*>(p));
  } else {
    *p = v;
  }
}
template <bool NT>
__device__ __forceinline__ void st16(double2* p, double2 v) {
  if constexpr (NT) {
    const qs_f64x2 t = {v.x, v.y};
    __builtin_nontemporal_store(t, reinterpret_cast<qs_f64x2*>(p));
  } else {
    *p = v;
  }
}
// one interleaved complex amplitude (8 or 16 bytes) at p = &re
template <bool NT>
__device__ __forceinline__ void ld_amp(const float* p, float* re, float* im) {
  if constexpr (NT) {
    const qs_f32x2 t = __builtin_nontemporal_load(reinterpret_cast<const qs_f32x2*>(p));
    *re = t.x;
    *im = t.y;
  } else {
    *re = p[0];
    *im = p[1];
  }
}
template <bool NT>
__device__ __forceinline__ void ld_amp(const double* p, double* re, double* im) {
  if constexpr (NT) {
    const qs_f64x2 t = __builtin_nontemporal_load(reinterpret_cast<const qs_f64x2*>(p));
    *re = t.x;
    *im = t.y;
  } else {
    *re = p[0];
    *im = p[1];
  }
}
template <bool NT>
__device__ __forceinline__ void st_amp(float* p, float re, float im) {
  if constexpr (NT) {
    const qs_f32x2 t = {re, im};
    __builtin_nontemporal_store(t, reinterpret_cast<qs_f32x2*>(p));
  } else {
    p[0] = re;
    p[1] = im;
  }
}
template <bool NT>
__device__ __forceinline__ void st_amp(double* p, double re, double im) {
  if constexpr (NT) {
    const qs_f64x2 t = {re, im};
    __builtin_nontemporal_store(t, reinterpret_cast<qs_f64x2*>(p));
  } else {
    p[0] = re;
    p[1] = im;
  }
}

// ---------------------------------------------------------------- gates
// Each launcher enqueues on `s` and returns the launch status.
template <typename R>
hipError_t launch_apply_1q(R* amps, int n, int t, const Mat2<R>& m, hipStream_t s);

// Controlled 2x2: `fixed` holds the sorted control and target bits,
// `set_mask` the control bits that must be 1, `tbit` the target bit.
template <typename R>
hipError_t launch_apply_ctrl(R* amps, int n, const BitSet16& fixed, uint64_t set_mask,
                             int tbit, const Mat2<R>& m, hipStream_t s);

// Multiply amplitudes with bits a and b set by (c, s).
template <typename R>
hipError_t launch_cphase(R* amps, int n, int a, int b, R cr, R ci, hipStream_t s);

// Physical exchange of bits a and b.
template <typename R>
hipError_t launch_bitswap(R* amps, int n, int a, int b, hipStream_t s);

// Dense k-qubit block; `mat` is a device array of 2^k x 2^k complex values
// (interleaved, row-major) in the state's precision, `qubits` the k bits.
template <typename R>
hipError_t launch_apply_fused(R* amps, int n, const int* qubits, int k, const R* mat,
                              hipStream_t s);
// The same for k <= 2 with the host matrix (FP64, interleaved, row-major)
// cast to R and passed in the kernel arguments: no device copy of it.
template <typename R>
hipError_t launch_apply_small(R* amps, int n, const int* qubits, int k, const double* host_mat,
                              hipStream_t s);

// Tile geometry of a k-qubit block on the matrix cores: the tile holds the
// contiguous low bits [0, C) and the block bits at or above C (qhi, h of
// them); tpos[j] is the tile bit of block row bit j; lowblk lists the block
// bits below C.
struct FusedGeom {
  int k, C, h, nlow;
  int qhi[6];
  int tpos[6];
  int lowblk[6];
  int swz;  // LDS entry of tile index x: x ^ ((x >> swz) & 15) (swz >= 16: x)
};
bool fused_geometry(int n, const int* qubits, int k, FusedGeom* g, int amp_bytes);

// block of k = 4 or 5 qubits on the matrix cores (v_mfma_f32_16x16x4f32 for
// complex64, v_mfma_f64_16x16x4f64 for complex128); returns
// hipErrorNotSupported when the state is too small for the tile.
hipError_t launch_fused_mfma(float* amps, int n, const int* qubits, int k, const float* mat,
                             hipStream_t s);
hipError_t launch_fused_mfma(double* amps, int n, const int* qubits, int k, const double* mat,
                             hipStream_t s);

// ---------------------------------------------------------------- batches
// One item of a batched launch: block (q, row bit order; sorted ascending) on
// the ket at amplitude offset amp_off of the arena; its tiles of 256 groups
// start at first_tile; its matrix at complex offset mat_off.
struct BatchItem {
  uint64_t amp_off;
  uint64_t first_tile;
  uint64_t mat_off;
  int n, k;
  int q[6];
  int sorted[6];
};
template <typename R>
hipError_t launch_batch_fused(R* arena, const BatchItem* items, int nitems, uint64_t tiles, int k,
                              const R* mats, hipStream_t s);
template <typename R>
hipError_t launch_batch_reset(R* arena, uint64_t total_amps, const uint64_t* offs, int count,
                              hipStream_t s);

// ---------------------------------------------------------------- factorized mode
// scratch: factor_scratch_doubles() doubles of device memory; inner products
// land in scratch[0..1] (Re, Im).
int factor_scratch_doubles();
template <typename R>
hipError_t launch_compose(R* c, const R* a, int na, const R* b, int nb, hipStream_t s);
// Bloch sums of the qubit at bit t (Re s, Im s, z0, z1) written to out[0..3],
// which may be host memory mapped into the device address space.
template <typename R>
hipError_t launch_bloch(const R* a, int nq, int t, double* scratch, double* out, hipStream_t s);
// Bloch sums of G = 2..5 qubits (local bits `bits`, ascending) in one sweep:
// out[4j .. 4j+3] for bits[j].
template <typename R>
hipError_t launch_bloch_multi(const R* a, int nq, const int* bits, int G, double* scratch,
                              double* out, hipStream_t s);
// Two-qubit rounding: the unnormalized 4x4 reduced density matrix of the
// qubits at bits t1 != t2 of a subsystem of nq >= 2 qubits, in float64, to
// out[16] (rho_00..rho_33, then Re/Im of rho_01, 02, 03, 12, 13, 23; index m
// = bit t1 + 2 bit t2); scratch as for launch_bloch.
// counter / flag / target / seq: the completion signal of launch_bloch_batch,
// only for subsystems of at most 2^15 amplitudes (one workgroup; counter =
// nullptr otherwise).
template <typename R>
hipError_t launch_pair_rho(const R* a, int nq, int t1, int t2, double* scratch, double* out,
                           unsigned* counter, unsigned* flag, unsigned target, unsigned seq,
                           hipStream_t s);
// b (nq - 2 qubits) = scale * <phi| a over bits t1, t2 (the two bits removed,
// the others in order), and pair (2 qubits) = phi; nq >= 3.
template <typename R>
hipError_t launch_decompose_pair(R* b, const R* a, int nq, int t1, int t2, const double phi[8],
                                 double scale, R* pair, hipStream_t s);
// The Bloch sums of several subsystems in one launch, one workgroup each:
// item i reads 2^nq amplitudes (nq <= kBlochBatchQubits) and writes, for each
// of its G (1..5) target bits (ascending, distinct, < nq), the four sums
// Re s, Im s, z0, z1 to out[item.out + 4j ..]. The item table may live in
// mapped host memory.
constexpr int kBlochBatchQubits = 15;
template <typename R>
struct BlochItem {
  const R* amps;
  int nq, G;
  int bits[5];
  int out;
  int op;  // launch_ops_bloch: the operation to run on amps first, or -1
};
// host_items: the same table in host memory; up to kBlochArgItems items travel
// in the kernel arguments instead of being read through `items`.
constexpr int kBlochArgItems = 64;
// counter (device) / flag (host-mapped): when counter is not null, the
// workgroup that completes the launch's count, target = the counter's value
// before the launch + nitems, stores seq into *flag after every sum is
// visible to the host (a completion signal that needs no stream
// synchronization).
template <typename R>
hipError_t launch_bloch_batch(const BlochItem<R>* host_items, const BlochItem<R>* items,
                              int nitems, double* out, unsigned* counter, unsigned* flag,
                              unsigned target, unsigned seq, hipStream_t s);
// Process-wide: small operation tables in the kernel arguments (1, default) or
// always read from mapped host memory (0).
extern int g_kernarg_tables;
// Independent operations on many small subsystems in one launch, one
// workgroup each (the large ones go through the single-operation launchers,
// whose arithmetic these repeat term for term):
//   kind 0, nb > 0: c = a (x) b (a's qubits at the low na bits), then the 4x4
//                   matrix m on local bits t0 (row bit 0) and t1 (row bit 1)
//   kind 0, nb = 0: the matrix on a in place (c == a)
//   kind 1:         c[u] = (conj(phi0) a[i0(u)] + conj(phi1) a[i1(u)]) scale,
//                   i0/i1 = u with 0/1 inserted at bit t0 (na qubits in a),
//                   and single = phi (the new one-qubit subsystem)
// Every operation reads and writes at most 2^kFactOpQubits amplitudes; no
// operation of a launch reads what another one writes.
constexpr int kFactOpQubits = 15;
template <typename R>
struct FactOp {
  const R* a;
  const R* b;
  R* c;
  R* single;
  int kind, na, nb, t0, t1, pad;
  double phi[4];
  double scale;
  R m[32];  // 4x4, row-major, interleaved
};
// Queued operations and the sweeps that read their results in one launch:
// workgroup i first runs ops[items[i].op] (when >= 0; its output is
// items[i].amps), then, after a barrier, the sweep of items[i], as
// launch_bloch_batch (same completion signal). Every operation belongs to
// exactly one item. Up to kFusedItems items and fused_arg_ops<R>() operations
// travel in the kernel arguments; larger tables are read through items/ops.
constexpr int kFusedItems = 16;
template <typename R>
constexpr int fused_arg_ops();
template <typename R>
hipError_t launch_ops_bloch(const BlochItem<R>* host_items, const BlochItem<R>* items, int nitems,
                            const FactOp<R>* host_ops, const FactOp<R>* ops, int nops,
                            double* out, unsigned* counter, unsigned* flag, unsigned target,
                            unsigned seq, hipStream_t s);
// Operations per launch that fit the kernel arguments (under 4 KiB).
template <typename R>
constexpr int fact_arg_ops() {
  return int(3584 / sizeof(FactOp<R>));
}
template <typename R>
constexpr int fused_arg_ops() {
  return int((3584 - kFusedItems * sizeof(BlochItem<R>)) / sizeof(FactOp<R>));
}
template <typename R>
hipError_t launch_fact_ops(const FactOp<R>* host_ops, const FactOp<R>* ops, int nops,
                           hipStream_t s);
// The kind-0 operation of FactOp over a grid, for any size: c = a (x) b (or a
// in place when nb = 0, c == a), then the 4x4 matrix m (interleaved,
// row-major, converted to R) on local bits t0, t1.
template <typename R>
hipError_t launch_merge_gate(R* c, const R* a, int na, const R* b, int nb, int t0, int t1,
                             const double m[32], hipStream_t s);
// One-qubit gates on many small subsystems in one launch: workgroup i applies
// the gates gates[items[i].g0 .. + ng) in order to subsystem items[i], held in
// LDS meanwhile. Every item has 1 <= nq <= max_nq <= kFact1qMaxQubits. Both
// tables may live in mapped host memory.
constexpr int kFact1qMaxQubits = 12;
template <typename R>
struct Fact1qItem {
  R* amps;
  int nq, g0, ng, pad;
};
template <typename R>
struct Fact1qGate {
  R m[8];  // 2x2 matrix, row-major, interleaved
  int t, pad;
};
// host_items / host_gates: the same tables in host memory; small ones travel
// in the kernel arguments (up to kFact1qArgItems items and
// fact1q_arg_gates<R>() gates, under 4 KiB).
constexpr int kFact1qArgItems = 32;
template <typename R>
constexpr int fact1q_arg_gates() {
  return int((3584 - kFact1qArgItems * sizeof(Fact1qItem<R>)) / sizeof(Fact1qGate<R>));
}
template <typename R>
hipError_t launch_fact_1q_batch(const Fact1qItem<R>* host_items, const Fact1qItem<R>* items,
                                int nitems, const Fact1qGate<R>* host_gates,
                                const Fact1qGate<R>* gates, int ngates, int max_nq,
                                hipStream_t s);
// A one-qubit subsystem: the two amplitudes amp = {Re a0, Im a0, Re a1, Im a1}.
template <typename R>
hipError_t launch_store_single(R* dst, const double amp[4], hipStream_t s);
// phi = {Re phi0, Im phi0, Re phi1, Im phi1}
template <typename R>
hipError_t launch_decompose(R* b, const R* a, int nq, int t, const double phi[4], double scale,
                            hipStream_t s);
template <typename R>
hipError_t launch_inner(const R* a, const R* b, uint64_t count, double* scratch, hipStream_t s);

// ---------------------------------------------------------------- tile passes
// Row bits of a tile (physical, ascending); the low bits [0, tile_low_bits)
// are always in the tile.
constexpr int kTileRowBits = 7;
struct TileRows {
  int b[kTileRowBits];
};
int tile_low_bits(int dtype);
extern int g_tile_low_c64;  // low tile bits of complex64 passes: 5 or 6
// One pass: `rounds` holds nrounds int4 {bits packed 8 per byte, first gate,
// gate count, 0}; `gates` int2 {kind | j1 << 4 | j2 << 8, matrix offset in R};
// mats the matrices (interleaved). Needs n >= tile_low_bits + kTileRowBits.
template <typename R>
hipError_t launch_tile_pass(R* a, int n, int low_bits, const TileRows& rows, const void* rounds,
                            int nrounds, const void* gates, const R* mats, hipStream_t s);
// Batched complex64 tile passes: one item = one pass of one ket of an arena
// of n >= kBatchTileLow + kTileRowBits qubits; items sorted by first_tile,
// the tiles of item i are [first_tile_i, first_tile_{i+1}); its rounds are
// rounds[r0 .. r0 + nr) (int4 as for launch_tile_mfma).
constexpr int kBatchTileLow = 5;
struct TileItem {
  uint64_t amp_off;     // amplitude offset of the ket in the arena
  uint64_t first_tile;  // first workgroup of the item
  TileRows rows;
  int r0, nr;
};
hipError_t launch_tile_mfma_batch(float* arena, const TileItem* items, int nitems, uint64_t tiles,
                                  const void* rounds, const float* amats, hipStream_t s);
// Floats of one dense round's matrix-core operands: for each of 4 K-steps the
// lane's entries of Re U, Im U and Re U + Im U (12 per lane, 64 lanes).
constexpr int kRoundOperands = 768;
// Complex64 pass with dense 4-qubit rounds on the matrix cores: `rounds`
// int4 {bits packed 8 per byte, offset of the round's operands in amats
// (kRoundOperands floats, lane order), 0, 0}.
hipError_t launch_tile_mfma(float* a, int n, int low_bits, const TileRows& rows,
                            const void* rounds, int nrounds, const float* amats, hipStream_t s);

// ---------------------------------------------------------------- QFT passes
// One pass of a QFT on the qubit range [start, start+len): the stages of the
// bits [lo, hi), each a butterfly on its bit and the phase controlled by the
// other range bits, then a multiplication by `scale`.
//   LDS: contiguous tile of 2^tile amplitudes (bits [0, tile)), hi <= tile.
//   COL: tile of 2^(hi-lo) strided rows x contiguous columns.
//   REG: each thread holds the 2^(hi-lo) amplitudes of its group.
struct QftPass {
  enum Kind { LDS = 0, COL = 1, REG = 2 };
  int kind;
  int lo, hi;
  int tile;
  double scale;
};

// Process-wide tuning knobs of the pass planner.
struct QftTuning {
  int lds_bits = 0;   // contiguous tile bits (0: by size, 12 or 11; at most 13 / 12)
  int high_kind = 0;  // passes above the tile: 0 strided LDS tiles, 1 registers
  int threads = 0;    // thread cap of the LDS tile launches: 256, 512, or 0 = by pass width
  int round_bits = 4; // widest register round inside an LDS tile (4 or 5)
  int col_max = 8;    // most bits of a strided LDS pass: 7 (512-byte rows) or 8 (256-byte)
  int col_rows = 0;   // 1: 7-bit strided passes with 256-byte rows (32 KiB tiles);
                      // 2: also 8-bit ones with 128-byte rows (complex64)
  int stream = 0;     // streaming (non-temporal) accesses of the LDS tile passes:
                      // 0 when the state exceeds the last-level cache, 1 always, 2 never
};

// `rev` = the range is stored bit-reversed (after an earlier transform's
// relabelling); `sign` = +1 forward, -1 conjugated (inverse transform).
template <typename R>
hipError_t launch_qft_pass(R* amps, int n, int start, int len, const QftPass& pass, int sign,
                           bool rev, const QftTuning& tune, hipStream_t s);

// Pass plan in launch order; returns the number of passes (-1 if more than
// max_passes).
template <typename R>
int qft_plan(int n, int start, int len, bool rev, const QftTuning& tune, QftPass* out,
             int max_passes);

// ---------------------------------------------------------------- state setup
template <typename R>
hipError_t launch_set_basis(R* amps, int n, uint64_t x, hipStream_t s);

// dst (state precision) <- src (Rs precision), count complex values.
template <typename Rd, typename Rs>
hipError_t launch_convert(Rd* dst, const Rs* src, uint64_t count, hipStream_t s);

// ---------------------------------------------------------------- reductions
// Squared norm in float64: partial sums per block into `partial` (nblocks
// doubles, see reduce_blocks), then a fixed-order final sum into out[0].
int reduce_blocks(uint64_t count);
template <typename R>
hipError_t launch_norm(const R* amps, uint64_t count, double* partial, double* out,
                       hipStream_t s);

// probs[x] = |a_x|^2 for x in [0, count)
template <typename R>
hipError_t launch_probs(const R* amps, uint64_t count, double* probs, hipStream_t s);

// out[j] = a[phys(idx[j])] as complex double, phys maps logical to physical bits
struct Perm64 {
  int n;
  int8_t p[64];
};
template <typename R>
hipError_t launch_gather(const R* amps, const uint64_t* idx, uint64_t m, Perm64 perm,
                         double* out, hipStream_t s);
// out[j] *= a[local index of idx[j]], bit t of the local index = bit bits.p[t]
// of idx[j]
template <typename R>
hipError_t launch_gather_mul(const R* a, const uint64_t* idx, uint64_t m, Perm64 bits,
                             double* out, hipStream_t s);

}  // namespace qs
