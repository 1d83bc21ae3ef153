// C ABI of the simulator: argument checks, state handles, the qubit relabel
// map and dispatch to the HIP kernels. No simulation arithmetic happens here
// beyond building small gate matrices and twiddle tables on the host in
// float64 and rounding them once to the state's precision.
#include <algorithm>
#include <atomic>
#include <mutex>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/qs.h"
#include "circuit.h"
#include "factor.h"
#include "qs_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

// ------------------------------------------------------------------ allocator
qs_alloc_fn g_alloc = nullptr;
qs_free_fn g_free = nullptr;
void* g_user = nullptr;
int g_live_states = 0;
qs::QftTuning g_qft_tune;
int g_fused_mfma = 1;  // blocks of 4-5 qubits on the matrix cores (FP32 / FP64)
int g_tile_mfma = 1;   // complex64 tile passes with dense rounds on the matrix cores

void* dev_alloc(size_t bytes) {
  if (g_alloc) return g_alloc(bytes, g_user);
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(void* p) {
  if (!p) return;
  if (g_free) {
    g_free(p, g_user);
  } else {
    (void)hipFree(p);
  }
}

constexpr size_t kMatBytes = size_t(2) * (1u << 6) * (1u << 6) * sizeof(double);
constexpr uint64_t kStageAmps = uint64_t(1) << 22;  // staging chunk for host transfers

}  // namespace

// Per-launch timing: while enabled, every kernel launch of a state is
// bracketed by two HIP events on the state's stream and tagged with its name
// and algorithmic bytes.
struct ProfRec {
  const char* name;
  double bytes;
  hipEvent_t a, b;
};

struct qs_state {
  int n = 0;
  int dtype = QS_C64;
  void* amps = nullptr;
  hipStream_t stream = nullptr;
  int perm[64];          // logical qubit -> physical bit
  bool poisoned = false;
  const char* poison_why = nullptr;  // set when not a device error poisoned it
  void* mat = nullptr;   // device slot for gate matrices
  double* red = nullptr; // reduction scratch: partials + result
  bool prof = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  qs::FactorState* fact = nullptr;  // set for factorized (approximate-mode) states
};

// Staging of qs_amplitudes_gather_noalloc: the index list (uint64) followed
// by the outputs (complex float64) of at most QS_GATHER_NOALLOC_MAX entries.
// Each GPU holds its own copy for the life of the process. In host code the
// array's name is not a device address: kernels and copies get the address
// that hipGetSymbolAddress returns for the device (noalloc_scratch).
constexpr uint64_t kNoAllocMax = QS_GATHER_NOALLOC_MAX;
constexpr size_t kNoAllocIdxBytes = kNoAllocMax * sizeof(uint64_t);
static __device__ __align__(256) unsigned char scratch[kNoAllocIdxBytes + kNoAllocMax * 2 * sizeof(double)];

namespace {

uint64_t dim(const qs_state* st) { return uint64_t(1) << st->n; }
// reduction scratch of every state: norm partials or Bloch/inner partials
size_t scratch_doubles() {
  const size_t a = size_t(qs::reduce_blocks(0)) + 1, b = size_t(qs::factor_scratch_doubles());
  return a > b ? a : b;
}
size_t amp_bytes(int dtype) { return dtype == QS_C64 ? 8 : 16; }
double ab(const qs_state* st) { return double(amp_bytes(st->dtype)); }

int check_state(const qs_state* st) {
  if (!st) return fail(QS_E_INVAL, "state is NULL");
  if (st->poisoned)
    return fail(QS_E_DEVICE, "state is unusable after an earlier %s",
                st->poison_why ? st->poison_why : "device error");
  return QS_OK;
}

int device_error(qs_state* st, hipError_t e, const char* what) {
  if (e == hipSuccess) return QS_OK;
  if (st) st->poisoned = true;
  return fail(QS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Device address of `scratch` on the GPU that holds the state's amplitudes,
// looked up once per device with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int noalloc_scratch(qs_state* st, void** out) {
  hipPointerAttribute_t attr{};
  hipError_t e = hipPointerGetAttributes(&attr, st->amps);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(QS_E_DEVICE, "locating the state's device: %s", hipGetErrorString(e));
  }
  const int dev = attr.device;
  if (dev < 0 || dev >= kMaxDevices) return fail(QS_E_DEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(QS_E_DEVICE, "address of the no-allocation staging array: %s",
                  hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return QS_OK;
}

int check_qubit(const qs_state* st, int q, const char* name) {
  if (q < 0 || q >= st->n)
    return fail(QS_E_INVAL, "%s %d out of range [0, %d)", name, q, st->n);
  return QS_OK;
}

int check_finite(const double* v, size_t count) {
  if (!v) return fail(QS_E_INVAL, "matrix pointer is NULL");
  for (size_t i = 0; i < count; ++i)
    if (!std::isfinite(v[i])) return fail(QS_E_INVAL, "matrix entry %zu is not finite", i);
  return QS_OK;
}

template <typename R>
qs::Mat2<R> to_mat2(const double m[8]) {
  qs::Mat2<R> out;
  for (int e = 0; e < 4; ++e) {
    out.re[e] = static_cast<R>(m[2 * e]);
    out.im[e] = static_cast<R>(m[2 * e + 1]);
  }
  return out;
}

hipEvent_t pool_event(qs_state* st) {
  if (!st->pool.empty()) {
    hipEvent_t e = st->pool.back();
    st->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch when profiling is on.
struct ProfScope {
  qs_state* st;
  bool on;
  ProfScope(qs_state* s, const char* name, double bytes) : st(s), on(s->prof) {
    if (!on) return;
    ProfRec r{name, bytes, pool_event(st), pool_event(st)};
    if (!r.a || !r.b) {
      on = false;
      return;
    }
    (void)hipEventRecord(r.a, st->stream);
    st->recs.push_back(r);
  }
  ~ProfScope() {
    if (on) (void)hipEventRecord(st->recs.back().b, st->stream);
  }
};

// Dense block on physical bits phys[0..k) with a device matrix in the state's
// precision: blocks of 4 or 5 qubits go to the matrix cores (FP32 for
// complex64, FP64 for complex128) when the state holds a full tile,
// everything else to the vector-FMA kernel.
hipError_t launch_block(qs_state* st, const int* phys, int k, const void* dmat) {
  static const char* names[] = {"", "fused1", "fused2", "fused3", "fused4", "fused5", "fused6"};
  static const char* mnames[] = {"", "", "", "", "fused4_mfma", "fused5_mfma", ""};
  const double bytes = 2.0 * std::ldexp(1.0, st->n) * ab(st);
  qs::FusedGeom geom;
  const bool mfma = g_fused_mfma && (k == 4 || k == 5) &&
                    qs::fused_geometry(st->n, phys, k, &geom, int(ab(st)));
  if (st->dtype == QS_C64) {
    if (mfma) {
      ProfScope ps(st, mnames[k], bytes);
      return qs::launch_fused_mfma(static_cast<float*>(st->amps), st->n, phys, k,
                                   static_cast<const float*>(dmat), st->stream);
    }
    ProfScope ps(st, names[k], bytes);
    return qs::launch_apply_fused(static_cast<float*>(st->amps), st->n, phys, k,
                                  static_cast<const float*>(dmat), st->stream);
  }
  if (mfma) {
    ProfScope ps(st, mnames[k], bytes);
    return qs::launch_fused_mfma(static_cast<double*>(st->amps), st->n, phys, k,
                                 static_cast<const double*>(dmat), st->stream);
  }
  ProfScope ps(st, names[k], bytes);
  return qs::launch_apply_fused(static_cast<double*>(st->amps), st->n, phys, k,
                                static_cast<const double*>(dmat), st->stream);
}

// Physical exchange of bits pa and pb.
int phys_swap(qs_state* st, int pa, int pb) {
  ProfScope ps(st, "bitswap", 2.0 * std::ldexp(1.0, st->n - 1) * ab(st));
  hipError_t e;
  if (st->dtype == QS_C64)
    e = qs::launch_bitswap(static_cast<float*>(st->amps), st->n, pa, pb, st->stream);
  else
    e = qs::launch_bitswap(static_cast<double*>(st->amps), st->n, pa, pb, st->stream);
  return device_error(st, e, "bit swap");
}

// Move amplitudes so that logical qubit q sits at physical bit q again.
int materialize(qs_state* st) {
  for (int q = 0; q < st->n; ++q) {
    if (st->perm[q] == q) continue;
    int q2 = -1;  // logical qubit currently at physical bit q
    for (int k = 0; k < st->n; ++k)
      if (st->perm[k] == q) q2 = k;
    const int p = st->perm[q];
    int rc = phys_swap(st, p, q);
    if (rc) return rc;
    st->perm[q] = q;
    st->perm[q2] = p;
  }
  return QS_OK;
}

void reset_perm(qs_state* st) {
  for (int q = 0; q < 64; ++q) st->perm[q] = q;
}

int sync(qs_state* st, const char* what) {
  return device_error(st, hipStreamSynchronize(st->stream), what);
}

// Status of a factorized-mode call; a device error poisons the state.
int fact_rc(qs_state* st, int rc) {
  if (rc == QS_E_DEVICE) st->poisoned = true;
  return rc;
}

}  // namespace

namespace qs {

void set_last_error(const char* msg) { g_err = msg; }
void* device_alloc(size_t bytes) { return dev_alloc(bytes); }
void device_free(void* p) { dev_free(p); }

// Drops a circuit's plan and its device copies (after an edit or a re-plan).
// Process-wide generation numbers: a circuit gets a fresh one when created
// and whenever its gate list changes, so (address, generation) identifies
// one gate list even when a freed circuit's address is reused.
uint64_t next_generation() {
  static std::atomic<uint64_t> gen{0};
  return ++gen;
}

void circuit_invalidate(qs_circuit* c) {
  // launches already queued may still read the matrices
  if (c->dmat[0] || c->dmat[1] || c->tcache[0].dev || c->tcache[1].dev) (void)hipDeviceSynchronize();
  for (int p = 0; p < 2; ++p) {
    if (c->dmat[p]) dev_free(c->dmat[p]);
    c->dmat[p] = nullptr;
    c->off[p].clear();
    if (c->tcache[p].dev) dev_free(c->tcache[p].dev);
    c->tcache[p].dev = nullptr;
    c->tcache[p].key.clear();
    c->tcache[p].plan = qs::TilePlan();
  }
  c->planned = false;
  c->blocks.clear();
  c->bplan_ok = false;
  c->bplan = qs::TilePlan();
  c->generation = next_generation();
}

}  // namespace qs

namespace {


}  // namespace

extern "C" {

const char* qs_last_error(void) { return g_err.c_str(); }

int qs_version(void) { return 100; }

int qs_tune_set(const char* key, int64_t value) {
  if (!key) return fail(QS_E_INVAL, "key is NULL");
  if (!std::strcmp(key, "qft.lds_bits")) {
    if (value < 0 || value > 13) return fail(QS_E_INVAL, "qft.lds_bits %lld outside [0, 13]", (long long)value);
    g_qft_tune.lds_bits = int(value);
  } else if (!std::strcmp(key, "qft.high_pass")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "qft.high_pass must be 0 or 1");
    g_qft_tune.high_kind = int(value);
  } else if (!std::strcmp(key, "fused.mfma")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "fused.mfma must be 0 or 1");
    g_fused_mfma = int(value);
  } else if (!std::strcmp(key, "qft.threads")) {
    if (value != 0 && value != 256 && value != 512)
      return fail(QS_E_INVAL, "qft.threads must be 0 (by pass width), 256 or 512");
    g_qft_tune.threads = int(value);
  } else if (!std::strcmp(key, "qft.round_bits")) {
    if (value != 4 && value != 5) return fail(QS_E_INVAL, "qft.round_bits must be 4 or 5");
    g_qft_tune.round_bits = int(value);
  } else if (!std::strcmp(key, "qft.col_rows")) {
    if (value < 0 || value > 2) return fail(QS_E_INVAL, "qft.col_rows must be 0, 1 or 2");
    g_qft_tune.col_rows = int(value);
  } else if (!std::strcmp(key, "gate.dense_ctrl")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "gate.dense_ctrl must be 0 or 1");
    qs::g_dense_ctrl = int(value);
  } else if (!std::strcmp(key, "gate.shuffle_bits")) {
    if (value < 0 || value > 6) return fail(QS_E_INVAL, "gate.shuffle_bits must be in [0, 6]");
    qs::g_shuffle_bits = int(value);
  } else if (!std::strcmp(key, "sweep.stream")) {
    if (value < 0 || value > 2) return fail(QS_E_INVAL, "sweep.stream must be 0, 1 or 2");
    qs::g_sweep_stream = int(value);
  } else if (!std::strcmp(key, "qft.stream")) {
    if (value < 0 || value > 2) return fail(QS_E_INVAL, "qft.stream must be 0, 1 or 2");
    g_qft_tune.stream = int(value);
  } else if (!std::strcmp(key, "qft.col_max")) {
    if (value != 7 && value != 8) return fail(QS_E_INVAL, "qft.col_max must be 7 or 8");
    g_qft_tune.col_max = int(value);
  } else if (!std::strcmp(key, "tile.low_bits")) {
    if (value < 4 || value > 6) return fail(QS_E_INVAL, "tile.low_bits must be 4, 5 or 6");
    qs::g_tile_low_c64 = int(value);
  } else if (!std::strcmp(key, "tile.mfma")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "tile.mfma must be 0 or 1");
    g_tile_mfma = int(value);
  } else if (!std::strcmp(key, "factor.tile_1q")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.tile_1q must be 0 or 1");
    qs::g_tile_1q = int(value);
  } else if (!std::strcmp(key, "factor.fuse_ops")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.fuse_ops must be 0 or 1");
    qs::g_fuse_ops = int(value);
  } else if (!std::strcmp(key, "factor.hold")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.hold must be 0 or 1");
    qs::g_hold = int(value);
  } else if (!std::strcmp(key, "factor.kickback")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.kickback must be 0 or 1");
    qs::g_kickback = int(value);
  } else if (!std::strcmp(key, "factor.done_flag")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.done_flag must be 0 or 1");
    qs::g_done_flag = int(value);
  } else if (!std::strcmp(key, "factor.kernarg_tables")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.kernarg_tables must be 0 or 1");
    qs::g_kernarg_tables = int(value);
  } else if (!std::strcmp(key, "factor.unobservable")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.unobservable must be 0 or 1");
    qs::g_unobservable = int(value);
  } else if (!std::strcmp(key, "factor.defer")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.defer must be 0 or 1");
    qs::g_defer_sep = int(value);
  } else if (!std::strcmp(key, "factor.batch_1q")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.batch_1q must be 0 or 1");
    qs::g_batch_1q = int(value);
  } else if (!std::strcmp(key, "factor.multi_test")) {
    if (value < 0 || value > 1) return fail(QS_E_INVAL, "factor.multi_test must be 0 or 1");
    qs::g_multi_test = int(value);

  } else {
    return fail(QS_E_INVAL, "unknown tuning key '%s'", key);
  }
  return QS_OK;
}

int qs_tune_get(const char* key, int64_t* value) {
  if (!key || !value) return fail(QS_E_INVAL, "NULL argument");
  if (!std::strcmp(key, "qft.lds_bits")) *value = g_qft_tune.lds_bits;
  else if (!std::strcmp(key, "qft.high_pass")) *value = g_qft_tune.high_kind;
  else if (!std::strcmp(key, "qft.threads")) *value = g_qft_tune.threads;
  else if (!std::strcmp(key, "fused.mfma")) *value = g_fused_mfma;
  else if (!std::strcmp(key, "qft.round_bits")) *value = g_qft_tune.round_bits;
  else if (!std::strcmp(key, "factor.multi_test")) *value = qs::g_multi_test;
  else if (!std::strcmp(key, "factor.batch_1q")) *value = qs::g_batch_1q;
  else if (!std::strcmp(key, "factor.defer")) *value = qs::g_defer_sep;
  else if (!std::strcmp(key, "factor.unobservable")) *value = qs::g_unobservable;
  else if (!std::strcmp(key, "factor.kernarg_tables")) *value = qs::g_kernarg_tables;
  else if (!std::strcmp(key, "factor.done_flag")) *value = qs::g_done_flag;
  else if (!std::strcmp(key, "factor.fuse_ops")) *value = qs::g_fuse_ops;
  else if (!std::strcmp(key, "factor.hold")) *value = qs::g_hold;
  else if (!std::strcmp(key, "factor.kickback")) *value = qs::g_kickback;
  else if (!std::strcmp(key, "factor.tile_1q")) *value = qs::g_tile_1q;
  else if (!std::strcmp(key, "tile.mfma")) *value = g_tile_mfma;
  else if (!std::strcmp(key, "qft.col_max")) *value = g_qft_tune.col_max;
  else if (!std::strcmp(key, "qft.col_rows")) *value = g_qft_tune.col_rows;
  else if (!std::strcmp(key, "qft.stream")) *value = g_qft_tune.stream;
  else if (!std::strcmp(key, "sweep.stream")) *value = qs::g_sweep_stream;
  else if (!std::strcmp(key, "gate.shuffle_bits")) *value = qs::g_shuffle_bits;
  else if (!std::strcmp(key, "gate.dense_ctrl")) *value = qs::g_dense_ctrl;
  else if (!std::strcmp(key, "tile.low_bits")) *value = qs::g_tile_low_c64;
  else return fail(QS_E_INVAL, "unknown tuning key '%s'", key);
  return QS_OK;
}

int qs_set_allocator(qs_alloc_fn alloc_fn, qs_free_fn free_fn, void* user) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr))
    return fail(QS_E_INVAL, "allocator and free function must both be set or both be NULL");
  if (g_live_states) return fail(QS_E_INVAL, "allocator cannot change while states are alive");
  g_alloc = alloc_fn;
  g_free = free_fn;
  g_user = user;
  return QS_OK;
}

int qs_alloc(int n, int dtype, qs_state** out) {
  if (!out) return fail(QS_E_INVAL, "out is NULL");
  if (n < 1 || n > QS_MAX_QUBITS) return fail(QS_E_INVAL, "n = %d outside [1, %d]", n, QS_MAX_QUBITS);
  if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", dtype);
  qs_state* st = new qs_state();
  st->n = n;
  st->dtype = dtype;
  reset_perm(st);
  const size_t bytes = size_t(1) << n;
  st->amps = dev_alloc(bytes * amp_bytes(dtype));
  st->mat = dev_alloc(kMatBytes);
  st->red = static_cast<double*>(dev_alloc(sizeof(double) * scratch_doubles()));
  if (!st->amps || !st->mat || !st->red) {
    dev_free(st->amps);
    dev_free(st->mat);
    dev_free(st->red);
    delete st;
    return fail(QS_E_NOMEM, "device allocation of %zu bytes failed", bytes * amp_bytes(dtype));
  }
  ++g_live_states;
  hipError_t e = dtype == QS_C64
                     ? qs::launch_set_basis(static_cast<float*>(st->amps), n, 0, st->stream)
                     : qs::launch_set_basis(static_cast<double*>(st->amps), n, 0, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  if (e != hipSuccess) {
    dev_free(st->amps);
    dev_free(st->mat);
    dev_free(st->red);
    delete st;
    --g_live_states;
    return fail(QS_E_DEVICE, "initialising the state: %s", hipGetErrorString(e));
  }
  *out = st;
  return QS_OK;
}

int qs_alloc_factorized(int n, int dtype, uint64_t max_amps, qs_state** out) {
  if (!out) return fail(QS_E_INVAL, "out is NULL");
  if (n < 1 || n > 63) return fail(QS_E_INVAL, "n = %d outside [1, 63]", n);
  if (dtype != QS_C64 && dtype != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", dtype);
  if (max_amps < 2) return fail(QS_E_INVAL, "max_amps must be at least 2");
  qs_state* st = new qs_state();
  st->n = n;
  st->dtype = dtype;
  reset_perm(st);
  st->mat = dev_alloc(kMatBytes);
  st->red = static_cast<double*>(dev_alloc(sizeof(double) * scratch_doubles()));
  double* hstat = nullptr;
  double* dstat = nullptr;
  if (!st->mat || !st->red ||
      hipHostMalloc(reinterpret_cast<void**>(&hstat),
                    qs::FactorState::kStatDoubles * sizeof(double), hipHostMallocMapped) !=
          hipSuccess ||
      hipHostGetDevicePointer(reinterpret_cast<void**>(&dstat), hstat, 0) != hipSuccess) {
    if (hstat) (void)hipHostFree(hstat);
    dev_free(st->mat);
    dev_free(st->red);
    delete st;
    return fail(QS_E_NOMEM, "device allocation failed");
  }
  st->fact = new qs::FactorState();
  st->fact->hstat = hstat;
  st->fact->dstat = dstat;
  st->fact->n = n;
  st->fact->dtype = dtype;
  st->fact->max_amps = max_amps;
  st->fact->tau = dtype == QS_C64 ? 1e-6 : 1e-12;
  st->fact->scratch = st->red;
  st->fact->mat = st->mat;
  ++g_live_states;
  if (int rc = qs::fact_init(st->fact)) {
    qs::fact_drain(st->fact);
    dev_free(st->mat);
    dev_free(st->red);
    (void)hipHostFree(hstat);
    delete st->fact;
    delete st;
    --g_live_states;
    return rc;
  }
  *out = st;
  return QS_OK;
}

int qs_free(qs_state* st) {
  if (!st) return QS_OK;
  (void)hipStreamSynchronize(st->stream);
  if (st->fact) {
    qs::fact_drain(st->fact);
    (void)hipHostFree(st->fact->hstat);
    delete st->fact;
  }
  dev_free(st->amps);
  dev_free(st->mat);
  dev_free(st->red);
  for (auto& r : st->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : st->pool) (void)hipEventDestroy(e);
  delete st;
  --g_live_states;
  return QS_OK;
}

int qs_set_stream(qs_state* st, void* hip_stream) {
  if (int rc = check_state(st)) return rc;
  st->stream = static_cast<hipStream_t>(hip_stream);
  if (st->fact) st->fact->stream = st->stream;
  return QS_OK;
}

int qs_synchronize(qs_state* st) {
  if (int rc = check_state(st)) return rc;
  return sync(st, "synchronize");
}

int qs_info(const qs_state* st, int* n, int* dtype) {
  if (!st) return fail(QS_E_INVAL, "state is NULL");
  if (n) *n = st->n;
  if (dtype) *dtype = st->dtype;
  return QS_OK;
}

int qs_set_basis(qs_state* st, uint64_t x) {
  if (int rc = check_state(st)) return rc;
  if (x >= dim(st)) return fail(QS_E_INVAL, "basis index %llu >= 2^%d", (unsigned long long)x, st->n);
  if (st->fact) return qs::fact_set_basis(st->fact, x);
  reset_perm(st);
  hipError_t e = st->dtype == QS_C64
                     ? qs::launch_set_basis(static_cast<float*>(st->amps), st->n, x, st->stream)
                     : qs::launch_set_basis(static_cast<double*>(st->amps), st->n, x, st->stream);
  return device_error(st, e, "set basis");
}

int qs_set_amplitudes(qs_state* st, const void* host, uint64_t count, int host_dtype) {
  if (int rc = check_state(st)) return rc;
  if (!host) return fail(QS_E_INVAL, "host pointer is NULL");
  if (count != dim(st)) return fail(QS_E_INVAL, "count %llu != 2^%d", (unsigned long long)count, st->n);
  if (host_dtype != QS_C64 && host_dtype != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", host_dtype);
  if (st->fact) return fail(QS_E_UNSUPPORTED, "a factorized state cannot take a dense vector");
  reset_perm(st);
  const size_t hb = amp_bytes(host_dtype), sb = amp_bytes(st->dtype);
  if (host_dtype == st->dtype) {
    hipError_t e = hipMemcpyAsync(st->amps, host, count * hb, hipMemcpyHostToDevice, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    return device_error(st, e, "upload");
  }
  const uint64_t chunk = count < kStageAmps ? count : kStageAmps;
  void* stage = dev_alloc(chunk * hb);
  if (!stage) return fail(QS_E_NOMEM, "staging allocation failed");
  hipError_t e = hipSuccess;
  for (uint64_t off = 0; off < count && e == hipSuccess; off += chunk) {
    const uint64_t c = count - off < chunk ? count - off : chunk;
    e = hipMemcpyAsync(stage, static_cast<const char*>(host) + off * hb, c * hb,
                       hipMemcpyHostToDevice, st->stream);
    if (e != hipSuccess) break;
    char* dst = static_cast<char*>(st->amps) + off * sb;
    if (st->dtype == QS_C64)
      e = qs::launch_convert(reinterpret_cast<float*>(dst), static_cast<const double*>(stage), c, st->stream);
    else
      e = qs::launch_convert(reinterpret_cast<double*>(dst), static_cast<const float*>(stage), c, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  }
  dev_free(stage);
  return device_error(st, e, "upload");
}

// ------------------------------------------------------------------ gates

int qs_apply_1q(qs_state* st, int q, const double m[8]) {
  if (int rc = check_state(st)) return rc;
  if (int rc = check_qubit(st, q, "qubit")) return rc;
  if (int rc = check_finite(m, 8)) return rc;
  if (st->fact) return fact_rc(st, qs::fact_apply(st->fact, &q, 1, m));
  const int t = st->perm[q];
  ProfScope ps(st, "apply_1q", 2.0 * std::ldexp(1.0, st->n) * ab(st));
  hipError_t e;
  if (st->dtype == QS_C64)
    e = qs::launch_apply_1q(static_cast<float*>(st->amps), st->n, t, to_mat2<float>(m), st->stream);
  else
    e = qs::launch_apply_1q(static_cast<double*>(st->amps), st->n, t, to_mat2<double>(m), st->stream);
  return device_error(st, e, "apply_1q");
}

int qs_apply_ctrl(qs_state* st, const int* ctrls, int nctrl, uint64_t ctrl_values, int target,
                  const double m[8]) {
  if (int rc = check_state(st)) return rc;
  if (!ctrls && nctrl > 0) return fail(QS_E_INVAL, "ctrls is NULL");
  if (nctrl < 1 || nctrl > 8) return fail(QS_E_INVAL, "nctrl = %d outside [1, 8]", nctrl);
  if (int rc = check_qubit(st, target, "target")) return rc;
  if (int rc = check_finite(m, 8)) return rc;
  if (nctrl + 1 > st->n) return fail(QS_E_INVAL, "too many qubits for n = %d", st->n);
  qs::BitSet16 fixed{};
  uint64_t set_mask = 0, seen = uint64_t(1) << target;
  for (int j = 0; j < nctrl; ++j) {
    if (int rc = check_qubit(st, ctrls[j], "control")) return rc;
    if (seen & (uint64_t(1) << ctrls[j])) return fail(QS_E_INVAL, "qubit %d used twice", ctrls[j]);
    seen |= uint64_t(1) << ctrls[j];
    const int p = st->perm[ctrls[j]];
    fixed.pos[fixed.n++] = p;
    if ((ctrl_values >> j) & 1) set_mask |= uint64_t(1) << p;
  }
  if (st->fact) {
    // controlled matrix on (ctrls..., target): m where the controls match
    if (nctrl + 1 > QS_MAX_FUSED) return fail(QS_E_UNSUPPORTED, "factorized gates act on <= %d qubits", QS_MAX_FUSED);
    const int k = nctrl + 1, D = 1 << k;
    std::vector<double> full(size_t(2) * D * D, 0.0);
    for (int i = 0; i < D; ++i) full[2 * (size_t(i) * D + i)] = 1.0;
    const int base = int(ctrl_values & ((uint64_t(1) << nctrl) - 1)), top = 1 << nctrl;
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        const size_t e = size_t(base + i * top) * D + (base + j * top);
        full[2 * e] = m[2 * (2 * i + j)];
        full[2 * e + 1] = m[2 * (2 * i + j) + 1];
      }
    int qq[QS_MAX_FUSED];
    for (int j = 0; j < nctrl; ++j) qq[j] = ctrls[j];
    qq[nctrl] = target;
    return fact_rc(st, qs::fact_apply(st->fact, qq, k, full.data()));
  }
  const int tbit = st->perm[target];
  fixed.pos[fixed.n++] = tbit;
  for (int i = 1; i < fixed.n; ++i)
    for (int j = i; j > 0 && fixed.pos[j - 1] > fixed.pos[j]; --j) std::swap(fixed.pos[j], fixed.pos[j - 1]);
  ProfScope ps(st, "apply_ctrl", 2.0 * std::ldexp(1.0, st->n - nctrl) * ab(st));
  hipError_t e;
  if (st->dtype == QS_C64)
    e = qs::launch_apply_ctrl(static_cast<float*>(st->amps), st->n, fixed, set_mask, tbit,
                              to_mat2<float>(m), st->stream);
  else
    e = qs::launch_apply_ctrl(static_cast<double*>(st->amps), st->n, fixed, set_mask, tbit,
                              to_mat2<double>(m), st->stream);
  return device_error(st, e, "apply_ctrl");
}

int qs_apply_cphase(qs_state* st, int a, int b, double theta) {
  if (int rc = check_state(st)) return rc;
  if (int rc = check_qubit(st, a, "qubit a")) return rc;
  if (int rc = check_qubit(st, b, "qubit b")) return rc;
  if (a == b) return fail(QS_E_INVAL, "controlled phase needs two distinct qubits");
  if (!std::isfinite(theta)) return fail(QS_E_INVAL, "theta is not finite");
  const double cr = std::cos(theta), ci = std::sin(theta);
  if (st->fact) {
    double d[32] = {0};
    d[0] = d[10] = d[20] = 1.0;
    d[30] = cr;
    d[31] = ci;
    const int qq[2] = {a, b};
    return fact_rc(st, qs::fact_apply(st->fact, qq, 2, d));
  }
  ProfScope ps(st, "cphase", 2.0 * std::ldexp(1.0, st->n - 2) * ab(st));
  hipError_t e;
  if (st->dtype == QS_C64)
    e = qs::launch_cphase(static_cast<float*>(st->amps), st->n, st->perm[a], st->perm[b],
                          float(cr), float(ci), st->stream);
  else
    e = qs::launch_cphase(static_cast<double*>(st->amps), st->n, st->perm[a], st->perm[b], cr, ci,
                          st->stream);
  return device_error(st, e, "apply_cphase");
}

int qs_apply_swap(qs_state* st, int a, int b) {
  if (int rc = check_state(st)) return rc;
  if (int rc = check_qubit(st, a, "qubit a")) return rc;
  if (int rc = check_qubit(st, b, "qubit b")) return rc;
  if (st->fact) return qs::fact_swap(st->fact, a, b);
  std::swap(st->perm[a], st->perm[b]);
  return QS_OK;
}

int qs_apply_gate(qs_state* st, int kind, const int* qubits, int nq, const double* params) {
  if (int rc = check_state(st)) return rc;
  if (!qubits) return fail(QS_E_INVAL, "qubits is NULL");
  if (kind < QS_GATE_H || kind > QS_GATE_CU3) return fail(QS_E_INVAL, "unknown gate kind %d", kind);
  const int arity = kind >= QS_GATE_CZ ? 2 : 1;
  if (kind == QS_GATE_CU3 ? (nq < 2 || nq > 9) : nq != arity)
    return fail(QS_E_INVAL, "gate kind %d on %d qubits", kind, nq);
  const int np = kind == QS_GATE_CP ? 1 : kind == QS_GATE_U3 ? 3 : kind == QS_GATE_CU3 ? 4 : 0;
  if (np > 0) {
    if (!params) return fail(QS_E_INVAL, "gate kind %d needs parameters", kind);
    for (int i = 0; i < np; ++i)
      if (!std::isfinite(params[i])) return fail(QS_E_INVAL, "parameter %d is not finite", i);
  }
  auto to8 = [](const std::vector<qs::cd>& u, double* m) {
    for (int e = 0; e < 4; ++e) {
      m[2 * e] = u[e].real();
      m[2 * e + 1] = u[e].imag();
    }
  };
  std::vector<qs::cd> u;
  int k = 0;
  double m2[8];
  switch (kind) {
    case QS_GATE_SWAP: return qs_apply_swap(st, qubits[0], qubits[1]);
    case QS_GATE_CP: return qs_apply_cphase(st, qubits[0], qubits[1], params[0]);
    case QS_GATE_CZ: return qs_apply_cphase(st, qubits[0], qubits[1], 3.14159265358979323846);
    case QS_GATE_CU3: {
      const int nctrl = nq - 1;
      const double v = params[3];
      if (!(v >= 0.0 && v < std::ldexp(1.0, nctrl) && v == std::floor(v)))
        return fail(QS_E_INVAL, "control values %g are not a %d-bit mask", v, nctrl);
      (void)qs::gate_matrix(QS_GATE_U3, 1, params, &u, &k);
      to8(u, m2);
      return qs_apply_ctrl(st, qubits, nctrl, uint64_t(v), qubits[nctrl], m2);
    }
    default: break;
  }
  if (!qs::gate_matrix(kind, arity, params, &u, &k)) return fail(QS_E_INVAL, "gate kind %d", kind);
  if (k == 1) {
    to8(u, m2);
    return qs_apply_1q(st, qubits[0], m2);
  }
  if (kind == QS_GATE_ISWAP) {
    double m4[32];
    for (int e = 0; e < 16; ++e) {
      m4[2 * e] = u[e].real();
      m4[2 * e + 1] = u[e].imag();
    }
    return qs_apply_fused(st, qubits, 2, m4);
  }
  // CX, CY, AX, AY, AZ: local bit 0 the control, bit 1 the target; the
  // target's 2x2 sits where the control takes its value cv
  const int cv = (kind == QS_GATE_CX || kind == QS_GATE_CY) ? 1 : 0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      const qs::cd x = u[size_t(cv + 2 * i) * 4 + (cv + 2 * j)];
      m2[2 * (2 * i + j)] = x.real();
      m2[2 * (2 * i + j) + 1] = x.imag();
    }
  return qs_apply_ctrl(st, qubits, 1, uint64_t(cv), qubits[1], m2);
}

int qs_apply_fused(qs_state* st, const int* qubits, int k, const double* m) {
  if (int rc = check_state(st)) return rc;
  if (!qubits) return fail(QS_E_INVAL, "qubits is NULL");
  if (k < 1 || k > QS_MAX_FUSED || k > st->n)
    return fail(QS_E_INVAL, "k = %d outside [1, min(%d, n)]", k, QS_MAX_FUSED);
  const size_t D = size_t(1) << k;
  if (int rc = check_finite(m, 2 * D * D)) return rc;
  int phys[QS_MAX_FUSED];
  uint64_t seen = 0;
  for (int j = 0; j < k; ++j) {
    if (int rc = check_qubit(st, qubits[j], "qubit")) return rc;
    if (seen & (uint64_t(1) << qubits[j])) return fail(QS_E_INVAL, "qubit %d used twice", qubits[j]);
    seen |= uint64_t(1) << qubits[j];
    phys[j] = st->perm[qubits[j]];
  }
  if (st->fact) return fact_rc(st, qs::fact_apply(st->fact, qubits, k, m));
  hipError_t e;
  if (st->dtype == QS_C64) {
    std::vector<float> mf(2 * D * D);
    for (size_t i = 0; i < mf.size(); ++i) mf[i] = static_cast<float>(m[i]);
    e = hipMemcpyAsync(st->mat, mf.data(), mf.size() * sizeof(float), hipMemcpyHostToDevice, st->stream);
  } else {
    e = hipMemcpyAsync(st->mat, m, 2 * D * D * sizeof(double), hipMemcpyHostToDevice, st->stream);
  }
  if (e == hipSuccess) e = launch_block(st, phys, k, st->mat);
  return device_error(st, e, "apply_fused");
}

// The multi-stage passes of the QFT on bits [start, start + len) of a dense
// vector of nq qubits at amps (the state's own or a subsystem's), stored in
// natural or bit-reversed order; no relabelling.
int qft_passes(qs_state* st, void* amps, int nq, int start, int len, bool reversed, int inverse) {
  qs::QftPass plan[64];
  const int np = st->dtype == QS_C64
                     ? qs::qft_plan<float>(nq, start, len, reversed, g_qft_tune, plan, 64)
                     : qs::qft_plan<double>(nq, start, len, reversed, g_qft_tune, plan, 64);
  if (np < 0) return fail(QS_E_UNSUPPORTED, "QFT pass plan failed");
  const int sign = inverse ? -1 : 1;
  static const char* kind_names[3][9] = {
      {"qft_lds", "qft_lds", "qft_lds", "qft_lds", "qft_lds", "qft_lds", "qft_lds", "qft_lds",
       "qft_lds"},
      {"", "qft_col1", "qft_col2", "qft_col3", "qft_col4", "qft_col5", "qft_col6", "qft_col7",
       "qft_col8"},
      {"", "qft_reg1", "qft_reg2", "qft_reg3", "qft_reg4", "qft_reg5", "", "", ""}};
  for (int k = 0; k < np; ++k) {
    const int g = plan[k].kind == qs::QftPass::LDS ? 0 : plan[k].hi - plan[k].lo;
    ProfScope ps(st, kind_names[plan[k].kind][g <= 8 ? g : 0],
                 2.0 * std::ldexp(1.0, nq) * ab(st));
    hipError_t e =
        st->dtype == QS_C64
            ? qs::launch_qft_pass(static_cast<float*>(amps), nq, start, len, plan[k], sign,
                                  reversed, g_qft_tune, st->stream)
            : qs::launch_qft_pass(static_cast<double*>(amps), nq, start, len, plan[k], sign,
                                  reversed, g_qft_tune, st->stream);
    if (int rc = device_error(st, e, "qft pass")) return rc;
  }
  return QS_OK;
}

// The QFT circuit gate by gate on a factorized state: for j from the top of
// the range down, H(j) then CP(m, j, pi / 2^(j - m)) for m from j - 1 down,
// then the reversing SWAPs (relabels); the inverse is the reversed sequence
// with negated angles. With the Z-eigenstate shortcut a basis input stays a
// product state (every CP has a control still in a Z eigenstate).
int qft_factorized(qs_state* st, int start, int len, int inverse) {
  // With no separation policy (an exact run) and the whole range inside one
  // subsystem as a block of consecutive local bits (ascending, or descending
  // as a previous transform leaves it), the gate sequence equals the dense
  // multi-stage passes on that subsystem's buffer, then the reversal as a
  // relabelling of the block.
  int t0 = 0;
  bool descending = false;
  qs::FactorState* f = st->fact;
  if (f->policy == QS_SEP_NONE) {
    const int si = qs::fact_block(f, start, len, &t0, &descending);
    if (si >= 0) {
      if (int rc = fact_rc(st, qs::fact_sync(f))) return rc;
      qs::Sub& S = f->subs[si];
      if (int rc = qft_passes(st, S.amps, S.nq, t0, len, descending, inverse)) return rc;
      for (int i = 0; i < len / 2; ++i) std::swap(S.q[t0 + i], S.q[t0 + len - 1 - i]);
      S.known = false;
      return QS_OK;
    }
  }
  qs_circuit* c = nullptr;
  if (int rc = qs_circuit_create(st->n, &c)) return rc;
  struct G {
    int kind, a, b;
    double th;
  };
  std::vector<G> seq;
  for (int j = start + len - 1; j >= start; --j) {
    seq.push_back({QS_GATE_H, j, 0, 0.0});
    for (int m = j - 1; m >= start; --m)
      seq.push_back({QS_GATE_CP, m, j, M_PI / std::ldexp(1.0, j - m)});
  }
  for (int i = 0; i < len / 2; ++i) seq.push_back({QS_GATE_SWAP, start + i, start + len - 1 - i, 0.0});
  if (inverse) {
    std::reverse(seq.begin(), seq.end());
    for (auto& g : seq) g.th = -g.th;
  }
  int rc = QS_OK;
  for (const auto& g : seq) {
    const int q[2] = {g.a, g.b};
    rc = qs_circuit_add_gate(c, g.kind, q, &g.th);
    if (rc) break;
  }
  if (rc == QS_OK) rc = qs_run(st, c);
  qs_circuit_free(c);
  return rc;
}

int qs_qft(qs_state* st, int start, int len, int inverse) {
  if (int rc = check_state(st)) return rc;
  if (start < 0 || len < 1 || start + len > st->n)
    return fail(QS_E_INVAL, "qubit range [%d, %d) outside [0, %d)", start, start + len, st->n);
  if (st->fact) return qft_factorized(st, start, len, inverse);
  // natural order, bit-reversed (left by an earlier transform), or anything
  // else, which is first moved back to the identity labelling
  bool identity = true, reversed = true;
  for (int k = 0; k < len; ++k) {
    identity &= st->perm[start + k] == start + k;
    reversed &= st->perm[start + k] == start + len - 1 - k;
  }
  if (!identity && !reversed) {
    if (int rc = materialize(st)) return rc;
    reversed = false;
  } else if (identity) {
    reversed = false;
  }
  if (int rc = qft_passes(st, st->amps, st->n, start, len, reversed, inverse)) return rc;
  // final bit reversal of the range, as a relabelling
  for (int i = 0; i < len / 2; ++i) std::swap(st->perm[start + i], st->perm[start + len - 1 - i]);
  return QS_OK;
}

// ------------------------------------------------------------------ circuits

int qs_circuit_free(qs_circuit* c) {
  if (!c) return QS_OK;
  qs::circuit_invalidate(c);
  delete c;
  return QS_OK;
}

namespace {

// The tile plan of circuit c for the state's precision and current labelling
// (planned on physical bits), uploaded once and cached in the circuit.
int tile_plan_for(qs_state* st, qs_circuit* c, qs_circuit::TileCache** out) {
  const int prec = st->dtype == QS_C64 ? 0 : 1;
  qs_circuit::TileCache& tc = c->tcache[prec];
  std::vector<int> key(st->perm, st->perm + st->n);
  if (tc.dev && tc.key == key && tc.plan.dense == (st->dtype == QS_C64 && g_tile_mfma) &&
      tc.plan.C == qs::tile_low_bits(st->dtype)) {
    *out = &tc;
    return QS_OK;
  }
  if (tc.dev) {
    (void)hipDeviceSynchronize();  // queued passes may still read the old tables
    dev_free(tc.dev);
    tc.dev = nullptr;
  }
  std::vector<qs::Gate> phys = c->gates;
  for (auto& g : phys)
    for (int j = 0; j < g.k; ++j) g.q[j] = st->perm[g.q[j]];
  const bool dense = st->dtype == QS_C64 && g_tile_mfma;
  tc.plan = qs::plan_tiles(phys, st->n, qs::tile_low_bits(st->dtype), qs::kTileRowBits, 4, dense);
  std::vector<unsigned char> host;
  size_t gates_at = 0, mats_at = 0, emb_at = 0;
  qs::tile_tables(tc.plan, prec == 0, &host, &gates_at, &mats_at, &emb_at);
  const size_t total = host.size();
  void* d = dev_alloc(std::max<size_t>(total, 256));
  if (!d) return fail(QS_E_NOMEM, "allocating %zu bytes of tile tables", total);
  const hipError_t e = hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dev_free(d);
    return device_error(st, e, "uploading tile tables");
  }
  tc.dev = d;
  tc.key = key;
  tc.gates_off = gates_at;
  tc.mats_off = mats_at;  // block-step matrices (and sparse-round matrices)
  tc.emb_off = emb_at;
  *out = &tc;
  return QS_OK;
}

int run_tiles(qs_state* st, qs_circuit* c) {
  qs_circuit::TileCache* tc = nullptr;
  if (int rc = tile_plan_for(st, c, &tc)) return rc;
  const char* base = static_cast<const char*>(tc->dev);
  const double bytes = 2.0 * std::ldexp(1.0, st->n) * ab(st);
  for (const auto& stp : tc->plan.steps) {
    hipError_t e;
    if (stp.block) {
      const void* dm = base + tc->mats_off + 2 * stp.mat * (st->dtype == QS_C64 ? 4 : 8);
      e = launch_block(st, stp.blk.q, stp.blk.k, dm);
    } else {
      qs::TileRows rows;
      for (int j = 0; j < qs::kTileRowBits; ++j) rows.b[j] = stp.hb[j];
      const void* rd = base + size_t(stp.r0) * 4 * sizeof(int32_t);
      const void* gt = base + tc->gates_off;
      if (tc->plan.dense) {
        ProfScope ps(st, "tile_mfma", bytes);
        e = qs::launch_tile_mfma(static_cast<float*>(st->amps), st->n, tc->plan.C, rows, rd,
                                 stp.nr, reinterpret_cast<const float*>(base + tc->emb_off),
                                 st->stream);
      } else {
        ProfScope ps(st, "tile_pass", bytes);
        e = st->dtype == QS_C64
                ? qs::launch_tile_pass(static_cast<float*>(st->amps), st->n, tc->plan.C, rows, rd,
                                       stp.nr, gt,
                                       reinterpret_cast<const float*>(base + tc->mats_off),
                                       st->stream)
                : qs::launch_tile_pass(static_cast<double*>(st->amps), st->n, tc->plan.C, rows,
                                       rd, stp.nr, gt,
                                       reinterpret_cast<const double*>(base + tc->mats_off),
                                       st->stream);
      }
    }
    if (int rc = device_error(st, e, "tile pass")) return rc;
  }
  return QS_OK;
}

}  // namespace

// Runs a circuit on a dense state as tile passes (unless blocks were chosen;
// the state must hold one tile's bits) or as planned blocks (planned with
// the default block width first if needed), one sweep each; the circuit's
// SWAP renaming is then folded into the state's labels. Factorized states
// apply the gates one by one.
int qs_run(qs_state* st, qs_circuit* c) {
  if (int rc = check_state(st)) return rc;
  if (!c) return fail(QS_E_INVAL, "circuit is NULL");
  if (c->n != st->n) return fail(QS_E_INVAL, "circuit has %d qubits, state %d", c->n, st->n);
  if (st->fact) {
    // approximate mode: gate by gate, so that the separation policy runs after
    // every multi-qubit gate; positions are the labels at the start. Runs of
    // one-qubit gates go together (one launch over the small subsystems; a
    // one-qubit gate never changes any qubit's eps), and with the plain
    // schedule the tests wait until a gate touches their subsystem, so that
    // the tests pending on many subsystems share one launch.
    qs::FactorState* f = st->fact;
    std::vector<double> m;
    std::vector<int> q1;
    std::vector<double> m1;
    // The host copies of one-qubit subsystems follow each one-qubit gate as it
    // is queued (so that the Z-eigenstate shortcut sees the circuit's state);
    // a gate the shortcut reduces to one qubit joins the queued run.
    auto flush_1q = [&]() -> int {
      if (q1.empty()) return QS_OK;
      f->mirrors_ahead = true;
      const int rc = qs::fact_apply_1q_run(f, q1.data(), m1.data(), int(q1.size()));
      f->mirrors_ahead = false;
      q1.clear();
      m1.clear();
      return rc;
    };
    auto push_1q = [&](int q, const double* g8) -> int {
      // the tests due on q's subsystem run before any gate after them, so
      // that a qubit they split off starts its host copy before this gate
      if (qs::fact_pending_on(f, &q, 1))
        if (int rc = qs::fact_settle(f)) return rc;
      q1.push_back(q);
      m1.insert(m1.end(), g8, g8 + 8);
      qs::fact_mirror_1q(f, q, g8);
      return QS_OK;
    };
    // Exact runs hold controlled phases and inversions between two
    // subsystems back (Table I: buffered and moved around H) while later
    // gates commute with them. The state is then the held gates applied to
    // the subsystems' ket (with the queued one-qubit run); held gates commute
    // with each other, so any of them may be applied first. Each is applied
    // with the shortcuts when a gate does not commute with it and at the end.
    const bool hold = qs::g_hold && f->policy == QS_SEP_NONE;
    std::vector<qs::HeldGate>& held = f->held;
    held.clear();
    auto apply_held = [&](const qs::HeldGate& hg) -> int {
      if (int rc = flush_1q()) return rc;
      int q2[2] = {hg.c, hg.t}, k2 = 2;
      std::vector<double> h2(32);
      qs::held_matrix(hg, h2.data());
      qs::fact_reduce(f, q2, &k2, &h2);
      if (k2 == 2) qs::fact_kickback(f, q2, &k2, &h2);
      if (k2 < 2) ++f->held_removed;  // no merge after all
      if (k2 == 0) return QS_OK;
      return qs::fact_apply(f, q2, k2, h2.data());
    };
    auto apply_held_on = [&](const int* qq, int k, const qs::HeldGate* with) -> int {
      for (size_t i = 0; i < held.size();) {
        const qs::HeldGate& hg = held[i];
        bool on = false;
        for (int j = 0; j < k; ++j) on |= hg.c == qq[j] || hg.t == qq[j];
        if (on && !(with && qs::held_commute(*with, hg))) {
          const qs::HeldGate x = hg;
          held.erase(held.begin() + long(i));
          if (int rc = apply_held(x)) return rc;
          continue;
        }
        ++i;
      }
      return QS_OK;
    };
    // a one-qubit gate moves in front of the held gates on its qubit (which
    // it conjugates), or the ones it cannot pass are applied first
    auto hold_1q = [&](int q, const double* u) -> int {
      for (size_t i = 0; i < held.size();) {
        qs::HeldGate& hg = held[i];
        if ((hg.c == q || hg.t == q) && !qs::held_pass_1q(&hg, q, u)) {
          const qs::HeldGate x = hg;
          held.erase(held.begin() + long(i));
          if (int rc = apply_held(x)) return rc;
          continue;
        }
        ++i;
      }
      return push_1q(q, u);
    };
    // a controlled phase or inversion that commutes with every held gate on
    // its qubits (the others applied first) and spans two subsystems is held,
    // folded into a held gate on the same control and target if there is one;
    // *taken = 1 when the gate needs nothing more (held, folded or reduced)
    auto hold_2q = [&](const int* qq, const std::vector<double>& gm, int* taken) -> int {
      *taken = 0;
      qs::HeldGate g;
      if (!qs::held_classify(gm.data(), qq, &g)) return apply_held_on(qq, 2, nullptr);
      if (int rc = apply_held_on(qq, 2, &g)) return rc;
      // (both shortcuts need an operand that is a subsystem of its own)
      int q2[2] = {g.c, g.t}, k2 = 2;
      std::vector<double> h2(32);
      qs::held_matrix(g, h2.data());
      if (qs::fact_reduce(f, q2, &k2, &h2) || qs::fact_kickback(f, q2, &k2, &h2)) {
        *taken = 1;  // applied to the ket at once: one qubit or nothing
        return k2 == 0 ? QS_OK : push_1q(q2[0], h2.data());
      }
      if (qs::fact_sub_of(f, g.c) == qs::fact_sub_of(f, g.t)) return QS_OK;
      *taken = 1;
      ++f->held_in;
      for (size_t i = 0; i < held.size(); ++i) {
        qs::HeldGate& hg = held[i];
        // phases with d0 = 1 are symmetric: one on the reversed pair is read
        // with this orientation
        if (hg.c == g.t && hg.t == g.c && !hg.inv && !g.inv &&
            std::abs(hg.d0 - 1.0) <= 1e-13 && std::abs(g.d0 - 1.0) <= 1e-13)
          std::swap(hg.c, hg.t);
        if (hg.c != g.c || hg.t != g.t) continue;
        // g after hg: the target matrices multiply
        const std::complex<double> A[4] = {g.inv ? 0.0 : g.d0, g.inv ? g.d0 : 0.0,
                                           g.inv ? g.d1 : 0.0, g.inv ? 0.0 : g.d1};
        const std::complex<double> B[4] = {hg.inv ? 0.0 : hg.d0, hg.inv ? hg.d0 : 0.0,
                                           hg.inv ? hg.d1 : 0.0, hg.inv ? 0.0 : hg.d1};
        double p4[32];
        qs::HeldGate x;
        x.c = g.c;
        x.t = g.t;
        std::fill(p4, p4 + 32, 0.0);
        p4[0] = p4[20] = 1.0;
        for (int r = 0; r < 2; ++r)
          for (int cc = 0; cc < 2; ++cc) {
            const std::complex<double> v = A[2 * r] * B[cc] + A[2 * r + 1] * B[2 + cc];
            const int e = 4 * (1 + 2 * r) + (1 + 2 * cc);
            p4[2 * e] = v.real();
            p4[2 * e + 1] = v.imag();
          }
        const int qc[2] = {g.c, g.t};
        if (!qs::held_classify(p4, qc, &x)) {  // (a product of two such is one)
          const qs::HeldGate old = hg;
          held.erase(held.begin() + long(i));
          if (int rc = apply_held(old)) return rc;
          return apply_held(g);
        }
        held.erase(held.begin() + long(i));
        ++f->held_removed;  // g folded in
        if (!x.inv && std::abs(x.d0 - x.d1) <= 1e-13) {
          // control 1: a global phase d0 on the target = diag(1, d0) on the control
          ++f->held_removed;
          if (std::abs(x.d0 - 1.0) <= 1e-13) return QS_OK;  // cancelled
          const double u[8] = {1.0, 0.0, 0.0, 0.0, 0.0, 0.0, x.d0.real(), x.d0.imag()};
          return push_1q(x.c, u);
        }
        held.push_back(x);
        return QS_OK;
      }
      held.push_back(g);
      return QS_OK;
    };
    auto apply_all = [&]() -> int {
      for (const auto& g : c->gates) {
        m.resize(2 * g.m.size());
        for (size_t i = 0; i < g.m.size(); ++i) {
          m[2 * i] = g.m[i].real();
          m[2 * i + 1] = g.m[i].imag();
        }
        int qq[QS_MAX_FUSED], k = g.k;
        for (int j = 0; j < k; ++j) qq[j] = g.q[j];
        if (k >= 2) {
          if (qs::fact_pending_on(f, qq, k)) {  // the tests due before this gate
            if (int rc = flush_1q()) return rc;
            if (int rc = qs::fact_settle(f)) return rc;
          }
          if (hold) {
            // with no held gate on its qubits the gate commutes with all of
            // them, and the shortcut may take it at once
            bool touched = false;
            for (const auto& hg : held)
              for (int j = 0; j < k; ++j) touched |= hg.c == qq[j] || hg.t == qq[j];
            if (!touched && qs::fact_reduce(f, qq, &k, &m)) {
              if (k == 0) continue;
              if (k == 1) {
                if (int rc = push_1q(qq[0], m.data())) return rc;
                continue;
              }
            }
            int taken = 0;
            if (k == 2) {
              if (int rc = hold_2q(qq, m, &taken)) return rc;
            } else if (int rc = apply_held_on(qq, k, nullptr)) {
              return rc;
            }
            if (taken) continue;
          }
          if (qs::fact_reduce(f, qq, &k, &m) && k == 0) continue;
          // (a gate reduced here already commutes with every held gate)
          if (k == 1) {
            if (int rc = push_1q(qq[0], m.data())) return rc;
            continue;
          }
        }
        if (k == 1) {
          if (int rc = hold ? hold_1q(qq[0], m.data()) : push_1q(qq[0], m.data())) return rc;
          continue;
        }
        if (int rc = flush_1q()) return rc;
        if (int rc = qs::fact_apply(f, qq, k, m.data())) return rc;
      }
      while (!held.empty()) {
        const qs::HeldGate x = held.front();
        held.erase(held.begin());
        if (int rc = apply_held(x)) return rc;
      }
      return flush_1q();
    };
    // A failed gate leaves the gates before it applied; the gates still held
    // then are applied too (they commute with each other), so that the state
    // is that prefix of the circuit. If one of them fails as well, the state
    // is none of the circuit's and the handle refuses every later call.
    auto apply_all_or_prefix = [&]() -> int {
      const int rc = apply_all();
      if (rc == QS_OK || held.empty()) return rc;
      const std::string why = g_err;
      while (!held.empty()) {
        const qs::HeldGate x = held.front();
        held.erase(held.begin());
        if (apply_held(x) != QS_OK || flush_1q() != QS_OK) {
          held.clear();
          st->poisoned = true;
          st->poison_why = "run that failed with gates held back";
          break;
        }
      }
      g_err = why;
      return rc;
    };
    qs::fact_begin_run(f);
    if (int rc = fact_rc(st, qs::fact_end_run(f, apply_all_or_prefix()))) return rc;
    return fact_rc(st, qs::fact_relabel(f, c->pos.data()));
  }
  if (c->tiles != 0 && !c->gates.empty() &&
      st->n >= qs::tile_low_bits(st->dtype) + qs::kTileRowBits) {
    if (int rc = run_tiles(st, c)) return rc;
    int np[64];
    for (int q = 0; q < st->n; ++q) np[q] = st->perm[c->pos[q]];
    for (int q = 0; q < st->n; ++q) st->perm[q] = np[q];
    return QS_OK;
  }
  if (!c->planned)
    if (int rc = qs::circuit_plan_blocks(c, c->kmax)) return rc;
  const int prec = st->dtype == QS_C64 ? 0 : 1;
  if (!c->dmat[prec] && !c->blocks.empty()) {
    size_t total = 0;
    c->off[prec].clear();
    for (const auto& b : c->blocks) {
      c->off[prec].push_back(total);
      total += 2 * b.m.size();
    }
    const size_t esz = prec == 0 ? sizeof(float) : sizeof(double);
    void* d = dev_alloc(total * esz);
    if (!d) return fail(QS_E_NOMEM, "allocating %zu bytes of block matrices", total * esz);
    hipError_t e;
    if (prec == 0) {
      std::vector<float> h(total);
      for (size_t bi = 0; bi < c->blocks.size(); ++bi)
        for (size_t i = 0; i < c->blocks[bi].m.size(); ++i) {
          h[c->off[0][bi] + 2 * i] = float(c->blocks[bi].m[i].real());
          h[c->off[0][bi] + 2 * i + 1] = float(c->blocks[bi].m[i].imag());
        }
      e = hipMemcpy(d, h.data(), total * esz, hipMemcpyHostToDevice);
    } else {
      std::vector<double> h(total);
      for (size_t bi = 0; bi < c->blocks.size(); ++bi)
        for (size_t i = 0; i < c->blocks[bi].m.size(); ++i) {
          h[c->off[1][bi] + 2 * i] = c->blocks[bi].m[i].real();
          h[c->off[1][bi] + 2 * i + 1] = c->blocks[bi].m[i].imag();
        }
      e = hipMemcpy(d, h.data(), total * esz, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
      dev_free(d);
      return device_error(st, e, "uploading block matrices");
    }
    c->dmat[prec] = d;
  }
  const size_t esz = prec == 0 ? sizeof(float) : sizeof(double);
  for (size_t bi = 0; bi < c->blocks.size(); ++bi) {
    const qs::Block& b = c->blocks[bi];
    int phys[QS_MAX_FUSED];
    for (int j = 0; j < b.k; ++j) phys[j] = st->perm[b.q[j]];
    const void* dm = static_cast<const char*>(c->dmat[prec]) + c->off[prec][bi] * esz;
    if (int rc = device_error(st, launch_block(st, phys, b.k, dm), "run block")) return rc;
  }
  int np[64];
  for (int q = 0; q < st->n; ++q) np[q] = st->perm[c->pos[q]];
  for (int q = 0; q < st->n; ++q) st->perm[q] = np[q];
  return QS_OK;
}

// ------------------------------------------------------------------ approximate mode

int qs_set_separation_policy(qs_state* st, int policy, double p) {
  if (int rc = check_state(st)) return rc;
  if (!st->fact) return fail(QS_E_UNSUPPORTED, "separation applies to factorized states");
  if (policy != QS_SEP_NONE && policy != QS_SEP_AFTER_2Q && policy != QS_SEP_AFTER_2Q_PAIRS)
    return fail(QS_E_INVAL, "unknown policy %d", policy);
  if (!(p >= 0.0 && p <= 1.0)) return fail(QS_E_INVAL, "p = %g outside [0, 1]", p);
  st->fact->policy = policy;
  st->fact->p = p;
  return QS_OK;
}

int qs_try_separate_pair(qs_state* st, int qa, int qb, double p, int* rounded) {
  if (int rc = check_state(st)) return rc;
  if (!st->fact) return fail(QS_E_INVAL, "the pair rounding applies to factorized states");
  if (qa < 0 || qb < 0 || qa >= st->n || qb >= st->n || qa == qb)
    return fail(QS_E_INVAL, "bad pair (%d, %d)", qa, qb);
  if (!(p >= 0.0 && p <= 1.0)) return fail(QS_E_INVAL, "p = %g outside [0, 1]", p);
  bool r = false;
  if (int rc = fact_rc(st, qs::fact_test_pair(st->fact, qa, qb, p, &r))) return rc;
  if (rounded) *rounded = r ? 1 : 0;
  return QS_OK;
}

int qs_hermitian4_top(const double* h, double* lambda, double* phi) {
  if (!h || !lambda || !phi) return fail(QS_E_INVAL, "NULL argument");
  for (int i = 0; i < 32; ++i)
    if (!std::isfinite(h[i])) return fail(QS_E_INVAL, "non-finite matrix entry");
  qs::fact_hermitian4_top(h, lambda, phi);
  return QS_OK;
}

int qs_try_separate(qs_state* st, double p, int* n_separated) {
  if (int rc = check_state(st)) return rc;
  if (!(p >= 0.0 && p <= 1.0)) return fail(QS_E_INVAL, "p = %g outside [0, 1]", p);
  if (!st->fact) {
    if (n_separated) *n_separated = 0;
    return QS_OK;
  }
  return fact_rc(st, qs::fact_try_separate(st->fact, p, n_separated));
}

int qs_mark_dirty(qs_state* st, uint64_t mask) {
  if (int rc = check_state(st)) return rc;
  if (!st->fact) return QS_OK;
  if (st->n < 64) mask &= (uint64_t(1) << st->n) - 1;
  st->fact->dirty |= mask;
  return QS_OK;
}

int qs_fidelity_estimate(const qs_state* st, double* F) {
  if (!st || !F) return fail(QS_E_INVAL, "NULL argument");
  *F = st->fact ? st->fact->F : 1.0;
  return QS_OK;
}

int qs_subsystems(const qs_state* st, int* qubit_to_sub, int* sizes, int* nsub) {
  if (!st || !nsub) return fail(QS_E_INVAL, "NULL argument");
  if (!st->fact) {
    if (qubit_to_sub)
      for (int q = 0; q < st->n; ++q) qubit_to_sub[q] = 0;
    if (sizes) sizes[0] = st->n;
    *nsub = 1;
    return QS_OK;
  }
  const auto& subs = st->fact->subs;
  for (int s = 0; s < int(subs.size()); ++s) {
    if (sizes) sizes[s] = subs[s].nq;
    if (qubit_to_sub)
      for (int t = 0; t < subs[s].nq; ++t) qubit_to_sub[subs[s].q[t]] = s;
  }
  *nsub = int(subs.size());
  return QS_OK;
}

int qs_subsystem_qubits(const qs_state* st, int s, int* qubits, int* nq) {
  if (!st || !nq) return fail(QS_E_INVAL, "NULL argument");
  if (!st->fact) return fail(QS_E_UNSUPPORTED, "dense state");
  if (s < 0 || s >= int(st->fact->subs.size())) return fail(QS_E_INVAL, "subsystem %d out of range", s);
  *nq = st->fact->subs[s].nq;
  if (qubits)
    for (int t = 0; t < *nq; ++t) qubits[t] = st->fact->subs[s].q[t];
  return QS_OK;
}

int qs_set_attempt_log(qs_state* st, qs_attempt* buf, uint64_t cap, uint64_t* count) {
  if (int rc = check_state(st)) return rc;
  if (!st->fact) return fail(QS_E_UNSUPPORTED, "attempts happen on factorized states");
  if ((buf == nullptr) != (count == nullptr)) return fail(QS_E_INVAL, "buf and count go together");
  st->fact->log = buf;
  st->fact->log_cap = cap;
  st->fact->log_count = count;
  if (count) *count = 0;
  return QS_OK;
}

int qs_expand(qs_state* fact, qs_state* dense) {
  if (int rc = check_state(fact)) return rc;
  if (int rc = check_state(dense)) return rc;
  if (!fact->fact || dense->fact) return fail(QS_E_INVAL, "expand takes a factorized and a dense state");
  if (fact->n != dense->n || fact->dtype != dense->dtype)
    return fail(QS_E_INVAL, "states differ in width or precision");
  (void)hipStreamSynchronize(dense->stream);
  int perm[64];
  if (int rc = fact_rc(fact, qs::fact_expand(fact->fact, dense->amps, perm))) return rc;
  for (int q = 0; q < fact->n; ++q) dense->perm[q] = perm[q];
  return QS_OK;
}

int qs_inner_product(qs_state* a, qs_state* b, double* re, double* im) {
  if (int rc = check_state(a)) return rc;
  if (int rc = check_state(b)) return rc;
  if (!re || !im) return fail(QS_E_INVAL, "NULL output");
  if (a->fact || b->fact) return fail(QS_E_UNSUPPORTED, "inner product of dense states");
  if (a->n != b->n || a->dtype != b->dtype) return fail(QS_E_INVAL, "states differ in width or precision");
  if (int rc = materialize(a)) return rc;
  if (int rc = materialize(b)) return rc;
  (void)hipStreamSynchronize(b->stream);
  hipError_t e = a->dtype == QS_C64
                     ? qs::launch_inner(static_cast<const float*>(a->amps), static_cast<const float*>(b->amps), dim(a), a->red, a->stream)
                     : qs::launch_inner(static_cast<const double*>(a->amps), static_cast<const double*>(b->amps), dim(a), a->red, a->stream);
  double v[2] = {0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(v, a->red, sizeof v, hipMemcpyDeviceToHost, a->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(a->stream);
  *re = v[0];
  *im = v[1];
  return device_error(a, e, "inner product");
}

int qs_set_proposer(qs_state* st, qs_mlp* net, const qs_propose_cfg* cfg) {
  if (int rc = check_state(st)) return rc;
  if (!st->fact) return fail(QS_E_UNSUPPORTED, "proposals apply to factorized states");
  if (net) {
    if (!cfg) return fail(QS_E_INVAL, "cfg is NULL");
    if (!(cfg->cutoff >= 0.0 && cfg->cutoff <= 1.0))
      return fail(QS_E_INVAL, "cutoff %g outside [0, 1]", cfg->cutoff);
    if (cfg->flags & ~QS_PROPOSE_RETEST_ON_MERGE)
      return fail(QS_E_INVAL, "unknown proposer flags %#x", unsigned(cfg->flags));
    if (cfg->min_qubits < 2 || cfg->min_qubits > 64)
      return fail(QS_E_INVAL, "min_qubits %d outside [2, 64]", int(cfg->min_qubits));
    st->fact->cutoff = cfg->cutoff;
    st->fact->propose_flags = cfg->flags;
    st->fact->propose_min = cfg->min_qubits;
  }
  st->fact->proposer = net;
  if (!net) {
    st->fact->dirty |= st->fact->deferred;
    st->fact->deferred = 0;
  }
  return QS_OK;
}

int qs_set_feature_log(qs_state* st, float* buf, uint64_t cap) {
  if (int rc = check_state(st)) return rc;
  if (!st->fact) return fail(QS_E_UNSUPPORTED, "features belong to factorized states");
  st->fact->feat_log = buf;
  st->fact->feat_cap = buf ? cap : 0;
  return QS_OK;
}

int qs_shortcut_count(const qs_state* st, uint64_t* count) {
  if (int rc = check_state(st)) return rc;
  if (!count) return fail(QS_E_INVAL, "count is NULL");
  *count = st->fact ? st->fact->shortcuts : 0;
  return QS_OK;
}

int qs_held_count(const qs_state* st, uint64_t* held, uint64_t* removed) {
  if (int rc = check_state(st)) return rc;
  if (!held || !removed) return fail(QS_E_INVAL, "held or removed is NULL");
  *held = st->fact ? st->fact->held_in : 0;
  *removed = st->fact ? st->fact->held_removed : 0;
  return QS_OK;
}

int qs_proposer_stats(const qs_state* st, uint64_t* skipped, uint64_t* fallback_tests) {
  if (!st) return fail(QS_E_INVAL, "state is NULL");
  if (skipped) *skipped = st->fact ? st->fact->skipped : 0;
  if (fallback_tests) *fallback_tests = st->fact ? st->fact->fallback_tests : 0;
  return QS_OK;
}

// ------------------------------------------------------------------ profiling

int qs_profile_start(qs_state* st) {
  if (int rc = check_state(st)) return rc;
  if (int rc = sync(st, "profile start")) return rc;
  for (auto& r : st->recs) {
    st->pool.push_back(r.a);
    st->pool.push_back(r.b);
  }
  st->recs.clear();
  st->prof = true;
  return QS_OK;
}

int qs_profile_stop(qs_state* st, qs_kernel_stat* out, int max_out, int* count) {
  if (int rc = check_state(st)) return rc;
  if (!count || (max_out > 0 && !out)) return fail(QS_E_INVAL, "NULL output");
  st->prof = false;
  if (int rc = sync(st, "profile stop")) return rc;
  int nk = 0;
  for (auto& r : st->recs) {
    float ms = 0.f;
    hipError_t e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return device_error(st, e, "event timing");
    int k = 0;
    while (k < nk && std::strcmp(out[k].name, r.name) != 0) ++k;
    if (k == nk) {
      if (nk >= max_out) continue;
      std::memset(&out[k], 0, sizeof out[k]);
      std::snprintf(out[k].name, sizeof out[k].name, "%s", r.name);
      ++nk;
    }
    out[k].launches += 1;
    out[k].total_ms += ms;
    out[k].bytes += r.bytes;
  }
  for (auto& r : st->recs) {
    st->pool.push_back(r.a);
    st->pool.push_back(r.b);
  }
  st->recs.clear();
  *count = nk;
  return QS_OK;
}

// ------------------------------------------------------------------ readout

// Dense copy of a factorized state (at most 30 qubits) for full readouts.
static int dense_copy(qs_state* st, qs_state** out) {
  if (st->n > 30) return fail(QS_E_UNSUPPORTED, "full readout of a factorized state needs n <= 30");
  qs_state* d = nullptr;
  if (int rc = qs_alloc(st->n, st->dtype, &d)) return rc;
  d->stream = st->stream;
  if (int rc = qs_expand(st, d)) {
    qs_free(d);
    return rc;
  }
  *out = d;
  return QS_OK;
}

int qs_amplitudes(qs_state* st, void* host_out, uint64_t count, int out_dtype) {
  if (int rc = check_state(st)) return rc;
  if (!host_out) return fail(QS_E_INVAL, "output pointer is NULL");
  if (count != dim(st)) return fail(QS_E_INVAL, "count %llu != 2^%d", (unsigned long long)count, st->n);
  if (out_dtype != QS_C64 && out_dtype != QS_C128) return fail(QS_E_INVAL, "unknown dtype %d", out_dtype);
  if (st->fact) {
    qs_state* d = nullptr;
    if (int rc = dense_copy(st, &d)) return rc;
    const int rc = qs_amplitudes(d, host_out, count, out_dtype);
    qs_free(d);
    return rc;
  }
  if (int rc = materialize(st)) return rc;
  const size_t ob = amp_bytes(out_dtype), sb = amp_bytes(st->dtype);
  if (out_dtype == st->dtype) {
    hipError_t e = hipMemcpyAsync(host_out, st->amps, count * sb, hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
    return device_error(st, e, "download");
  }
  const uint64_t chunk = count < kStageAmps ? count : kStageAmps;
  void* stage = dev_alloc(chunk * ob);
  if (!stage) return fail(QS_E_NOMEM, "staging allocation failed");
  hipError_t e = hipSuccess;
  for (uint64_t off = 0; off < count && e == hipSuccess; off += chunk) {
    const uint64_t c = count - off < chunk ? count - off : chunk;
    const char* src = static_cast<const char*>(st->amps) + off * sb;
    if (out_dtype == QS_C128)
      e = qs::launch_convert(static_cast<double*>(stage), reinterpret_cast<const float*>(src), c, st->stream);
    else
      e = qs::launch_convert(static_cast<float*>(stage), reinterpret_cast<const double*>(src), c, st->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(static_cast<char*>(host_out) + off * ob, stage, c * ob, hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  }
  dev_free(stage);
  return device_error(st, e, "download");
}

int qs_amplitudes_gather(qs_state* st, const uint64_t* idx, uint64_t m, double* out) {
  if (int rc = check_state(st)) return rc;
  if (m == 0) return QS_OK;
  if (!idx || !out) return fail(QS_E_INVAL, "NULL pointer");
  for (uint64_t j = 0; j < m; ++j)
    if (idx[j] >= dim(st)) return fail(QS_E_INVAL, "index %llu >= 2^%d", (unsigned long long)idx[j], st->n);
  if (st->fact) return fact_rc(st, qs::fact_gather(st->fact, idx, m, out));
  qs::Perm64 perm{};
  perm.n = st->n;
  for (int q = 0; q < st->n; ++q) perm.p[q] = static_cast<int8_t>(st->perm[q]);
  uint64_t* didx = static_cast<uint64_t*>(dev_alloc(m * sizeof(uint64_t)));
  double* dout = static_cast<double*>(dev_alloc(m * 2 * sizeof(double)));
  if (!didx || !dout) {
    dev_free(didx);
    dev_free(dout);
    return fail(QS_E_NOMEM, "staging allocation failed");
  }
  hipError_t e = hipMemcpyAsync(didx, idx, m * sizeof(uint64_t), hipMemcpyHostToDevice, st->stream);
  if (e == hipSuccess)
    e = st->dtype == QS_C64 ? qs::launch_gather(static_cast<const float*>(st->amps), didx, m, perm, dout, st->stream)
                            : qs::launch_gather(static_cast<const double*>(st->amps), didx, m, perm, dout, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, m * 2 * sizeof(double), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  dev_free(didx);
  dev_free(dout);
  return device_error(st, e, "gather");
}

int qs_amplitudes_gather_noalloc(qs_state* st, const uint64_t* idx, uint64_t m, double* out) {
  if (int rc = check_state(st)) return rc;
  if (m == 0) return QS_OK;
  if (!idx || !out) return fail(QS_E_INVAL, "NULL pointer");
  if (m > kNoAllocMax)
    return fail(QS_E_INVAL, "%llu indices exceed the no-allocation limit %llu",
                (unsigned long long)m, (unsigned long long)kNoAllocMax);
  if (st->fact) return fail(QS_E_UNSUPPORTED, "factorized states: use qs_amplitudes_gather");
  for (uint64_t j = 0; j < m; ++j)
    if (idx[j] >= dim(st)) return fail(QS_E_INVAL, "index %llu >= 2^%d", (unsigned long long)idx[j], st->n);
  void* base = nullptr;
  if (int rc = noalloc_scratch(st, &base)) return rc;
  uint64_t* didx = static_cast<uint64_t*>(base);
  double* dout = reinterpret_cast<double*>(static_cast<char*>(base) + kNoAllocIdxBytes);
  qs::Perm64 perm{};
  perm.n = st->n;
  for (int q = 0; q < st->n; ++q) perm.p[q] = static_cast<int8_t>(st->perm[q]);
  hipError_t e = hipMemcpyAsync(didx, idx, m * sizeof(uint64_t), hipMemcpyHostToDevice, st->stream);
  if (e == hipSuccess)
    e = st->dtype == QS_C64 ? qs::launch_gather(static_cast<const float*>(st->amps), didx, m, perm, dout, st->stream)
                            : qs::launch_gather(static_cast<const double*>(st->amps), didx, m, perm, dout, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, dout, m * 2 * sizeof(double), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  return device_error(st, e, "gather");
}

int qs_probs(qs_state* st, double* out, uint64_t count) {
  if (int rc = check_state(st)) return rc;
  if (!out) return fail(QS_E_INVAL, "output pointer is NULL");
  if (count != dim(st)) return fail(QS_E_INVAL, "count %llu != 2^%d", (unsigned long long)count, st->n);
  if (st->fact) {
    qs_state* d = nullptr;
    if (int rc = dense_copy(st, &d)) return rc;
    const int rc = qs_probs(d, out, count);
    qs_free(d);
    return rc;
  }
  if (int rc = materialize(st)) return rc;
  const uint64_t chunk = count < kStageAmps ? count : kStageAmps;
  double* stage = static_cast<double*>(dev_alloc(chunk * sizeof(double)));
  if (!stage) return fail(QS_E_NOMEM, "staging allocation failed");
  const size_t sb = amp_bytes(st->dtype);
  hipError_t e = hipSuccess;
  for (uint64_t off = 0; off < count && e == hipSuccess; off += chunk) {
    const uint64_t c = count - off < chunk ? count - off : chunk;
    const char* src = static_cast<const char*>(st->amps) + off * sb;
    e = st->dtype == QS_C64 ? qs::launch_probs(reinterpret_cast<const float*>(src), c, stage, st->stream)
                            : qs::launch_probs(reinterpret_cast<const double*>(src), c, stage, st->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(out + off, stage, c * sizeof(double), hipMemcpyDeviceToHost, st->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  }
  dev_free(stage);
  return device_error(st, e, "probs");
}

int qs_norm(qs_state* st, double* out) {
  if (int rc = check_state(st)) return rc;
  if (!out) return fail(QS_E_INVAL, "output pointer is NULL");
  if (st->fact) return fact_rc(st, qs::fact_norm(st->fact, out));
  const int nb = qs::reduce_blocks(dim(st));
  hipError_t e = st->dtype == QS_C64
                     ? qs::launch_norm(static_cast<const float*>(st->amps), dim(st), st->red, st->red + nb, st->stream)
                     : qs::launch_norm(static_cast<const double*>(st->amps), dim(st), st->red, st->red + nb, st->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(out, st->red + nb, sizeof(double), hipMemcpyDeviceToHost, st->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(st->stream);
  return device_error(st, e, "norm");
}

int qs_check(qs_state* st, double tol) {
  double nrm = 0;
  if (int rc = qs_norm(st, &nrm)) return rc;
  if (!(std::fabs(nrm - 1.0) <= tol))
    return fail(QS_E_NUMERIC, "norm %.17g differs from 1 by more than %g", nrm, tol);
  return QS_OK;
}

}  // extern "C"
