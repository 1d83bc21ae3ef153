// Factorized ket of the approximate mode (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <vector>

#include "../../include/qs.h"

namespace qs {

// One subsystem: q[t] is the qubit stored at bit t of its amplitude index.
struct Sub {
  int nq = 0;
  int q[64] = {0};
  void* amps = nullptr;  // 2^nq amplitudes, device, owned
  uint64_t phase = 0;    // deferred separation: the gate its dirty qubits wait on
  uint64_t phase_gates = 0;  // multi-qubit gates applied when that phase began
  bool plain = false;    // deferred separation: exact tests without the proposer
  int pend_a = -1, pend_b = -1;  // deferred pair policy: the pair test its gate made due
  // one-qubit subsystems: a float64 host copy of the two amplitudes when they
  // are known (set at creation from host values, kept through one-qubit
  // gates); it decides the Z-eigenstate shortcuts
  bool known = false;
  double h[4] = {0, 0, 0, 0};
};

// A controlled gate held back instead of merging its two subsystems: when
// qubit c is 1, qubit t takes diag(d0, d1) (a phase, inv false) or
// [[0, d0], [d1, 0]] (an inversion, inv true).
struct HeldGate {
  int c = 0, t = 0;
  bool inv = false;
  std::complex<double> d0{1.0, 0.0}, d1{1.0, 0.0};
};

struct FactorState {
  int n = 0;
  int dtype = QS_C64;
  uint64_t max_amps = 0;
  hipStream_t stream = nullptr;
  std::vector<Sub> subs;
  double F = 1.0;          // fidelity estimate, Eq. fid_model
  uint64_t dirty = 0;      // qubits whose reduced state may have changed
  int policy = QS_SEP_NONE;
  double p = 0.0;          // SDRP threshold parameter of the policy
  double tau = 1e-6;       // tolerance of the exact-separability test (Sec. III-A)
  qs_attempt* log = nullptr;
  uint64_t log_cap = 0;
  uint64_t* log_count = nullptr;
  double* scratch = nullptr;  // device reduction scratch
  // pinned, mapped host buffer of Bloch sums: 4 per target qubit, up to 5
  // targets for each of up to 32 subsystems (those of two qubits or more)
  static constexpr int kStatDoubles = 32 * 4 * 5;
  double* hstat = nullptr;
  double* dstat = nullptr;    // its device address
  // Deferred separation (plain schedule inside qs_run): the tests due after a
  // multi-qubit gate wait until a later gate touches that subsystem or the run
  // ends, and the tests pending on many subsystems then share one launch and
  // one synchronization. A subsystem's tests read only its own amplitudes, so
  // the decisions are those of testing at once; the attempts are logged, and
  // F updated, in the order of the gates that caused them.
  struct Decision {
    uint64_t phase;
    int q, nsub;
    double eps;
    bool rounded;
    int partner;     // a pair attempt's second qubit, else -1
    uint64_t gates;  // multi-qubit gates applied before the test (its place in the circuit)
  };
  bool defer = false;
  bool flushing = false;
  uint64_t phase_next = 0, cur_phase = 0, cur_gates = 0;
  std::vector<Decision> pend;
  std::vector<float> pend_feat;         // features of each held-back attempt (feature log on)
  float cur_feat[QS_MLP_INPUTS] = {0};  // features of the attempt being decided
  uint64_t prop = 0;                    // learned schedule: scored, proposed, not yet tested
  // While deferring, merges with their two-qubit gate and projections are
  // queued and launched together at the next point that reads device data.
  // No queued operation reads another's output (a gate on a subsystem whose
  // tests are pending runs those tests first, which launches the queue), and
  // buffers freed meanwhile return to the pool only after the launch.
  struct QOp {
    int kind = 0;  // 0: merge (nb > 0) or in place (nb = 0), then the gate; 1: projection
    void *a = nullptr, *b = nullptr, *c = nullptr, *single = nullptr;
    int na = 0, nb = 0, t0 = 0, t1 = 0;
    double phi[4] = {0, 0, 0, 0};
    double scale = 1.0;
    double m[32] = {0};
  };
  std::vector<QOp> qops;
  std::vector<std::pair<int, void*>> late_free;
  // mapped pinned slots for the tables of batched one-qubit gates; a slot is
  // reused only after the event recorded behind its launch has completed
  static constexpr int kRingSlots = 4;
  static constexpr size_t kSlotBytes = size_t(64) << 10;
  void* ring_host[kRingSlots] = {nullptr};
  void* ring_dev[kRingSlots] = {nullptr};
  hipEvent_t ring_ev[kRingSlots] = {nullptr};
  bool ring_used[kRingSlots] = {false};
  int ring_next = 0;
  // completion signal of the batched sweeps: a device counter, a host-mapped
  // flag the last workgroup sets to the launch's sequence number
  unsigned* sig_count = nullptr;
  unsigned* sig_host = nullptr;
  unsigned* sig_dev = nullptr;
  unsigned sig_total = 0, sig_seq = 0;
  // device copy of the tile-pass tables of the last one-qubit run on a large
  // subsystem (rewritten in stream order)
  void* tile_dev = nullptr;
  size_t tile_cap = 0;
  // recycled subsystem buffers of at most kPoolQubits qubits, by qubit count
  static constexpr int kPoolQubits = 20;
  std::vector<void*> pool[kPoolQubits + 1];
  void* mat = nullptr;        // device slot for one gate matrix
  // bookkeeping behind the proposal features (host only, no state sweeps)
  std::vector<double> eps_last, eps_prev;  // last two measured eps (-1: none)
  std::vector<int> rounded_last, tests, gates_since, partner, merged_last;
  int recent[8] = {0};
  int recent_n = 0;
  double recent_eps = -1.0;
  uint64_t gate_count = 0;  // multi-qubit gates applied (or queued) so far
  // learned proposal
  qs_mlp* proposer = nullptr;
  double cutoff = 0.5;
  int propose_flags = 0;         // QS_PROPOSE_*
  int propose_min = 2;           // smallest subsystem scored by the network
  uint64_t deferred = 0;        // dirty qubits skipped on the network's advice
  uint64_t skipped = 0, fallback_tests = 0;
  uint64_t shortcuts = 0;  // operands dropped by the Z-eigenstate shortcut
  // controlled phases and inversions held back between subsystems during one
  // qs_run (the state is these gates applied to the subsystems' ket)
  std::vector<HeldGate> held;
  uint64_t held_in = 0, held_removed = 0;
  // set while the one-qubit gates being applied are already in the host
  // copies of the one-qubit subsystems (qs_run updates them as it queues)
  bool mirrors_ahead = false;
  float* feat_log = nullptr;
  uint64_t feat_cap = 0;
};

// Process-wide: measure several dirty qubits of one subsystem per sweep (1,
// default) or one qubit per sweep (0). Decisions are the same either way.
extern int g_multi_test;
// Process-wide: runs of consecutive one-qubit gates in one launch over the
// small subsystems (1, default) or one launch per gate (0).
extern int g_batch_1q;
// Process-wide: deferred separation in qs_run (1, default) or the tests
// right after every multi-qubit gate (0). Decisions are the same either way.
extern int g_defer_sep;
// Process-wide: one-qubit runs on subsystems of more than 2^12 amplitudes as
// tile passes (1, default) or one launch per gate (0).
extern int g_tile_1q;
// Process-wide: the unobservable shortcuts (1, default): a multi-qubit gate
// whose operand is a one-qubit subsystem in a Z eigenstate that the gate
// keeps is restricted to that value (a controlled gate on |0> disappears, on
// |1> it becomes a gate on the target), so no merge happens; 0: off.
extern int g_unobservable;
// Process-wide: wait for batched sweeps by their completion flag (1, default)
// or by synchronizing the stream (0).
extern int g_done_flag;
// Process-wide: queued operations run in the launch of the sweeps that read
// their results (1, default) or in a launch of their own (0).
extern int g_fuse_ops;
// Process-wide: in qs_run on a factorized state with no separation policy,
// controlled phases and inversions between two subsystems are held back and
// moved past later gates where they commute (one-qubit gates on their target
// conjugate them, so H turns a controlled Z into a controlled X), merging
// only when a gate does not commute or the run ends (1, default); 0: off.
extern int g_hold;
// Process-wide: the kickback shortcut of held gates (fact_kickback; 1,
// default) or not (0), separately from holding them.
extern int g_kickback;

// The 32 proposal features of qubit q (threshold p) from the bookkeeping.
void fact_features(const FactorState* f, int q, double p, float* out);

// All return QS_* status codes and set the thread's error message.
int fact_init(FactorState* f);                     // n one-qubit |0> subsystems
void fact_release(FactorState* f);                 // returns every subsystem buffer
void fact_drain(FactorState* f);                   // frees the recycled buffers too
int fact_set_basis(FactorState* f, uint64_t x);    // n one-qubit basis states
int fact_apply(FactorState* f, const int* qubits, int k, const double* m);
// count one-qubit gates in order: gate i on qubits[i] with the 2x2 matrix
// m + 8 i (interleaved, row-major). Subsystems of at most 2^12 amplitudes get
// one workgroup each in a single launch that applies their gates in order;
// larger subsystems get one launch per gate.
int fact_apply_1q_run(FactorState* f, const int* qubits, const double* m, int count);
// A circuit run: fact_begin_run turns deferred separation on when the
// separation runs after every multi-qubit gate and no dirty qubit is left from
// before; fact_end_run runs the pending tests and turns
// it off. fact_end_run returns rc when it is an error (after the pending tests,
// unless rc is a device error), else its own status.
void fact_begin_run(FactorState* f);
int fact_end_run(FactorState* f, int rc);
// The subsystem holding qubits start .. start+len-1 at consecutive local bits
// t0 .. t0+len-1, in ascending (qubit start at t0) or descending order, with
// len >= 2; -1 if there is none.
int fact_block(const FactorState* f, int start, int len, int* t0, bool* descending);
// Launches whatever is queued (device buffers are then current on the stream).
int fact_sync(FactorState* f);
// Deferred mode: does any of the k qubits lie in a subsystem with tests
// pending? fact_settle runs every pending test.
bool fact_pending_on(const FactorState* f, const int* qubits, int k);
int fact_settle(FactorState* f);
// The Z-eigenstate shortcut on its own: restricts the gate (qubits[0..*k),
// matrix *m) in place and returns true if any operand was dropped; *k = 0
// when nothing is left to apply. Host only.
bool fact_reduce(FactorState* f, int* qubits, int* k, std::vector<double>* m);
// A two-qubit gate (4x4, interleaved, local bit j = qubits[j]) that is a
// controlled gate whose target matrix is M, with its target a known one-qubit
// subsystem in an eigenstate of M (eigenvalue lambda, up to a relative weight
// of 1e-24 off it), acts as diag(1, lambda) on the control alone: restricted
// in place (*k = 1) and true. Host only.
bool fact_kickback(FactorState* f, int* qubits, int* k, std::vector<double>* m);
// Held gates (host only). held_classify: is the 4x4 gate m on (q0, q1) a
// controlled phase or inversion (g set, control taken as q0 where both read
// so)? held_commute: do two held gates commute? held_pass_1q: moves the
// one-qubit gate u on q (a qubit of g) to before g, updating g (u on the
// target conjugates M; on the control u must be diagonal, or g a symmetric
// phase that is re-read with q as target); false (g unchanged) when the
// result is no phase or inversion. held_matrix: the 4x4 on (g.c, g.t).
bool held_classify(const double* m, const int* qubits, HeldGate* g);
bool held_commute(const HeldGate& a, const HeldGate& b);
bool held_pass_1q(HeldGate* g, int q, const double* u);
void held_matrix(const HeldGate& g, double* m);
// Index of the subsystem holding qubit q, or -1.
int fact_sub_of(const FactorState* f, int q);
// Applies a one-qubit gate to the host copy of q's subsystem (when it is a
// known one-qubit subsystem); the device amplitudes are not touched.
void fact_mirror_1q(FactorState* f, int q, const double* m);
int fact_swap(FactorState* f, int a, int b);       // relabel
int fact_relabel(FactorState* f, const int* pos);  // label v -> q where pos[q] = v
int fact_try_separate(FactorState* f, double p, int* n_separated);
// The two-qubit rounding of qubits qa, qb when they share a subsystem of three
// or more qubits (no test otherwise): eps_B = 1 - the largest eigenvalue of
// their reduced density matrix; at eps_B <= p/2 (+ tau) the pair becomes its
// own subsystem (qa at bit 0) and the rest of its old subsystem is dirty.
int fact_test_pair(FactorState* f, int qa, int qb, double p, bool* rounded);
// The pair rounding's host step: the largest eigenvalue and its phase-fixed
// unit eigenvector of the Hermitian part of the 4x4 matrix h (interleaved,
// row-major), by cyclic Jacobi rotations on the 8x8 real embedding.
void fact_hermitian4_top(const double* h, double* lam, double* phi);
int fact_gather(FactorState* f, const uint64_t* idx, uint64_t m, double* out);
int fact_norm(FactorState* f, double* out);
// Dense copy in `dense` (2^n amplitudes of the same precision); perm_out[q]
// receives the bit of qubit q in that copy.
int fact_expand(FactorState* f, void* dense, int* perm_out);
int fact_largest(const FactorState* f);

}  // namespace qs
