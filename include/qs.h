/*
 * qs.h -- C ABI of the MI355X (gfx950) state-vector simulator.
 *
 * The library computes |psi_C> = C |psi_0> for an n-qubit ket stored as 2^n
 * complex amplitudes (Sec. II of the paper: Schroedinger picture, circuits of
 * k-local gates), including the quantum Fourier transform of Eqs. qft/dft, and
 * the approximate mode of Sec. III (factorized ket, one-qubit Schmidt test and
 * SDRP rounding of Eq. sdrp, fidelity model of Eq. fid_model).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Qubit q is bit q of the amplitude index; qubit 0 is the least significant.
 *  - Every call returns an int status: QS_OK (0) or a negative QS_E_* code.
 *    Nothing aborts, throws across the ABI or prints. After an error,
 *    qs_last_error() returns a message for the calling thread.
 *  - Gate calls are asynchronous on the state's stream (qs_set_stream). Calls
 *    that return host data synchronize that stream before returning.
 *  - Host arrays passed in are owned by the caller and are read before the
 *    call returns; host arrays passed out are written before it returns.
 *    Device memory of a state is owned by the state and freed by qs_free.
 *  - Gate matrices are host double arrays, complex interleaved (re, im),
 *    row-major. For a k-qubit matrix, row/column bit j belongs to qubits[j].
 *  - After QS_E_DEVICE (a HIP runtime error) the state is poisoned: every
 *    later call on it except qs_free returns QS_E_DEVICE. A factorized run
 *    that cannot bring its state to a prefix of the circuit poisons it too
 *    (qs_run).
 */
#ifndef QS_H
#define QS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qs_state qs_state;

/* amplitude storage types */
enum { QS_C64 = 1,   /* complex float: interleaved (re, im) float32, 8 B  */
       QS_C128 = 2   /* complex double: interleaved (re, im) float64, 16 B */ };

/* status codes */
enum {
  QS_OK = 0,
  QS_E_INVAL = -1,       /* bad argument: qubit out of range, duplicate qubit,
                            NULL pointer, unknown dtype, k too large,
                            non-finite matrix entry, size mismatch */
  QS_E_NOMEM = -2,       /* device allocation failed; the state is unchanged */
  QS_E_CAPACITY = -3,    /* a merge would exceed the amplitude cap; unchanged */
  QS_E_DEVICE = -4,      /* HIP runtime error (or a poisoned state) */
  QS_E_NUMERIC = -5,     /* norm drift beyond the tolerance given to qs_check */
  QS_E_UNSUPPORTED = -6  /* valid request this build does not serve */
};

#define QS_MAX_QUBITS 34       /* dense states: 2^34 c64 amplitudes = 128 GiB */
#define QS_MAX_FUSED 6         /* largest k of qs_apply_fused */

/* ------------------------------------------------------------ errors */

/* Message of the last failing call on this thread ("" if none). The pointer
 * stays valid until the next failing call on the same thread. */
const char* qs_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int qs_version(void);

/* ------------------------------------------------------------ memory */

/* Device allocator hooks, process-wide. alloc_fn returns device memory of at
 * least `bytes` bytes (256-B aligned) or NULL; free_fn releases it. `user` is
 * passed through. NULL for both restores hipMalloc/hipFree. Must not be
 * changed while any state is alive. */
typedef void* (*qs_alloc_fn)(size_t bytes, void* user);
typedef void (*qs_free_fn)(void* ptr, void* user);
int qs_set_allocator(qs_alloc_fn alloc_fn, qs_free_fn free_fn, void* user);

/* ------------------------------------------------------------ lifecycle */

/* Dense state of n qubits (1 <= n <= QS_MAX_QUBITS) in |0...0>.
 * dtype is QS_C64 or QS_C128. On success *out owns 2^n amplitudes of device
 * memory. QS_E_NOMEM if the allocation fails (then *out is untouched). */
int qs_alloc(int n, int dtype, qs_state** out);

/* Release a state and its device memory (waits for its stream first).
 * NULL is accepted and ignored. */
int qs_free(qs_state* st);

/* Bind the HIP stream (a hipStream_t passed as void*) on which every later
 * kernel of this state is launched. Not owned; NULL means the null stream. */
int qs_set_stream(qs_state* st, void* hip_stream);

/* Wait until all work queued for this state has finished. */
int qs_synchronize(qs_state* st);

/* Number of qubits and storage type of a state. */
int qs_info(const qs_state* st, int* n, int* dtype);

/* ------------------------------------------------------------ initial states */

/* |x>, 0 <= x < 2^n. Clears any pending qubit relabelling. */
int qs_set_basis(qs_state* st, uint64_t x);

/* Upload 2^n amplitudes (count must equal 2^n) from host memory; host_dtype
 * QS_C64 or QS_C128, converted to the state's type on the device. The vector
 * is taken as given (not renormalized). Clears any pending relabelling. */
int qs_set_amplitudes(qs_state* st, const void* host, uint64_t count, int host_dtype);

/* ------------------------------------------------------------ gates (Sec. II) */

/* Any 2x2 matrix m (re00, im00, re01, im01, re10, im10, re11, im11) on qubit q:
 * for every index pair (i, i + 2^q) with bit q of i clear,
 * (a_i, a_{i+2^q}) <- m (a_i, a_{i+2^q}). */
int qs_apply_1q(qs_state* st, int q, const double m[8]);

/* Controlled 2x2: applies m to `target` on the amplitudes whose control bits
 * match: bit j of ctrl_values is the required value of ctrls[j] (1 = control,
 * 0 = anti-control, the "A" couplers of Sec. III-C). 1 <= nctrl <= 8. */
int qs_apply_ctrl(qs_state* st, const int* ctrls, int nctrl, uint64_t ctrl_values,
                  int target, const double m[8]);

/* Controlled phase: multiplies every amplitude with bits a and b both set by
 * e^{i theta} (the controlled R_Z-type phase of the QFT circuit, Sec. II-E). */
int qs_apply_cphase(qs_state* st, int a, int b, double theta);

/* SWAP of qubits a and b in O(1) by exchanging their labels (a constant-cost
 * SWAP, Table I). Amplitudes are moved only when a later call
 * needs the identity labelling (readout, QFT on a permuted range). */
int qs_apply_swap(qs_state* st, int a, int b);

/* Dense k-qubit block (1 <= k <= QS_MAX_FUSED): m is 2^k x 2^k complex
 * (2*4^k doubles), row/column bit j <-> qubits[j]. For every assignment of the
 * other n-k bits, the 2^k amplitudes that differ only in `qubits` are
 * multiplied by m. Blocks of 4 or 5 qubits run on the matrix cores
 * ("fused.mfma": FP32 for complex64, FP64 for complex128) once the state
 * holds a full tile (2^k x 128 amplitudes in complex64, 2^k x 64 in
 * complex128, more when the block has low bits); other widths and smaller
 * states on vector FMA. */
int qs_apply_fused(qs_state* st, const int* qubits, int k, const double* m);

/* A named gate (QS_GATE_* below) built in float64 inside the library and
 * applied with the calls above: one-qubit kinds with qs_apply_1q, CP and CZ
 * with qs_apply_cphase (CZ = CP(pi)), SWAP as a relabelling, iSWAP as a
 * two-qubit block, CX/CY/AX/AY/AZ as qs_apply_ctrl with one control
 * (qubits = {control, target}). QS_GATE_CU3 takes nq - 1 controls then the
 * target (2 <= nq <= 9) and params = {theta, phi, lambda, v}, v a mask of
 * the required control values (bit j for qubits[j]; v = 1 is a plain control
 * when nq = 2). params: U3 {theta, phi, lambda} (Sec. III-C), CP {theta},
 * else unused (may be NULL). QS_E_INVAL for an unknown kind, a wrong qubit
 * count, a repeated or out-of-range qubit, or a missing or non-finite
 * parameter, before any device work. */
int qs_apply_gate(qs_state* st, int kind, const int* qubits, int nq, const double* params);

/* Quantum Fourier transform (Eq. dft, omega = e^{+2 pi i / N}) on qubits
 * start .. start+len-1, including the final bit reversal (done as a
 * relabelling). inverse != 0 applies the inverse transform. Dense states run
 * multi-stage passes; factorized states run the QFT circuit gate by gate
 * (H, then the controlled phases of each stage, then the reversing SWAPs as
 * relabels; the inverse reversed with negated angles) under the state's
 * separation policy, where the Z-eigenstate shortcut keeps a basis input a
 * product state. */
int qs_qft(qs_state* st, int start, int len, int inverse);

/* ------------------------------------------------------------ approximate mode (Sec. III) */

/* A factorized state keeps the ket as a tensor product of kets on disjoint
 * qubit subsets, split as far as the state allows (Sec. II-A). Each subsystem is a
 * separate device buffer of 2^k amplitudes. A gate on qubits of different
 * subsystems first merges them (Kronecker product; the first operand's qubits
 * keep their bit positions). The one-qubit Schmidt test (Sec. III-A) computes
 * the Bloch vector r of a qubit's reduced state in float64, eps = (1-|r|)/2,
 * and, when eps <= p/2 (Eq. sdrp, plus a tolerance of 1e-6 for complex64 /
 * 1e-12 for complex128: exact separability tested to within rounding, Sec. III-A),
 * projects the qubit on the dominant eigenvector phi of its reduced state,
 * moves it into a one-qubit subsystem and multiplies the fidelity estimate by
 * 1 - eps (Eq. fid_model). */

/* separation policies */
enum { QS_SEP_NONE = 0,           /* only explicit qs_try_separate calls */
       QS_SEP_AFTER_2Q = 1,       /* after every multi-qubit gate */
       QS_SEP_AFTER_2Q_PAIRS = 2  /* as 1, then the two-qubit rounding of the
                                     operands of every two-qubit gate */ };

/* one separability attempt */
typedef struct {
  int32_t qubit;     /* tested qubit (the first of a pair) */
  int32_t n_sub;     /* qubits in its subsystem when tested */
  double eps;        /* (1 - |r|)/2, or 1 - lambda_max for a pair (float64) */
  int32_t rounded;   /* 1 if the qubit (pair) was separated */
  int32_t pair;      /* 0: one-qubit attempt; else 1 + the pair's second qubit */
  uint64_t gates;    /* multi-qubit gates applied to the state before this test:
                        the test sees the state after that many of them (its
                        place in the circuit, whether it ran at once or later
                        in a deferred flush) */
} qs_attempt;

/* Factorized state of n qubits (1 <= n <= 63), every qubit its own |0>
 * subsystem. A merge that would exceed max_amps amplitudes returns
 * QS_E_CAPACITY and leaves the state unchanged. */
int qs_alloc_factorized(int n, int dtype, uint64_t max_amps, qs_state** out);

/* Policy and threshold p (0 <= p <= 1) applied after gates. */
int qs_set_separation_policy(qs_state* st, int policy, double p);

/* Test the dirty qubits (those whose reduced state may have changed: both
 * operands of every multi-qubit gate since their last test, and the other
 * members of a subsystem that lost a qubit), lowest index first, until none
 * is dirty. *n_separated receives the number of roundings. No-op on dense
 * states. Synchronizes (each decision reads the statistics back). */
int qs_try_separate(qs_state* st, double p, int* n_separated);

/* Two-qubit rounding (Sec. III-A mentions the generalization of the rounding
 * to two-qubit subsystems without a rule; this is the reading used): when qa
 * and qb share a subsystem S of three or more qubits, rho_B is their 4x4
 * reduced density matrix (float64 sums, index m = bit of qa + 2 bit of qb),
 * eps_B = 1 - its largest eigenvalue (host Jacobi, float64). At eps_B <= p/2
 * (+ the same tolerance as above) S is projected on the dominant eigenvector
 * phi, the pair becomes a subsystem of its own (qa at bit 0, amplitudes phi),
 * the rest of S is marked dirty and F is multiplied by 1 - eps_B; *rounded
 * is set to 1. Qubits in different subsystems, or a subsystem of two qubits:
 * no test, *rounded = 0. The attempt is logged with pair = 1 + qb. QS_E_INVAL
 * on a dense state, equal or out-of-range qubits. Synchronizes. */
int qs_try_separate_pair(qs_state* st, int qa, int qb, double p, int* rounded);

/* The host step of the pair rounding, on its own (no device work): the
 * largest eigenvalue *lambda of the Hermitian part (h + h^H)/2 of the 4x4
 * complex matrix h (32 doubles, interleaved, row-major) and its unit
 * eigenvector phi (8 doubles, interleaved), phase-fixed so that its first
 * component of magnitude above 1e-9 of the largest is real and positive;
 * cyclic Jacobi rotations on the 8x8 real embedding, float64. QS_E_INVAL for
 * NULL pointers or non-finite entries. */
int qs_hermitian4_top(const double* h, double* lambda, double* phi);

/* Mark qubits (bit q of mask) dirty, e.g. to test a state built elsewhere. */
int qs_mark_dirty(qs_state* st, uint64_t mask);

/* Fidelity estimate F = prod (1 - eps_j) over all roundings so far
 * (Eq. fid_model); 1.0 for dense states. */
int qs_fidelity_estimate(const qs_state* st, double* F);

/* Subsystem table: qubit_to_sub[q] (n entries) and sizes[s] (up to n
 * entries) may be NULL; *nsub receives the number of subsystems. */
int qs_subsystems(const qs_state* st, int* qubit_to_sub, int* sizes, int* nsub);
/* Qubits of subsystem s in bit order (qubits[t] is stored at bit t). */
int qs_subsystem_qubits(const qs_state* st, int s, int* qubits, int* nq);

/* Record every attempt into a caller-owned array of cap entries; *count
 * counts all attempts (it can exceed cap; entries beyond cap are dropped).
 * NULL/NULL stops recording. The array must outlive the recording. */
int qs_set_attempt_log(qs_state* st, qs_attempt* buf, uint64_t cap, uint64_t* count);

/* Write the full ket of a factorized state into a dense state of the same
 * width and precision (its labels are set so that readouts are in qubit
 * order). */
int qs_expand(qs_state* factorized, qs_state* dense);

/* <a|b> of two dense states of equal width and precision, float64
 * accumulation in a fixed order (for Eq. fid_exact). Synchronizes. */
int qs_inner_product(qs_state* a, qs_state* b, double* re, double* im);

/* ------------------------------------------------------------ learned proposal */

/* A small network scores which dirty qubits to test: 32 features per qubit
 * -> 64 (tanh) -> 64 (tanh) -> 1 logit, score = sigmoid(logit), float32 on
 * the GPU. Parameters: W1[32][64], b1[64], W2[64][64], b2[64], W3[64], b3,
 * row-major with x @ W + b (6,337 floats). Training minimizes the mean
 * binary cross-entropy with Adam, on the GPU. */
#define QS_MLP_INPUTS 32
#define QS_MLP_PARAMS 6337
typedef struct qs_mlp qs_mlp;
typedef struct {
  uint32_t steps;   /* Adam steps */
  uint32_t batch;   /* rows per step (0 = 256); consecutive rows, wrapping */
  float lr, beta1, beta2, eps;
} qs_train_cfg;

int qs_mlp_create(qs_mlp** out);  /* all parameters zero */
int qs_mlp_free(qs_mlp* net);
int qs_mlp_set_stream(qs_mlp* net, void* hip_stream);
int qs_mlp_set_params(qs_mlp* net, const float* host, uint64_t count);
int qs_mlp_get_params(qs_mlp* net, float* host, uint64_t count);
/* scores[r] = sigmoid(logit of row r of X (rows x 32)). Synchronizes. */
int qs_mlp_forward(qs_mlp* net, const float* X, uint64_t rows, float* scores);
/* Gradient of the mean cross-entropy of (X, y) w.r.t. the parameters (same
 * layout as the parameters) and the loss. Synchronizes. */
int qs_mlp_grad(qs_mlp* net, const float* X, const float* y, uint64_t rows, float* grad,
                double* loss);
/* cfg->steps Adam steps on minibatches of consecutive rows (the caller
 * shuffles); *final_loss = mean loss over all rows afterwards. */
int qs_mlp_train(qs_mlp* net, const float* X, const float* y, uint64_t rows,
                 const qs_train_cfg* cfg, double* final_loss);

/* Use `net` to choose which dirty qubits of a factorized state to test: every
 * dirty qubit of a subsystem with at least cfg->min_qubits qubits is scored
 * from its features (qs_features layout) and only those scoring >=
 * cfg->cutoff get the exact Schmidt test, which alone decides any rounding
 * (the fidelity estimate keeps the plain rule); smaller subsystems keep the
 * plain schedule, since their exact test costs no more than a proposal.
 * Skipped qubits are deferred; before a merge that would exceed the
 * amplitude cap, every deferred qubit gets the exact test. With
 * QS_PROPOSE_RETEST_ON_MERGE in cfg->flags, the deferred qubits of the
 * subsystems a gate is about to merge are tested first, so a skipped
 * rounding cannot make a merged subsystem larger than it has to be.
 * net = NULL restores the plain schedule (cfg is then ignored). The network
 * must outlive its use; cfg is copied. */
#define QS_PROPOSE_RETEST_ON_MERGE 1
typedef struct qs_propose_cfg {
  double cutoff;      /* score threshold in [0, 1] */
  int32_t flags;      /* QS_PROPOSE_* */
  int32_t min_qubits; /* smallest subsystem whose qubits are scored, >= 2 */
} qs_propose_cfg;
int qs_set_proposer(qs_state* st, qs_mlp* net, const qs_propose_cfg* cfg);

/* Features recorded with each attempt (rows of QS_MLP_INPUTS floats aligned
 * with the attempt log): caller-owned buffer of cap rows; NULL stops. */
int qs_set_feature_log(qs_state* st, float* buf, uint64_t cap);

/* Number of exact tests skipped on the network's advice and of deferred
 * qubits tested by the capacity fallback, since the state was created. */
int qs_proposer_stats(const qs_state* st, uint64_t* skipped, uint64_t* fallback_tests);

/* Unobservable shortcut (Sec. II-B, "factor.unobservable"): a multi-qubit
 * gate on a factorized state whose operand is a one-qubit subsystem in a Z
 * eigenstate (a float64 host copy of its amplitudes puts at most 1e-24 of the
 * weight on the other basis state) that the gate keeps (every matrix entry
 * from that value to the other is exactly zero) is restricted to that value:
 * a controlled gate on |0> disappears, on |1> it acts on its target alone, a
 * controlled phase becomes a phase gate; no merge happens and no test is
 * due. *count receives the number of operands dropped so far. */
int qs_shortcut_count(const qs_state* st, uint64_t* count);

/* Held gates (Table I: controlled phases and inversions buffered and moved
 * around H; "factor.hold"). In qs_run on a factorized state with no
 * separation policy, a two-qubit gate that is a controlled phase (control 1:
 * diag(d0, d1) on the target) or inversion ([[0, d0], [d1, 0]]) between two
 * subsystems is held back instead of merging them. The state is the held
 * gates applied to the subsystems' ket; held gates commute with each other.
 * A later one-qubit gate on a held gate's target conjugates its matrix (H
 * turns a controlled Z into a controlled X), a diagonal one on its control
 * passes, a phase with d0 = 1 is symmetric; two held gates on the same
 * control and target (or two such phases on one pair, either way round)
 * multiply (a controlled Z twice cancels). A gate that
 * does not commute applies the held gate first, as does the end of the run;
 * a held gate is applied with the Z-eigenstate shortcut and with the
 * kickback shortcut: a controlled M whose target is a one-qubit subsystem in
 * an eigenstate of M (eigenvalue l, at most 1e-24 of the weight off it)
 * acts as diag(1, l) on its control (a controlled X onto |->: a Z on the
 * control). Entries within 1e-13 of zero or one are taken as such when
 * products are classified. The result is the circuit's state (to that
 * rounding). *held receives the gates held so far, *removed those that never
 * caused a merge of their own (folded, cancelled or reduced to one qubit). */
int qs_held_count(const qs_state* st, uint64_t* held, uint64_t* removed);

/* ------------------------------------------------------------ circuits */

/* A circuit is a host-side gate list on n qubits that is fused into dense
 * blocks of at most kmax qubits and run with one sweep per block. SWAP gates
 * are kept as a renaming of the positions the later gates act on and end up in
 * the state's labels (no data movement). */
typedef struct qs_circuit qs_circuit;

/* named gate kinds for qs_circuit_add_gate; two-qubit controlled kinds take
 * qubits = {control, target}; the "A" kinds act when the control is |0>
 * (the anti-controlled couplers of Sec. III-C) */
enum {
  QS_GATE_H = 1, QS_GATE_X = 2, QS_GATE_Y = 3, QS_GATE_Z = 4,
  QS_GATE_U3 = 5,     /* params = {theta, phi, lambda}: U of Sec. III-C */
  QS_GATE_CZ = 6, QS_GATE_ISWAP = 7,
  QS_GATE_CP = 8,     /* params = {theta}: e^{i theta} on |11> */
  QS_GATE_SWAP = 9, QS_GATE_CX = 10, QS_GATE_CY = 11,
  QS_GATE_AX = 12, QS_GATE_AY = 13, QS_GATE_AZ = 14,
  QS_GATE_CU3 = 15    /* qubits {control, target}, params = {theta, phi, lambda,
                         v}: U3 on the target when the control equals v (1, or
                         0 for an anti-control), identity otherwise */
};

/* Empty circuit on n qubits (1 <= n <= 64). */
int qs_circuit_create(int n, qs_circuit** out);
/* Release a circuit (waits for the device if its matrices are in use). */
int qs_circuit_free(qs_circuit* c);
/* Append a named gate; its matrix is built in float64. QS_E_INVAL for an
 * unknown kind, a qubit out of range or repeated, missing or non-finite
 * parameters. Invalidates an earlier plan. */
int qs_circuit_add_gate(qs_circuit* c, int kind, const int* qubits, const double* params);
/* Append a dense k-qubit matrix (1 <= k <= QS_MAX_FUSED), layout as in
 * qs_apply_fused. */
int qs_circuit_add_matrix(qs_circuit* c, const int* qubits, int k, const double* m);
/* Fuse the gate list into blocks of at most kmax qubits (1..QS_MAX_FUSED;
 * 0 = 5). Gates in order; a gate joins the open blocks it touches when their
 * union has at most kmax qubits, otherwise those blocks are closed. Block
 * matrices are products of the gates in float64. Called before any
 * qs_circuit_use_tiles, it also makes dense runs use these blocks. */
int qs_circuit_plan(qs_circuit* c, int kmax);

/* Run this circuit on dense states as tile passes (on != 0) or as fused
 * blocks (on = 0). Without either call, or qs_circuit_plan before it, dense
 * runs use tile passes: on MI355X they took 0.49-0.92 of the blocks' time
 * for random circuits of 1 to 10 layers at 20 and 30 qubits, and 0.53 at 32
 * qubits and 10 layers. A pass reads and writes the ket once for every one- and
 * two-qubit gate it holds: a tile is the contiguous low bits (complex64:
 * "tile.low_bits", 5 by default; complex128: 4) plus 7 bits chosen per pass, and the passes
 * are planned on the state's physical bits at the first run (re-planned when
 * the state's labelling differs). Gates too wide for a round (more than 4
 * qubits with "tile.mfma" on, more than 2 otherwise or for complex128) run
 * as dense blocks between passes. States with fewer qubits than a tile (its
 * low bits + 7) use fused blocks. Same results as the block path up to float rounding order. */
int qs_circuit_use_tiles(qs_circuit* c, int on);
/* Tile plan of the circuit for a state in the identity labelling (current
 * "tile.*" knobs): passes,
 * dense blocks and register rounds (any pointer may be NULL).
 * QS_E_UNSUPPORTED if the circuit has fewer qubits than a tile. */
int qs_circuit_tile_info(const qs_circuit* c, int dtype, int* passes, int* blocks, int* rounds);
/* Gate count, block count (-1 before planning) and widest block. */
int qs_circuit_info(const qs_circuit* c, int* ngates, int* nblocks, int* max_k);
/* Block i of a planned circuit: its width, its positions (position p = qubit p
 * before any SWAP of the circuit) and, if m != NULL, its 2^k x 2^k matrix
 * (2*4^k doubles, layout as in qs_apply_fused). */
int qs_circuit_block(const qs_circuit* c, int i, int* k, int* qubits, double* m);
/* Apply a circuit to a state of the same width: tile passes or blocks as
 * qs_circuit_use_tiles describes (blocks planned first if needed).
 * Block matrices are uploaded once per precision and kept with the circuit.
 * Blocks of 4-5 qubits run on the matrix cores. A factorized state
 * takes the gates one by one under its separation policy (see
 * qs_held_count for the gates an exact run holds back); when a gate fails
 * there (QS_E_CAPACITY: a merge past the state's cap), the gates before it
 * are applied, the gates still held back among them included, so the state
 * is that prefix of the circuit; if a held gate cannot be applied either, the
 * handle is left unusable (every later call but qs_free returns
 * QS_E_DEVICE). */
int qs_run(qs_state* st, qs_circuit* c);

/* ------------------------------------------------------------ batches */

/* Many independent small kets in one device arena, each starting in |0...0>.
 * A batched run applies one circuit per ket pass by pass: pass p applies the
 * p-th fused block of every circuit, with one launch per distinct block width
 * for the whole batch. */
typedef struct qs_batch qs_batch;

/* count kets of n_each[i] qubits (1..30), dtype QS_C64 or QS_C128. */
int qs_batch_create(int count, const int* n_each, int dtype, qs_batch** out);
int qs_batch_free(qs_batch* b);
/* Stream of every later launch (not owned; NULL = null stream). */
int qs_batch_set_stream(qs_batch* b, void* hip_stream);
/* Every ket back to |0...0> (two kernels, no memset: safe to mix with graph
 * replays). */
int qs_batch_reset(qs_batch* b);
/* Run circuits[i] on ket i (asynchronous). Circuits are planned with block
 * width kmax (1..5; 0 = 4) and may not contain SWAP gates. The work tables
 * and block matrices are uploaded before the launches. */
int qs_batch_run(qs_batch* b, qs_circuit* const* circuits, int kmax);
/* Record the launches of such a run into a HIP graph on the batch's stream
 * (must not be the null stream) without running them; qs_batch_replay then
 * launches the graph. The graph is kept until the next run or capture. */
int qs_batch_capture(qs_batch* b, qs_circuit* const* circuits, int kmax);
int qs_batch_replay(qs_batch* b);
/* on != 0 (the default): complex64 kets of at least 12 qubits run their
 * circuits as tile passes (as qs_circuit_use_tiles, tiles of 5 low + 7 chosen
 * bits, dense 4-qubit rounds on the matrix cores), batched as one launch per
 * pass index over every ket that has that pass; other kets (fewer qubits,
 * complex128, gates of more than 4 qubits) keep the block launches (1024
 * circuits of 12-20 qubits: 12.0-12.4 ms against 27.4 ms with blocks
 * only). on = 0: blocks for every ket. Drops a prepared run or graph;
 * applies to the next run or capture. */
int qs_batch_use_tiles(qs_batch* b, int on);
/* Launches per run of the last prepared run and arena size in amplitudes. */
int qs_batch_info(const qs_batch* b, int* launches, uint64_t* total_amps);
/* The 2^n_i amplitudes of ket i (out_dtype must be the batch's). Synchronizes. */
int qs_batch_amplitudes(qs_batch* b, int i, void* host_out, uint64_t count, int out_dtype);
int qs_batch_synchronize(qs_batch* b);

/* ------------------------------------------------------------ readout */

/* All 2^n amplitudes in index order (relabelling undone), converted to
 * out_dtype (QS_C64 or QS_C128). count must equal 2^n. Synchronizes. */
int qs_amplitudes(qs_state* st, void* host_out, uint64_t count, int out_dtype);

/* Amplitudes at m indices (each < 2^n) as complex double, interleaved
 * (2*m doubles). Synchronizes. */
int qs_amplitudes_gather(qs_state* st, const uint64_t* idx, uint64_t m, double* out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture that must not call hipMalloc, tight serving loops, harnesses that
 * forbid allocation): qs_amplitudes_gather on a dense state without any
 * allocation. The index list and the outputs are staged in a fixed
 * device-side array of the library (QS_GATHER_NOALLOC_MAX entries: 1.5 MiB
 * per GPU, held until the process ends), not in memory allocated per call.
 * m > QS_GATHER_NOALLOC_MAX gives QS_E_INVAL; a factorized state gives
 * QS_E_UNSUPPORTED (use qs_amplitudes_gather). Same output and argument
 * rules as qs_amplitudes_gather; synchronizes. Every call on one GPU shares
 * that staging array, so calls that overlap on one GPU (from several host
 * threads or streams) race: the caller serializes them. */
#define QS_GATHER_NOALLOC_MAX 65536
int qs_amplitudes_gather_noalloc(qs_state* st, const uint64_t* idx, uint64_t m, double* out);

/* |a_x|^2 for every x in index order, accumulated in float64. count = 2^n.
 * Synchronizes. */
int qs_probs(qs_state* st, double* out, uint64_t count);

/* Squared norm sum |a_x|^2, accumulated in float64 in a fixed reduction order
 * (bitwise repeatable). Synchronizes. */
int qs_norm(qs_state* st, double* out);

/* QS_E_NUMERIC if |norm - 1| > tol, else QS_OK. Synchronizes. */
int qs_check(qs_state* st, double tol);

/* ------------------------------------------------------------ tuning */

/* Process-wide knobs of the kernel planners (read by later calls):
 *   "qft.lds_bits"   bits of the contiguous LDS tile of the QFT's low pass:
 *                    1 to 13 for complex64 / 12 for complex128 (larger
 *                    values are clamped to that); 0 (default): 12, or 11
 *                    for complex64 states above 256 MiB when that adds no
 *                    pass;
 *   "qft.stream"     global accesses of the LDS tile passes: 0 (default)
 *                    streaming (non-temporal) for states above 256 MiB, plain
 *                    below (such states partly stay in the last-level
 *                    cache between passes); 1 always streaming; 2 never;
 *   "gate.shuffle_bits" complex64 one-qubit gates on bits 1 .. this value (at
 *                    most 6; default 6) hold contiguous amplitudes per lane and
 *                    exchange the partners (target bit flipped) by wavefront
 *                    shuffles; 0: strided pairs for every bit above 0. Same
 *                    results bit for bit;
 *   "gate.dense_ctrl" 1 (default): a singly controlled complex64 gate whose
 *                    control is on bit 0, 1 or 2 sweeps the whole state (as a
 *                    one-qubit gate on the target, the matrix applied where the
 *                    control matches); 0: only the half it changes. Same
 *                    results bit for bit;
 *   "sweep.stream"   global accesses of the gate sweeps, fused blocks and
 *                    tile passes: 0 (default) streaming (non-temporal) for
 *                    states above 256 MiB when every wave access covers
 *                    contiguous runs of at least 64 bytes (the lowest bit
 *                    the sweep fixes is high enough), plain otherwise; 1
 *                    always streaming; 2 never. Results are the same either
 *                    way, bit for bit;
 *   "qft.high_pass"  passes above that tile: 0 = strided LDS tiles, 1 =
 *                    register passes of up to 5 bits;
 *   "qft.col_max"    most bits of one strided LDS pass: 8 (default; 256-byte
 *                    rows) or 7 (512-byte rows), both 64 KiB tiles; a 7-bit
 *                    complex64 pass always has 512-byte rows unless
 *                    qft.col_rows = 1 (complex128 ones have 256-byte rows);
 *   "qft.col_rows"   1: strided passes of 7 bits use 256-byte rows (32 KiB
 *                    tiles); 2: also complex64 passes of 8 bits use 128-byte
 *                    rows (32 KiB); 0 (default): 512-byte rows for 7 bits
 *                    (complex128: 256), 256-byte rows for 8;
 *   "qft.threads"    thread cap of the LDS tile launches: 256, 512, or 0
 *                    (default: 512 for strided passes of 8 bits, 256 for
 *                    the others);
 *   "qft.round_bits" widest in-register round inside an LDS tile: 4 (default)
 *                    or 5 (complex64 only);
 *   "tile.low_bits"  contiguous low bits of a complex64 tile: 5 (default,
 *                    256-byte rows, 32 KiB tiles, four workgroups per CU),
 *                    6 (512-byte rows, 64 KiB) or 4 (128-byte rows, 16 KiB);
 *                    complex128 tiles always have 16-amplitude (256-byte)
 *                    rows, 32 KiB;
 *   "tile.mfma"      1 (default): complex64 tile passes run their rounds as
 *                    dense 4-qubit blocks on the matrix cores (any gate of at
 *                    most 4 qubits joins a pass); 0: one- and two-qubit gates
 *                    applied one by one in registers;
 *   "factor.multi_test" 1 (default): the plain separability schedule
 *                    measures the lowest dirty qubit together with the next
 *                    dirty qubits of its subsystem (up to 5, none skipped) in
 *                    one sweep; 0: one sweep per qubit. Same decisions;
 *   "factor.fuse_ops" 1 (default): queued merges and projections run in the
 *                    launch of the sweeps that read their results (each in
 *                    the workgroup that then sweeps its output); 0: in a
 *                    launch of their own first;
 *   "factor.done_flag" 1 (default): a round of batched sweeps of small
 *                    subsystems is waited for by a completion flag its last
 *                    workgroup writes to mapped host memory; 0: by a stream
 *                    synchronization;
 *   "factor.kernarg_tables" 1 (default): the tables of the batched launches
 *                    of the factorized mode (sweeps, merges, projections,
 *                    one-qubit runs) travel in the kernel arguments when they
 *                    fit; 0: always read from mapped host memory;
 *   "factor.unobservable" 1 (default): the Z-eigenstate shortcut described at
 *                    qs_shortcut_count; 0: every gate merges its operands;
 *   "factor.defer"   1 (default): in qs_run on a factorized state with the
 *                    plain schedule after every multi-qubit gate (no
 *                    proposer, no feature log), the tests due after a gate
 *                    wait until a later gate touches that subsystem or the
 *                    run ends; pending tests of many subsystems share one
 *                    launch and one synchronization. Decisions, the attempt
 *                    log order and F are those of testing at once; 0: test
 *                    right after every gate;
 *   "factor.tile_1q" 1 (default): in those runs, the one-qubit gates on a
 *                    subsystem of 2^13 amplitudes or more run as tile passes
 *                    (a few sweeps for all of them); 0: one sweep per gate;
 *   "factor.batch_1q" 1 (default): qs_run on a factorized state applies each
 *                    run of consecutive one-qubit gates in one launch over
 *                    the subsystems of at most 2^12 amplitudes (one
 *                    workgroup per subsystem); 0: one launch per gate;
 *   "factor.hold"    1 (default): the held gates described at qs_held_count;
 *                    0: every such gate merges its operands at once;
 *   "factor.kickback" 1 (default): a held gate whose target is a one-qubit
 *                    subsystem in an eigenstate of its matrix acts on its
 *                    control alone (qs_held_count); 0: off;
 *   "fused.mfma"     1 (default): blocks of 4 or 5 qubits run on the matrix
 *                    cores (FP32 for complex64, FP64 for complex128) when
 *                    their geometry fits; 0: vector FMA.
 * QS_E_INVAL for an unknown key or a value out of range. */
int qs_tune_set(const char* key, int64_t value);
int qs_tune_get(const char* key, int64_t* value);

/* ------------------------------------------------------------ timing */

/* Aggregated timing of one kernel kind between qs_profile_start and
 * qs_profile_stop: number of launches, summed duration measured with HIP
 * events on the state's stream, and summed algorithmic bytes (the bytes the
 * operation must read plus write: 2 * 2^n amplitudes for a full sweep). */
typedef struct {
  char name[48];
  uint64_t launches;
  double total_ms;
  double bytes;
} qs_kernel_stat;

/* Start recording every kernel launch of this state (synchronizes first;
 * discards earlier records). Adds two event records per launch. */
int qs_profile_start(qs_state* st);

/* Stop recording, synchronize, and aggregate per kernel kind into out
 * (at most max_out kinds, in first-launch order); *count receives the number
 * of kinds written. */
int qs_profile_stop(qs_state* st, qs_kernel_stat* out, int max_out, int* count);

#ifdef __cplusplus
}
#endif

#endif /* QS_H */
