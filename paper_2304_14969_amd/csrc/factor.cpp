// Approximate mode of Sec. III on the GPU: a ket kept as a product of
// subsystems (Sec. II-A), the one-qubit Schmidt test through the Bloch vector
// and the SDRP rounding of Eq. sdrp, with the fidelity model of Eq. fid_model.
//
// Host side: the subsystem table, the dirty-qubit schedule and the decisions
// (float64). Device side: every pass over amplitudes (compose, gate sweeps,
// Bloch statistics in float64, projection).
//
// Readings of the paper used here:
//  * rounding condition: inclusive eps <= p/2 (Eq. sdrp), plus a tolerance tau
//    that lets exact separability be tested to within rounding, Sec. III-A
//    (1e-6 for complex64 amplitudes,
//    whose eps carries ~1e-7 rounding error; 1e-12 for complex128);
//  * the projection keeps the dominant eigenvector phi of rho_q (the result of
//    rotating r to the |0> pole, post-selecting and rotating back), with phi_0
//    real and >= 0, phi = |0> when r = 0; the remainder is renormalized with
//    the weight (1 + |r|)/2 of the kept branch;
//  * schedule: after a multi-qubit gate both operands are dirty; a rounding
//    makes every other member of its subsystem dirty; the lowest-numbered
//    dirty qubit is tested until none is left (no other reduced state can
//    have changed);
//  * merge of subsystems A (first operand's) and B: c[iA + 2^nA iB] = a b.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "circuit.h"
#include "factor.h"
#include "mlp.h"
#include "qs_internal.h"

namespace qs {

int g_multi_test = 1;
int g_batch_1q = 1;
int g_defer_sep = 1;
int g_tile_1q = 1;
int g_unobservable = 1;
int g_kernarg_tables = 1;
int g_done_flag = 1;
int g_fuse_ops = 1;
int g_hold = 1;
int g_kickback = 1;

void* device_alloc(size_t bytes);
void device_free(void* p);
void set_last_error(const char* msg);
void note_test_impl(FactorState* f, int q, double eps, bool rounded);

namespace {

int ffail(int code, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return code;
}

int dev_err(hipError_t e, const char* what) {
  if (e == hipSuccess) return QS_OK;
  return ffail(QS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t amp_bytes(const FactorState* f) { return f->dtype == QS_C64 ? 8 : 16; }

constexpr int kMultiTest = 5;  // qubits per multi-qubit Bloch sweep
// most items of one sweep round (the stat buffer holds 4 sums per target)
constexpr int kMaxSweepItems = FactorState::kStatDoubles / (4 * kMultiTest);

int flush_pending(FactorState* f);
int ring_slot(FactorState* f, void** host, void** dev);
int launch_queue(FactorState* f);
void finish_queue(FactorState* f);
template <typename R>
void fill_op(const FactorState::QOp& q, FactOp<R>* o);

// Does any of the k qubits lie in a subsystem with dirty qubits?
bool touches_dirty(const FactorState* f, const int* qubits, int k);

// Upload a small host vector of complex doubles as the state's precision.
hipError_t upload(const FactorState* f, void* dst, const double* re_im, size_t count) {
  if (f->dtype == QS_C64) {
    std::vector<float> h(2 * count);
    for (size_t i = 0; i < 2 * count; ++i) h[i] = float(re_im[i]);
    return hipMemcpyAsync(dst, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice,
                          f->stream);
  }
  return hipMemcpyAsync(dst, re_im, 2 * count * sizeof(double), hipMemcpyHostToDevice, f->stream);
}

int find(const FactorState* f, int q, int* t) {
  for (int s = 0; s < int(f->subs.size()); ++s)
    for (int b = 0; b < f->subs[s].nq; ++b)
      if (f->subs[s].q[b] == q) {
        if (t) *t = b;
        return s;
      }
  return -1;
}

// Subsystem buffers: small ones are recycled through the state's pool (work
// on a state is ordered on its stream, so a returned buffer can be handed out
// again at once); larger ones go back to the allocator.
void* sub_alloc(FactorState* f, int nq) {
  if (nq <= FactorState::kPoolQubits && !f->pool[nq].empty()) {
    void* p = f->pool[nq].back();
    f->pool[nq].pop_back();
    return p;
  }
  return device_alloc((size_t(1) << nq) * amp_bytes(f));
}

void sub_free(FactorState* f, int nq, void* p) {
  if (!p) return;
  if (!f->qops.empty()) {  // a queued operation may still read it
    f->late_free.push_back({nq, p});
    return;
  }
  if (nq <= FactorState::kPoolQubits) {
    f->pool[nq].push_back(p);
    return;
  }
  device_free(p);
}

int new_single(FactorState* f, int q, const double amp[4], Sub* out) {
  Sub s;
  s.nq = 1;
  s.q[0] = q;
  s.known = true;
  for (int i = 0; i < 4; ++i) s.h[i] = amp[i];
  s.amps = sub_alloc(f, 1);
  if (!s.amps) return ffail(QS_E_NOMEM, "allocating a one-qubit subsystem");
  const hipError_t e = f->dtype == QS_C64
                           ? launch_store_single(static_cast<float*>(s.amps), amp, f->stream)
                           : launch_store_single(static_cast<double*>(s.amps), amp, f->stream);
  if (int rc = dev_err(e, "one-qubit subsystem")) {
    sub_free(f, 1, s.amps);
    return rc;
  }
  *out = s;
  return QS_OK;
}

void log_attempt(FactorState* f, int q, int nsub, double eps, bool rounded, int partner,
                 uint64_t gates) {
  if (!f->log || !f->log_count) return;
  if (*f->log_count < f->log_cap) {
    qs_attempt& a = f->log[*f->log_count];
    a.qubit = q;
    a.n_sub = nsub;
    a.eps = eps;
    a.rounded = rounded ? 1 : 0;
    a.pair = partner + 1;
    a.gates = gates;
  }
  ++*f->log_count;
}

// Eigen-decomposition of a real symmetric 8x8 matrix by cyclic Jacobi
// rotations (float64): w[k] and column k of V. Used on the real embedding
// [[Re H, -Im H], [Im H, Re H]] of a 4x4 Hermitian H, whose spectrum is H's
// with every eigenvalue twice; an eigenvector (x; y) gives H (x + i y) =
// lambda (x + i y).
void jacobi8(double A[8][8], double w[8], double V[8][8]) {
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) V[i][j] = i == j ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < 8; ++i)
      for (int j = 0; j < 8; ++j) {
        tot += A[i][j] * A[i][j];
        if (i != j) off += A[i][j] * A[i][j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < 7; ++p)
      for (int q = p + 1; q < 8; ++q) {
        if (A[p][q] == 0.0) continue;
        // rotation that zeroes A[p][q] (the smaller-angle root)
        const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 8; ++k) {  // columns p, q
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 8; ++k) {  // rows p, q
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
        for (int k = 0; k < 8; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - sn * vkq;
          V[k][q] = sn * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < 8; ++i) w[i] = A[i][i];
}

// The largest eigenvalue of the Hermitian 4x4 matrix hr + i hi and its unit
// eigenvector phi (interleaved), phase-fixed: its first component of
// magnitude above 1e-9 of the largest is made real and positive.
void hermitian4_top(const double hr[4][4], const double hi[4][4], double* lam, double phi[8]) {
  double A[8][8], w[8], V[8][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      A[i][j] = hr[i][j];
      A[i][j + 4] = -hi[i][j];
      A[i + 4][j] = hi[i][j];
      A[i + 4][j + 4] = hr[i][j];
    }
  jacobi8(A, w, V);
  int top = 0;
  for (int i = 1; i < 8; ++i)
    if (w[i] > w[top]) top = i;
  *lam = w[top];
  double mag = 0.0, big = 0.0;
  for (int m = 0; m < 4; ++m) {
    phi[2 * m] = V[m][top];
    phi[2 * m + 1] = V[m + 4][top];
    mag += phi[2 * m] * phi[2 * m] + phi[2 * m + 1] * phi[2 * m + 1];
  }
  mag = std::sqrt(mag);
  for (int i = 0; i < 8; ++i) phi[i] /= mag;
  for (int m = 0; m < 4; ++m) big = std::max(big, std::hypot(phi[2 * m], phi[2 * m + 1]));
  for (int m = 0; m < 4; ++m) {
    const double r = std::hypot(phi[2 * m], phi[2 * m + 1]);
    if (r > 1e-9 * big) {
      const double cr = phi[2 * m] / r, ci = -phi[2 * m + 1] / r;  // conj of the unit phase
      for (int j = 0; j < 4; ++j) {
        const double x = phi[2 * j], y = phi[2 * j + 1];
        phi[2 * j] = x * cr - y * ci;
        phi[2 * j + 1] = x * ci + y * cr;
      }
      break;
    }
  }
}

// Merge subsystem ib into ia (ia's qubits keep their bits); returns the
// index of the merged subsystem. The caller checked the capacity.
int merge(FactorState* f, int ia, int ib, int* out) {
  Sub& A = f->subs[ia];
  Sub& B = f->subs[ib];
  const int nq = A.nq + B.nq;
  void* c = sub_alloc(f, nq);
  if (!c) return ffail(QS_E_NOMEM, "allocating a %d-qubit subsystem", nq);
  hipError_t e = f->dtype == QS_C64
                     ? launch_compose(static_cast<float*>(c), static_cast<const float*>(A.amps),
                                      A.nq, static_cast<const float*>(B.amps), B.nq, f->stream)
                     : launch_compose(static_cast<double*>(c), static_cast<const double*>(A.amps),
                                      A.nq, static_cast<const double*>(B.amps), B.nq, f->stream);
  if (e != hipSuccess) {
    sub_free(f, nq, c);
    return dev_err(e, "compose");
  }
  Sub m;
  m.nq = nq;
  for (int t = 0; t < A.nq; ++t) m.q[t] = A.q[t];
  for (int t = 0; t < B.nq; ++t) m.q[A.nq + t] = B.q[t];
  m.amps = c;
  sub_free(f, A.nq, A.amps);
  sub_free(f, B.nq, B.amps);
  const int lo = std::min(ia, ib), hi = std::max(ia, ib);
  f->subs.erase(f->subs.begin() + hi);
  f->subs.erase(f->subs.begin() + lo);
  f->subs.push_back(m);
  *out = int(f->subs.size()) - 1;
  return QS_OK;
}

// The outcome of one test: bookkeeping for the proposal features, then the
// log entry and the fidelity factor (Eq. fid_model), held back while deferred
// tests run so that they follow the order of the gates.
void record(FactorState* f, int q, int nsub, double eps, bool rounded, int partner = -1) {
  if (partner < 0) note_test_impl(f, q, eps, rounded);
  if (f->flushing) {
    f->pend.push_back({f->cur_phase, q, nsub, eps, rounded, partner, f->cur_gates});
    if (f->feat_log) {
      if (partner >= 0) std::fill(f->cur_feat, f->cur_feat + QS_MLP_INPUTS, 0.0f);
      f->pend_feat.insert(f->pend_feat.end(), f->cur_feat, f->cur_feat + QS_MLP_INPUTS);
    }
    return;
  }
  if (rounded) f->F *= (1.0 - eps);
  log_attempt(f, q, nsub, eps, rounded, partner, f->gate_count);
}

// The decision on qubit q at bit t of subsystem si from its Bloch sums
// st = {Re s, Im s, z0, z1} (Sec. III-A, Eq. sdrp); *rounded on success.
int decide_qubit(FactorState* f, int q, int si, int t, const double st[4], double p,
                 bool* rounded) {
  *rounded = false;
  Sub& S = f->subs[si];
  // Bloch vector of rho_q (Sec. III-A, step 1) and eps = (1 - |r|)/2 (step 2)
  const double nrm = st[2] + st[3];
  if (!(nrm > 0.0)) return ffail(QS_E_NUMERIC, "subsystem of qubit %d has zero norm", q);
  const double rx = 2.0 * st[0] / nrm, ry = 2.0 * st[1] / nrm, rz = (st[2] - st[3]) / nrm;
  const double rn = std::sqrt(rx * rx + ry * ry + rz * rz);
  const double eps = std::min(std::max((1.0 - rn) / 2.0, 0.0), 0.5);
  if (!(eps <= p / 2.0 + f->tau)) {
    record(f, q, S.nq, eps, false);
    return QS_OK;
  }
  // dominant eigenvector phi of rho_q, phi_0 real >= 0 (steps 3-4)
  double phi[4];
  if (rn == 0.0) {
    phi[0] = 1.0; phi[1] = 0.0; phi[2] = 0.0; phi[3] = 0.0;
  } else {
    const double th = std::acos(std::max(-1.0, std::min(1.0, rz / rn)));
    const double az = std::atan2(ry, rx);
    phi[0] = std::cos(th / 2.0);
    phi[1] = 0.0;
    phi[2] = std::cos(az) * std::sin(th / 2.0);
    phi[3] = std::sin(az) * std::sin(th / 2.0);
  }
  // the kept branch carries weight (1 + |r|)/2 of the subsystem's norm
  const double scale = 1.0 / std::sqrt(0.5 * (1.0 + rn) * nrm);
  void* rest = sub_alloc(f, S.nq - 1);
  if (!rest) return ffail(QS_E_NOMEM, "allocating a %d-qubit subsystem", S.nq - 1);
  Sub single;
  if (f->defer) {  // queued: the projection and the new subsystem in one operation
    single.nq = 1;
    single.q[0] = q;
    single.known = true;
    for (int i = 0; i < 4; ++i) single.h[i] = phi[i];
    single.amps = sub_alloc(f, 1);
    if (!single.amps) {
      sub_free(f, S.nq - 1, rest);
      return ffail(QS_E_NOMEM, "allocating a one-qubit subsystem");
    }
    FactorState::QOp op;
    op.kind = 1;
    op.a = S.amps;
    op.c = rest;
    op.single = single.amps;
    op.na = S.nq;
    op.t0 = t;
    for (int i = 0; i < 4; ++i) op.phi[i] = phi[i];
    op.scale = scale;
    f->qops.push_back(op);
  } else if (int rc = new_single(f, q, phi, &single)) {
    sub_free(f, S.nq - 1, rest);
    return rc;
  }
  hipError_t e = hipSuccess;
  if (!f->defer)
    e = f->dtype == QS_C64
            ? launch_decompose(static_cast<float*>(rest), static_cast<const float*>(S.amps), S.nq,
                               t, phi, scale, f->stream)
            : launch_decompose(static_cast<double*>(rest), static_cast<const double*>(S.amps),
                               S.nq, t, phi, scale, f->stream);
  if (e != hipSuccess) {
    sub_free(f, S.nq - 1, rest);
    sub_free(f, 1, single.amps);
    return dev_err(e, "decompose");
  }
  const int nsub = S.nq;
  sub_free(f, S.nq, S.amps);
  S.amps = rest;
  S.known = false;
  for (int b = t; b + 1 < S.nq; ++b) S.q[b] = S.q[b + 1];
  S.nq -= 1;
  for (int b = 0; b < S.nq; ++b) f->dirty |= uint64_t(1) << S.q[b];
  f->subs.push_back(single);
  record(f, q, nsub, eps, true);
  *rounded = true;
  return QS_OK;
}

// Bookkeeping shared by every exact test: the qubit leaves the dirty and
// deferred sets, and its features (as seen before the test) are logged.
void begin_test(FactorState* f, int q, double p) {
  f->dirty &= ~(uint64_t(1) << q);
  f->deferred &= ~(uint64_t(1) << q);
  f->prop &= ~(uint64_t(1) << q);
  if (!f->feat_log || !f->log_count) return;
  if (f->flushing)
    fact_features(f, q, p, f->cur_feat);  // logged with the attempt, in gate order
  else if (*f->log_count < f->feat_cap)
    fact_features(f, q, p, f->feat_log + *f->log_count * QS_MLP_INPUTS);
}

// One separability attempt on qubit q (Eq. sdrp); *rounded on success.
int test_qubit(FactorState* f, int q, double p, bool* rounded) {
  *rounded = false;
  int t = 0;
  const int si = find(f, q, &t);
  if (si < 0) return ffail(QS_E_INVAL, "qubit %d not found", q);
  if (f->subs[si].nq == 1) {
    f->dirty &= ~(uint64_t(1) << q);
    f->deferred &= ~(uint64_t(1) << q);
    return QS_OK;
  }
  begin_test(f, q, p);
  const Sub& S = f->subs[si];
  hipError_t e = f->dtype == QS_C64
                     ? launch_bloch(static_cast<const float*>(S.amps), S.nq, t, f->scratch,
                                    f->dstat, f->stream)
                     : launch_bloch(static_cast<const double*>(S.amps), S.nq, t, f->scratch,
                                    f->dstat, f->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
  if (int rc = dev_err(e, "bloch")) return rc;
  const double st[4] = {f->hstat[0], f->hstat[1], f->hstat[2], f->hstat[3]};
  return decide_qubit(f, q, si, t, st, p, rounded);
}

// G >= 2 dirty qubits of subsystem si (ascending global numbers, local bits
// ts): their Bloch sums in one sweep, then the decisions in order, stopping
// at the first rounding (which changes the subsystem; the rest stay dirty).
// The decisions are those of testing the qubits one after another.
int test_batch(FactorState* f, int si, const int* qs_, const int* ts, int G, double p,
               int* count) {
  int order[kMultiTest], bits[kMultiTest];
  for (int i = 0; i < G; ++i) order[i] = i;
  std::sort(order, order + G, [ts](int x, int y) { return ts[x] < ts[y]; });
  for (int i = 0; i < G; ++i) bits[i] = ts[order[i]];
  const Sub& S = f->subs[si];
  hipError_t e = f->dtype == QS_C64
                     ? launch_bloch_multi(static_cast<const float*>(S.amps), S.nq, bits, G,
                                          f->scratch, f->dstat, f->stream)
                     : launch_bloch_multi(static_cast<const double*>(S.amps), S.nq, bits, G,
                                          f->scratch, f->dstat, f->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
  if (int rc = dev_err(e, "bloch")) return rc;
  double st[kMultiTest][4];
  for (int i = 0; i < G; ++i)
    for (int k = 0; k < 4; ++k) st[order[i]][k] = f->hstat[4 * i + k];
  for (int i = 0; i < G; ++i) {
    begin_test(f, qs_[i], p);
    bool rounded = false;
    if (int rc = decide_qubit(f, qs_[i], si, ts[i], st[i], p, &rounded)) return rc;
    if (rounded) {
      *count += 1;
      break;
    }
  }
  return QS_OK;
}

// Exact test of the lowest qubit of `mask` (dirty qubits only) and, with
// multi-qubit sweeps on, of the next ones of `mask` in ascending order while
// they share its subsystem (up to kMultiTest). *rounded if one was rounded.
int test_lowest(FactorState* f, uint64_t mask, double p, int* count, bool* rounded) {
  *rounded = false;
  mask &= f->dirty;
  if (!mask) return QS_OK;
  const int q = __builtin_ctzll(mask);
  int t = 0;
  const int si = find(f, q, &t);
  if (si < 0) return ffail(QS_E_INVAL, "qubit %d not found", q);
  int bq[kMultiTest] = {q}, bt[kMultiTest] = {t}, G = 1;
  if (g_multi_test && f->subs[si].nq > 1) {
    for (uint64_t d = mask & (mask - 1); d && G < kMultiTest; d &= d - 1) {
      const int q2 = __builtin_ctzll(d);
      int t2 = 0;
      if (find(f, q2, &t2) != si) break;
      bq[G] = q2;
      bt[G] = t2;
      ++G;
    }
  }
  const int before = *count;
  if (G == 1) {
    bool r = false;
    if (int rc = test_qubit(f, q, p, &r)) return rc;
    *count += r;
  } else if (int rc = test_batch(f, si, bq, bt, G, p, count)) {
    return rc;
  }
  *rounded = *count > before;
  return QS_OK;
}

// Plain schedule: the lowest-numbered dirty qubit until none is dirty (with
// multi-qubit sweeps, the next dirty qubits of its subsystem alongside).
int plain_separate(FactorState* f, double p, int* count) {
  while (f->dirty) {
    bool rounded = false;
    if (int rc = test_lowest(f, f->dirty, p, count, &rounded)) return rc;
  }
  return QS_OK;
}

// Learned schedule: dirty qubits of subsystems smaller than propose_min get
// the exact test directly; the others are scored in one forward pass, the
// rest deferred and the proposals tested in ascending order until one is
// rounded, after which the qubits made dirty are scored again.
int proposed_separate(FactorState* f, double p, int* count) {
  std::vector<int> cand;
  std::vector<float> X, score;
  while (f->dirty) {
    uint64_t small = 0;
    for (uint64_t d = f->dirty; d; d &= d - 1) {
      const int q = __builtin_ctzll(d);
      const int si = find(f, q, nullptr);
      if (si >= 0 && f->subs[si].nq < f->propose_min) small |= uint64_t(1) << q;
    }
    if (small) {
      bool rounded = false;
      if (int rc = test_lowest(f, small, p, count, &rounded)) return rc;
      continue;
    }
    cand.clear();
    for (uint64_t d = f->dirty; d; d &= d - 1) cand.push_back(__builtin_ctzll(d));
    X.assign(cand.size() * QS_MLP_INPUTS, 0.0f);
    for (size_t i = 0; i < cand.size(); ++i) fact_features(f, cand[i], p, &X[i * QS_MLP_INPUTS]);
    score.assign(cand.size(), 0.0f);
    if (int rc = mlp_scores(f->proposer, X.data(), cand.size(), score.data())) return rc;
    uint64_t prop = 0;
    for (size_t i = 0; i < cand.size(); ++i) {
      const uint64_t bit = uint64_t(1) << cand[i];
      if (score[i] >= f->cutoff) {
        prop |= bit;
      } else {
        f->dirty &= ~bit;
        f->deferred |= bit;
        ++f->skipped;
      }
    }
    while (prop & f->dirty) {
      bool rounded = false;
      if (int rc = test_lowest(f, prop, p, count, &rounded)) return rc;
      if (rounded) break;
    }
  }
  return QS_OK;
}

// Bookkeeping of one exact test (features of later proposals).
}  // namespace

void note_test_impl(FactorState* f, int q, double eps, bool rounded) {
  f->eps_prev[q] = f->eps_last[q];
  f->eps_last[q] = eps;
  f->rounded_last[q] = rounded ? 1 : 0;
  f->tests[q] += 1;
  f->gates_since[q] = 0;
  f->recent[f->recent_n % 8] = rounded ? 1 : 0;
  f->recent_n += 1;
  f->recent_eps = eps;
}

void fact_features(const FactorState* f, int q, double p, float* x) {
  for (int i = 0; i < QS_MLP_INPUTS; ++i) x[i] = 0.0f;
  auto eps_or = [](double e) { return e < 0.0 ? 0.5 : e; };
  auto purity = [](double e) { const double r = 1.0 - 2.0 * e; return 0.5 * (1.0 + r * r); };
  int ns = 1, nsub = int(f->subs.size()), largest = 1;
  for (const auto& s : f->subs) {
    largest = std::max(largest, s.nq);
    for (int t = 0; t < s.nq; ++t)
      if (s.q[t] == q) ns = s.nq;
  }
  const double el = eps_or(f->eps_last[q]), ep = eps_or(f->eps_prev[q]);
  const int pq = f->partner[q];
  int pns = 0;
  if (pq >= 0)
    for (const auto& s : f->subs)
      for (int t = 0; t < s.nq; ++t)
        if (s.q[t] == pq) pns = s.nq;
  int rec = 0;
  const int nrec = std::min(f->recent_n, 8);
  for (int i = 0; i < nrec; ++i) rec += f->recent[i];
  x[0] = float(ns / 32.0);
  x[1] = float(std::log2(double(ns)) / 6.0);
  x[2] = float(p);
  x[3] = float(el);                      // Bloch length |r| = 1 - 2 eps
  x[4] = float(ep);
  x[5] = float(purity(el));              // purity of the reduced state
  x[6] = float(purity(ep));
  x[7] = float(f->rounded_last[q]);
  x[8] = float(std::min(f->gates_since[q], 8) / 8.0);
  x[9] = float(std::min(f->tests[q], 32) / 32.0);
  x[10] = float(pq >= 0 ? eps_or(f->eps_last[pq]) : 0.5);
  x[11] = float(purity(x[10]));
  x[12] = float(pns / 32.0);
  x[13] = float(f->merged_last[q]);
  x[14] = float(nrec ? double(rec) / nrec : 0.0);
  x[15] = float(eps_or(f->recent_eps));
  x[16] = float(double(nsub) / f->n);
  x[17] = float(largest / 32.0);
  x[18] = float(el - p / 2.0);
  x[19] = f->tests[q] == 0 ? 1.0f : 0.0f;
  x[20] = float(std::min<uint64_t>(f->gate_count, 2000) / 2000.0);
}

int fact_init(FactorState* f) {
  f->subs.clear();
  f->eps_last.assign(f->n, -1.0);
  f->eps_prev.assign(f->n, -1.0);
  f->rounded_last.assign(f->n, 0);
  f->tests.assign(f->n, 0);
  f->gates_since.assign(f->n, 0);
  f->partner.assign(f->n, -1);
  f->merged_last.assign(f->n, 0);
  for (int q = 0; q < f->n; ++q) {
    const double zero[4] = {1.0, 0.0, 0.0, 0.0};
    Sub s;
    if (int rc = new_single(f, q, zero, &s)) {
      fact_release(f);
      return rc;
    }
    f->subs.push_back(s);
  }
  f->F = 1.0;
  f->dirty = 0;
  return dev_err(hipStreamSynchronize(f->stream), "init");
}

void fact_release(FactorState* f) {
  (void)hipStreamSynchronize(f->stream);
  f->qops.clear();  // only left behind by a device error
  std::vector<std::pair<int, void*>> late;
  late.swap(f->late_free);
  for (const auto& b : late) sub_free(f, b.first, b.second);
  for (auto& s : f->subs) sub_free(f, s.nq, s.amps);
  f->subs.clear();
}

void fact_drain(FactorState* f) {
  fact_release(f);
  for (int i = 0; i < FactorState::kRingSlots; ++i) {
    if (f->ring_ev[i]) (void)hipEventDestroy(f->ring_ev[i]);
    if (f->ring_host[i]) (void)hipHostFree(f->ring_host[i]);
    f->ring_ev[i] = nullptr;
    f->ring_host[i] = f->ring_dev[i] = nullptr;
    f->ring_used[i] = false;
  }
  for (auto& v : f->pool) {
    for (void* p : v) device_free(p);
    v.clear();
  }
  device_free(f->tile_dev);
  f->tile_dev = nullptr;
  f->tile_cap = 0;
  if (f->sig_host) (void)hipHostFree(f->sig_host);
  device_free(f->sig_count);
  f->sig_host = f->sig_dev = f->sig_count = nullptr;
}

int fact_set_basis(FactorState* f, uint64_t x) {
  fact_release(f);
  for (int q = 0; q < f->n; ++q) {
    const double b0[4] = {1.0, 0.0, 0.0, 0.0}, b1[4] = {0.0, 0.0, 1.0, 0.0};
    Sub s;
    if (int rc = new_single(f, q, ((x >> q) & 1) ? b1 : b0, &s)) return rc;
    f->subs.push_back(s);
  }
  f->F = 1.0;
  f->dirty = 0;
  f->deferred = 0;
  f->eps_last.assign(f->n, -1.0);
  f->eps_prev.assign(f->n, -1.0);
  f->rounded_last.assign(f->n, 0);
  f->tests.assign(f->n, 0);
  f->gates_since.assign(f->n, 0);
  f->partner.assign(f->n, -1);
  f->merged_last.assign(f->n, 0);
  return dev_err(hipStreamSynchronize(f->stream), "set basis");
}

int fact_largest(const FactorState* f) {
  int m = 0;
  for (const auto& s : f->subs) m = std::max(m, s.nq);
  return m;
}

// The two-qubit decision on qa (bit ta) and qb (bit tb) of subsystem sa from
// the unnormalized pair density sums st[16] (layout of launch_pair_rho).
int decide_pair(FactorState* f, int sa, int qa, int qb, int ta, int tb, const double* st, double p,
                bool* rounded) {
  *rounded = false;
  // H = rho (unnormalized), index m = bit ta + 2 bit tb
  double hr[4][4], hi[4][4];
  const double tr = st[0] + st[1] + st[2] + st[3];
  if (!(tr > 0.0)) return ffail(QS_E_NUMERIC, "subsystem of qubit %d has zero norm", qa);
  for (int m = 0; m < 4; ++m) {
    hr[m][m] = st[m] / tr;
    hi[m][m] = 0.0;
  }
  int k = 4;
  for (int m = 0; m < 4; ++m)
    for (int mp = m + 1; mp < 4; ++mp) {
      hr[m][mp] = st[k] / tr;
      hi[m][mp] = st[k + 1] / tr;
      hr[mp][m] = hr[m][mp];
      hi[mp][m] = -hi[m][mp];
      k += 2;
    }
  double lam = 0.0, phi[8];
  hermitian4_top(hr, hi, &lam, phi);
  const double eps = std::min(std::max(1.0 - lam, 0.0), 0.75);
  const Sub& S = f->subs[sa];
  const int nq = S.nq;
  if (!(eps <= p / 2.0 + f->tau)) {
    record(f, qa, nq, eps, false, qb);
    return QS_OK;
  }
  // <phi|psi> has squared norm lam * tr
  const double scale = 1.0 / std::sqrt(lam * tr);
  void* rest = sub_alloc(f, nq - 2);
  void* pair = sub_alloc(f, 2);
  if (!rest || !pair) {
    sub_free(f, nq - 2, rest);
    sub_free(f, 2, pair);
    return ffail(QS_E_NOMEM, "allocating the pair's subsystems");
  }
  const hipError_t e = f->dtype == QS_C64
          ? launch_decompose_pair(static_cast<float*>(rest), static_cast<const float*>(S.amps),
                                  nq, ta, tb, phi, scale, static_cast<float*>(pair), f->stream)
          : launch_decompose_pair(static_cast<double*>(rest), static_cast<const double*>(S.amps),
                                  nq, ta, tb, phi, scale, static_cast<double*>(pair), f->stream);
  if (e != hipSuccess) {
    sub_free(f, nq - 2, rest);
    sub_free(f, 2, pair);
    return dev_err(e, "pair projection");
  }
  Sub P;
  P.nq = 2;
  P.q[0] = qa;
  P.q[1] = qb;
  P.amps = pair;
  Sub& T = f->subs[sa];
  sub_free(f, T.nq, T.amps);
  T.amps = rest;
  T.known = false;
  int w2 = 0;
  for (int b = 0; b < T.nq; ++b)
    if (T.q[b] != qa && T.q[b] != qb) T.q[w2++] = T.q[b];
  T.nq = w2;
  for (int b = 0; b < T.nq; ++b) f->dirty |= uint64_t(1) << T.q[b];
  f->subs.push_back(P);
  record(f, qa, nq, eps, true, qb);
  *rounded = true;
  return QS_OK;
}

void fact_hermitian4_top(const double* h, double* lam, double* phi) {
  double hr[4][4], hi[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {  // the Hermitian part (h + h^H) / 2
      hr[i][j] = 0.5 * (h[2 * (4 * i + j)] + h[2 * (4 * j + i)]);
      hi[i][j] = 0.5 * (h[2 * (4 * i + j) + 1] - h[2 * (4 * j + i) + 1]);
    }
  hermitian4_top(hr, hi, lam, phi);
}

int fact_test_pair(FactorState* f, int qa, int qb, double p, bool* rounded) {
  *rounded = false;
  int ta = 0, tb = 0;
  const int sa = find(f, qa, &ta), sb = find(f, qb, &tb);
  if (sa < 0 || sb < 0 || qa == qb) return ffail(QS_E_INVAL, "bad pair (%d, %d)", qa, qb);
  if (sa != sb || f->subs[sa].nq < 3) return QS_OK;  // nothing to split off
  if (int rc = launch_queue(f)) return rc;
  const Sub& S0 = f->subs[sa];
  hipError_t e = f->dtype == QS_C64
                     ? launch_pair_rho(static_cast<const float*>(S0.amps), S0.nq, ta, tb,
                                       f->scratch, f->dstat, nullptr, nullptr, 0, 0, f->stream)
                     : launch_pair_rho(static_cast<const double*>(S0.amps), S0.nq, ta, tb,
                                       f->scratch, f->dstat, nullptr, nullptr, 0, 0, f->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
  if (int rc = dev_err(e, "pair density")) return rc;
  double st[16];
  for (int i = 0; i < 16; ++i) st[i] = f->hstat[i];
  return decide_pair(f, sa, qa, qb, ta, tb, st, p, rounded);
}

namespace {

// Exact tests, without the proposer, of the qubits of `mask` (skipped by the
// proposer earlier): at once, or (deferred mode) after the pending tests, in
// a flush of their own that logs them after every earlier gate's attempts.
int exact_retest(FactorState* f, uint64_t mask) {
  if (!f->defer) {
    f->dirty |= mask;
    int nsep = 0;
    return plain_separate(f, f->p, &nsep);
  }
  if (f->dirty)
    if (int rc = flush_pending(f)) return rc;
  f->dirty |= mask;
  const uint64_t phase = ++f->phase_next;
  for (auto& S : f->subs)
    for (int b = 0; b < S.nq; ++b)
      if ((mask >> S.q[b]) & 1) {
        S.plain = true;
        S.phase = phase;
        S.phase_gates = f->gate_count;
        break;
      }
  return flush_pending(f);
}

// A two-qubit gate: the merge (when the qubits lie in two subsystems) and the
// gate become one queued operation; the subsystem table changes at once, as
// merge() changes it. The capacity was checked.
int queue_gate2(FactorState* f, const int* qubits, const double* m) {
  ++f->gate_count;
  const int si = find(f, qubits[0], nullptr), sj = find(f, qubits[1], nullptr);
  for (int j = 0; j < 2; ++j) {
    f->gates_since[qubits[j]] += 1;
    f->partner[qubits[j]] = qubits[1 - j];
    f->merged_last[qubits[j]] = si != sj ? 1 : 0;
  }
  FactorState::QOp op;
  for (int i = 0; i < 32; ++i) op.m[i] = m[i];
  int target = si;
  if (si != sj) {
    const Sub A = f->subs[si], B = f->subs[sj];
    const int nq = A.nq + B.nq;
    void* c = sub_alloc(f, nq);
    if (!c) return ffail(QS_E_NOMEM, "allocating a %d-qubit subsystem", nq);
    Sub M;
    M.nq = nq;
    for (int t = 0; t < A.nq; ++t) M.q[t] = A.q[t];
    for (int t = 0; t < B.nq; ++t) M.q[A.nq + t] = B.q[t];
    M.amps = c;
    op.a = A.amps;
    op.b = B.amps;
    op.c = c;
    op.na = A.nq;
    op.nb = B.nq;
    f->qops.push_back(op);  // queued first, so that the frees below wait for it
    sub_free(f, A.nq, A.amps);
    sub_free(f, B.nq, B.amps);
    const int lo = std::min(si, sj), hi = std::max(si, sj);
    f->subs.erase(f->subs.begin() + hi);
    f->subs.erase(f->subs.begin() + lo);
    f->subs.push_back(M);
    target = int(f->subs.size()) - 1;
  } else {
    const Sub& S = f->subs[si];
    op.a = op.c = S.amps;
    op.na = S.nq;
    f->qops.push_back(op);
  }
  Sub& S = f->subs[target];
  FactorState::QOp& q = f->qops.back();
  for (int b = 0; b < S.nq; ++b) {
    if (S.q[b] == qubits[0]) q.t0 = b;
    if (S.q[b] == qubits[1]) q.t1 = b;
  }
  for (int j = 0; j < 2; ++j) f->dirty |= uint64_t(1) << qubits[j];
  S.phase = ++f->phase_next;
  S.phase_gates = f->gate_count;
  if (f->policy == QS_SEP_AFTER_2Q_PAIRS) {  // its pair test follows its one-qubit tests
    S.pend_a = qubits[0];
    S.pend_b = qubits[1];
  }
  return QS_OK;
}

}  // namespace

namespace {

// h <- m h for the host copy of a one-qubit subsystem (m: 2x2, interleaved).
void mirror_1q(Sub& S, const double* m) {
  if (S.nq != 1 || !S.known) return;
  // (callers skip this while the host copies already include the gate)
  const double a0r = S.h[0], a0i = S.h[1], a1r = S.h[2], a1i = S.h[3];
  S.h[0] = m[0] * a0r - m[1] * a0i + m[2] * a1r - m[3] * a1i;
  S.h[1] = m[0] * a0i + m[1] * a0r + m[2] * a1i + m[3] * a1r;
  S.h[2] = m[4] * a0r - m[5] * a0i + m[6] * a1r - m[7] * a1i;
  S.h[3] = m[4] * a0i + m[5] * a0r + m[6] * a1i + m[7] * a1r;
}

// Is qubit q a one-qubit subsystem in a Z eigenstate (up to a relative weight
// of 1e-24 on the other basis state)? *v receives the eigenvalue's bit.
bool z_eigenstate(const FactorState* f, int q, int* v) {
  const int si = find(f, q, nullptr);
  if (si < 0) return false;
  const Sub& S = f->subs[si];
  if (S.nq != 1 || !S.known) return false;
  const double p0 = S.h[0] * S.h[0] + S.h[1] * S.h[1], p1 = S.h[2] * S.h[2] + S.h[3] * S.h[3];
  if (p1 <= 1e-24 * (p0 + p1)) {
    *v = 0;
    return true;
  }
  if (p0 <= 1e-24 * (p0 + p1)) {
    *v = 1;
    return true;
  }
  return false;
}

// Restricts the k-qubit gate m (2^k x 2^k, interleaved) to value v of its
// local bit j, if the gate keeps that value (every entry from a column with
// bit j = v to a row with bit j != v is exactly zero): out is the (k-1)-qubit
// gate on the other bits, in order. False (out untouched) otherwise.
bool restrict_gate(const std::vector<double>& m, int k, int j, int v, std::vector<double>* out) {
  const int d = 1 << k;
  for (int r = 0; r < d; ++r) {
    if (((r >> j) & 1) == v) continue;
    for (int c = 0; c < d; ++c)
      if (((c >> j) & 1) == v && (m[2 * (r * d + c)] != 0.0 || m[2 * (r * d + c) + 1] != 0.0))
        return false;
  }
  const int dr = d / 2;
  auto ins = [j, v](int x) {
    const int lo = x & ((1 << j) - 1);
    return lo | (v << j) | ((x >> j) << (j + 1));
  };
  out->assign(size_t(2) * dr * dr, 0.0);
  for (int r = 0; r < dr; ++r)
    for (int c = 0; c < dr; ++c) {
      const size_t src = size_t(ins(r)) * d + ins(c);
      (*out)[2 * (r * dr + c)] = m[2 * src];
      (*out)[2 * (r * dr + c) + 1] = m[2 * src + 1];
    }
  return true;
}

bool is_identity(const std::vector<double>& m, int k) {
  const int d = 1 << k;
  for (int r = 0; r < d; ++r)
    for (int c = 0; c < d; ++c)
      if (m[2 * (r * d + c)] != (r == c ? 1.0 : 0.0) || m[2 * (r * d + c) + 1] != 0.0) return false;
  return true;
}

}  // namespace

void fact_mirror_1q(FactorState* f, int q, const double* m) {
  const int si = find(f, q, nullptr);
  if (si >= 0) mirror_1q(f->subs[si], m);
}

bool fact_reduce(FactorState* f, int* qubits, int* k, std::vector<double>* m) {
  if (*k < 2 || !g_unobservable) return false;
  std::vector<double> red;
  bool changed = false;
  for (int j = 0; j < *k && *k > 1;) {
    int v = 0;
    if (z_eigenstate(f, qubits[j], &v) && restrict_gate(*m, *k, j, v, &red)) {
      m->swap(red);
      for (int t = j; t + 1 < *k; ++t) qubits[t] = qubits[t + 1];
      --*k;
      changed = true;
      ++f->shortcuts;
      continue;
    }
    ++j;
  }
  if (changed && is_identity(*m, *k)) *k = 0;
  return changed;
}

namespace {

using cd = std::complex<double>;

// Entries below this (relative to the largest) count as zero when a product
// of unitaries is classified; it bounds the change a classification makes.
constexpr double kHeldTol = 1e-13;

// Is the 4x4 gate m (local bits 0, 1) the identity where local bit cl is 0,
// with no entry between cl = 0 and cl = 1? M receives the block where cl = 1
// (rows, columns by the other bit).
bool controlled_block(const double* m, int cl, cd M[4]) {
  const int tl = 1 - cl;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) {
      const cd v(m[2 * (4 * r + c)], m[2 * (4 * r + c) + 1]);
      const int cr = (r >> cl) & 1, cc = (c >> cl) & 1;
      if (cr != cc) {
        if (std::norm(v) > kHeldTol * kHeldTol) return false;
      } else if (cr == 0) {
        const double want = ((r >> tl) & 1) == ((c >> tl) & 1) ? 1.0 : 0.0;
        if (std::norm(v - want) > kHeldTol * kHeldTol) return false;
      } else {
        M[2 * ((r >> tl) & 1) + ((c >> tl) & 1)] = v;
      }
    }
  return true;
}

// M as a held gate's matrix: diagonal or anti-diagonal after snapping
// entries below the tolerance to zero.
bool phase_or_inversion(cd M[4], bool* inv, cd* d0, cd* d1) {
  double big = 0.0;
  for (int i = 0; i < 4; ++i) big = std::max(big, std::abs(M[i]));
  for (int i = 0; i < 4; ++i)
    if (std::abs(M[i]) <= kHeldTol * big) M[i] = 0.0;
  if (M[1] == 0.0 && M[2] == 0.0) {
    *inv = false;
    *d0 = M[0];
    *d1 = M[3];
    return true;
  }
  if (M[0] == 0.0 && M[3] == 0.0) {
    *inv = true;
    *d0 = M[1];
    *d1 = M[2];
    return true;
  }
  return false;
}

void held_block(const HeldGate& g, cd M[4]) {
  if (g.inv) {
    M[0] = 0.0, M[1] = g.d0, M[2] = g.d1, M[3] = 0.0;
  } else {
    M[0] = g.d0, M[1] = 0.0, M[2] = 0.0, M[3] = g.d1;
  }
}

}  // namespace

bool held_classify(const double* m, const int* qubits, HeldGate* g) {
  for (int cl = 0; cl < 2; ++cl) {
    cd M[4];
    if (!controlled_block(m, cl, M)) continue;
    HeldGate h;
    if (!phase_or_inversion(M, &h.inv, &h.d0, &h.d1)) return false;
    h.c = qubits[cl];
    h.t = qubits[1 - cl];
    *g = h;
    return true;
  }
  return false;
}

bool held_commute(const HeldGate& a, const HeldGate& b) {
  const bool share = a.c == b.c || a.c == b.t || a.t == b.c || a.t == b.t;
  if (!share || (!a.inv && !b.inv)) return true;  // disjoint, or both diagonal
  if (a.c == b.c && a.t == b.t) {                  // one pair, one orientation
    cd A[4], B[4];
    held_block(a, A);
    held_block(b, B);
    for (int r = 0; r < 2; ++r)
      for (int c = 0; c < 2; ++c) {
        const cd ab = A[2 * r] * B[c] + A[2 * r + 1] * B[2 + c];
        const cd ba = B[2 * r] * A[c] + B[2 * r + 1] * A[2 + c];
        if (std::abs(ab - ba) > kHeldTol) return false;
      }
    return true;
  }
  if (a.c == b.t && a.t == b.c) return false;  // one of them an inversion
  if (a.c == b.c) return true;                 // one control, two targets
  if (a.t == b.t)  // one target: two inversions [[0,x0],[x1,0]] commute iff a0 b1 = b0 a1
    return a.inv && b.inv && std::abs(a.d0 * b.d1 - b.d0 * a.d1) <= kHeldTol;
  if (a.c == b.t) return !b.inv;  // b acts on a's control
  return !a.inv;                  // a.t == b.c: a acts on b's control
}

bool held_pass_1q(HeldGate* g, int q, const double* u) {
  const cd U[4] = {{u[0], u[1]}, {u[2], u[3]}, {u[4], u[5]}, {u[6], u[7]}};
  HeldGate h = *g;
  if (q == h.c) {
    // a diagonal u keeps the control's projectors
    if (std::abs(U[1]) <= kHeldTol && std::abs(U[2]) <= kHeldTol) return true;
    // a phase with d0 = 1 is diag(1, 1, 1, d1): symmetric, so q may be its target
    if (h.inv || std::abs(h.d0 - 1.0) > kHeldTol) return false;
    std::swap(h.c, h.t);
  }
  if (q != h.t) return false;
  // u (control 1: M) = (control 1: u M u^dagger) u
  cd M[4], T[4], R[4];
  held_block(h, M);
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c) T[2 * r + c] = U[2 * r] * M[c] + U[2 * r + 1] * M[2 + c];
  for (int r = 0; r < 2; ++r)
    for (int c = 0; c < 2; ++c)
      R[2 * r + c] = T[2 * r] * std::conj(U[2 * c]) + T[2 * r + 1] * std::conj(U[2 * c + 1]);
  if (!phase_or_inversion(R, &h.inv, &h.d0, &h.d1)) return false;
  *g = h;
  return true;
}

void held_matrix(const HeldGate& g, double* m) {
  // local bit 0 = control, bit 1 = target
  std::fill(m, m + 32, 0.0);
  m[2 * (4 * 0 + 0)] = 1.0;
  m[2 * (4 * 2 + 2)] = 1.0;
  cd M[4];
  held_block(g, M);
  for (int tr = 0; tr < 2; ++tr)
    for (int tc = 0; tc < 2; ++tc) {
      const int e = 4 * (1 + 2 * tr) + (1 + 2 * tc);
      m[2 * e] = M[2 * tr + tc].real();
      m[2 * e + 1] = M[2 * tr + tc].imag();
    }
}

int fact_sub_of(const FactorState* f, int q) { return find(f, q, nullptr); }

bool fact_kickback(FactorState* f, int* qubits, int* k, std::vector<double>* m) {
  if (*k != 2 || !g_unobservable || !g_kickback) return false;
  for (int cl = 0; cl < 2; ++cl) {
    cd M[4];
    if (!controlled_block(m->data(), cl, M)) continue;
    const int si = find(f, qubits[1 - cl], nullptr);
    if (si < 0) return false;
    const Sub& S = f->subs[si];
    if (S.nq != 1 || !S.known) continue;
    const cd h0(S.h[0], S.h[1]), h1(S.h[2], S.h[3]);
    const double nn = std::norm(h0) + std::norm(h1);
    if (!(nn > 0.0)) continue;
    const cd m0 = M[0] * h0 + M[1] * h1, m1 = M[2] * h0 + M[3] * h1;
    const cd lam = (std::conj(h0) * m0 + std::conj(h1) * m1) / nn;
    if (std::norm(m0 - lam * h0) + std::norm(m1 - lam * h1) > 1e-24 * nn) continue;
    const int c = qubits[cl];
    qubits[0] = c;
    *k = std::abs(lam - 1.0) <= 1e-12 ? 0 : 1;
    m->assign({1.0, 0.0, 0.0, 0.0, 0.0, 0.0, lam.real(), lam.imag()});
    ++f->shortcuts;
    return true;
  }
  return false;
}

bool fact_pending_on(const FactorState* f, const int* qubits, int k) {
  return f->defer && f->dirty && touches_dirty(f, qubits, k);
}

int fact_settle(FactorState* f) { return f->defer && f->dirty ? flush_pending(f) : QS_OK; }

int fact_apply(FactorState* f, const int* qubits, int k, const double* m) {
  // deferred tests on the subsystems this gate touches come first (they may
  // split an operand off into a basis state the shortcut below can use)
  if (fact_pending_on(f, qubits, k))
    if (int rc = flush_pending(f)) return rc;
  // unobservable shortcut (Sec. II-B): operands in a Z eigenstate that the
  // gate keeps are dropped from it, so they need no merge
  if (k >= 2 && g_unobservable) {
    int qq[QS_MAX_FUSED], kq = k;
    for (int j = 0; j < k; ++j) qq[j] = qubits[j];
    std::vector<double> mm(m, m + (size_t(2) << (2 * k)));
    if (fact_reduce(f, qq, &kq, &mm)) return kq == 0 ? QS_OK : fact_apply(f, qq, kq, mm.data());
  }
  // capacity first, so that a refused gate leaves the state as it was
  int distinct[QS_MAX_FUSED], nd = 0, total = 0;
  for (int j = 0; j < k; ++j) {
    const int s = find(f, qubits[j], nullptr);
    if (s < 0) return ffail(QS_E_INVAL, "qubit %d not found", qubits[j]);
    if (std::find(distinct, distinct + nd, s) == distinct + nd) {
      distinct[nd++] = s;
      total += f->subs[s].nq;
    }
  }
  if (nd > 1 && f->deferred && (f->propose_flags & QS_PROPOSE_RETEST_ON_MERGE)) {
    // exact tests of the skipped qubits of the subsystems about to merge
    uint64_t mask = 0;
    for (int j = 0; j < nd; ++j) {
      const Sub& s = f->subs[distinct[j]];
      for (int b = 0; b < s.nq; ++b) mask |= uint64_t(1) << s.q[b];
    }
    mask &= f->deferred;
    if (mask) {
      f->fallback_tests += uint64_t(__builtin_popcountll(mask));
      f->deferred &= ~mask;
      if (int rc = exact_retest(f, mask)) return rc;
      nd = 0;
      total = 0;
      for (int j = 0; j < k; ++j) {
        const int s = find(f, qubits[j], nullptr);
        if (std::find(distinct, distinct + nd, s) == distinct + nd) {
          distinct[nd++] = s;
          total += f->subs[s].nq;
        }
      }
    }
  }
  const bool over = total >= 63 || (uint64_t(1) << total) > f->max_amps;
  if (over && f->defer && f->dirty)  // every skip the fallback must see happens first
    if (int rc = flush_pending(f)) return rc;
  if (over && f->deferred) {
    // exhaustive fallback: exact tests of every qubit the proposer skipped
    // may shrink the subsystems enough for the merge
    f->fallback_tests += uint64_t(__builtin_popcountll(f->deferred));
    const uint64_t mask = f->deferred;
    f->deferred = 0;
    if (int rc = exact_retest(f, mask)) return rc;
    nd = 0;
    total = 0;
    for (int j = 0; j < k; ++j) {
      const int s = find(f, qubits[j], nullptr);
      if (std::find(distinct, distinct + nd, s) == distinct + nd) {
        distinct[nd++] = s;
        total += f->subs[s].nq;
      }
    }
  }
  if (total >= 63 || (uint64_t(1) << total) > f->max_amps)
    return ffail(QS_E_CAPACITY, "gate needs a %d-qubit subsystem (cap %llu amplitudes)", total,
                 (unsigned long long)f->max_amps);
  if (k == 2) {  // merge and gate in one operation, queued or launched at once
    if (int rc = queue_gate2(f, qubits, m)) return rc;
    if (f->defer) return QS_OK;
    if (int rc = launch_queue(f)) return rc;
    if (f->policy == QS_SEP_NONE) return QS_OK;
    int nsep = 0;
    if (int rc = fact_try_separate(f, f->p, &nsep)) return rc;
    if (f->policy != QS_SEP_AFTER_2Q_PAIRS) return QS_OK;
    bool paired = false;
    if (int rc = fact_test_pair(f, qubits[0], qubits[1], f->p, &paired)) return rc;
    return paired ? fact_try_separate(f, f->p, &nsep) : QS_OK;
  }
  if (int rc = launch_queue(f)) return rc;
  // bookkeeping for the proposal features
  if (k >= 2) {
    ++f->gate_count;
    for (int j = 0; j < k; ++j) {
      f->gates_since[qubits[j]] += 1;
      f->partner[qubits[j]] = qubits[j == 0 ? 1 : 0];
      f->merged_last[qubits[j]] = nd > 1 ? 1 : 0;
    }
  }
  // merge every subsystem into the first operand's
  int si = find(f, qubits[0], nullptr);
  for (int j = 1; j < k; ++j) {
    const int sj = find(f, qubits[j], nullptr);
    if (sj != si)
      if (int rc = merge(f, si, sj, &si)) return rc;
  }
  Sub& S = f->subs[si];
  int local[QS_MAX_FUSED];
  for (int j = 0; j < k; ++j)
    for (int b = 0; b < S.nq; ++b)
      if (S.q[b] == qubits[j]) local[j] = b;
  hipError_t e;
  if (k == 1) {
    if (!f->mirrors_ahead) mirror_1q(S, m);
    if (f->dtype == QS_C64) {
      Mat2<float> mm;
      for (int i = 0; i < 4; ++i) { mm.re[i] = float(m[2 * i]); mm.im[i] = float(m[2 * i + 1]); }
      e = launch_apply_1q(static_cast<float*>(S.amps), S.nq, local[0], mm, f->stream);
    } else {
      Mat2<double> mm;
      for (int i = 0; i < 4; ++i) { mm.re[i] = m[2 * i]; mm.im[i] = m[2 * i + 1]; }
      e = launch_apply_1q(static_cast<double*>(S.amps), S.nq, local[0], mm, f->stream);
    }
  } else {
    const size_t D = size_t(1) << k;
    e = upload(f, f->mat, m, D * D);
    if (e == hipSuccess)
      e = f->dtype == QS_C64
              ? launch_apply_fused(static_cast<float*>(S.amps), S.nq, local, k,
                                   static_cast<const float*>(f->mat), f->stream)
              : launch_apply_fused(static_cast<double*>(S.amps), S.nq, local, k,
                                   static_cast<const double*>(f->mat), f->stream);
  }
  if (int rc = dev_err(e, "factorized gate")) return rc;
  if (k >= 2) {
    for (int j = 0; j < k; ++j) f->dirty |= uint64_t(1) << qubits[j];
    if (f->policy != QS_SEP_NONE && f->defer) {
      S.phase = ++f->phase_next;
      S.phase_gates = f->gate_count;
      return QS_OK;
    }
    if (f->policy != QS_SEP_NONE) {
      int nsep = 0;
      return fact_try_separate(f, f->p, &nsep);
    }
  }
  return QS_OK;
}

namespace {

// A free ring slot (waits for the launch that last used it); host and device
// addresses of its table memory.
int ring_slot(FactorState* f, void** host, void** dev) {
  const int i = f->ring_next;
  f->ring_next = (i + 1) % FactorState::kRingSlots;
  if (!f->ring_host[i]) {
    if (hipHostMalloc(&f->ring_host[i], FactorState::kSlotBytes, hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer(&f->ring_dev[i], f->ring_host[i], 0) != hipSuccess ||
        hipEventCreateWithFlags(&f->ring_ev[i], hipEventDisableTiming) != hipSuccess)
      return ffail(QS_E_NOMEM, "pinned table slot");
  } else if (f->ring_used[i]) {
    if (int rc = dev_err(hipEventSynchronize(f->ring_ev[i]), "table slot")) return rc;
  }
  *host = f->ring_host[i];
  *dev = f->ring_dev[i];
  return i;
}

uint64_t sub_mask(const Sub& S) {
  uint64_t m = 0;
  for (int b = 0; b < S.nq; ++b) m |= uint64_t(1) << S.q[b];
  return m;
}

bool touches_dirty(const FactorState* f, const int* qubits, int k) {
  for (int j = 0; j < k; ++j) {
    const int si = find(f, qubits[j], nullptr);
    if (si < 0) continue;
    const Sub& S = f->subs[si];
    for (int b = 0; b < S.nq; ++b)
      if ((f->dirty >> S.q[b]) & 1) return true;
  }
  return false;
}

// The completion signal's memory, made on first use (false if unavailable:
// the caller synchronizes the stream instead).
bool signal_ready(FactorState* f) {
  if (f->sig_host) return true;
  void* h = nullptr;
  void* d = nullptr;
  if (hipHostMalloc(&h, 64, hipHostMallocMapped) != hipSuccess) return false;
  if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
    (void)hipHostFree(h);
    return false;
  }
  auto* c = static_cast<unsigned*>(device_alloc(sizeof(unsigned)));
  if (!c || hipMemsetAsync(c, 0, sizeof(unsigned), f->stream) != hipSuccess ||
      hipStreamSynchronize(f->stream) != hipSuccess) {
    device_free(c);
    (void)hipHostFree(h);
    return false;
  }
  *static_cast<volatile unsigned*>(h) = 0;
  f->sig_host = static_cast<unsigned*>(h);
  f->sig_dev = static_cast<unsigned*>(d);
  f->sig_count = c;
  f->sig_total = 0;
  f->sig_seq = 0;
  return true;
}

// Waits until the flag shows `seq`; every few thousand polls the stream is
// queried, so that an error, or a stream that finished without the signal,
// ends the wait.
int wait_signal(FactorState* f, unsigned seq) {
  for (uint64_t i = 1;; ++i) {
    if (__atomic_load_n(static_cast<volatile unsigned*>(f->sig_host), __ATOMIC_ACQUIRE) == seq)
      return QS_OK;
    if ((i & 4095) == 0) {
      const hipError_t q = hipStreamQuery(f->stream);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) return dev_err(q, "bloch");
      if (__atomic_load_n(static_cast<volatile unsigned*>(f->sig_host), __ATOMIC_ACQUIRE) == seq)
        return QS_OK;
      return ffail(QS_E_DEVICE, "batched sweep finished without its completion signal");
    }
  }
}

// One round of deferred tests: for every subsystem with dirty qubits, up to
// kMultiTest of them (the lowest, ascending). Sweeps of subsystems of at most
// 2^kBlochBatchQubits amplitudes share one launch; larger ones keep their own
// launches; then one synchronization. The sums are those the one-at-a-time
// sweeps compute (same kernels' order), so the decisions are too.
template <typename R>
int flush_round(FactorState* f, bool* any) {
  struct Item {
    int si, G;                         // G = 0: the subsystem's pending pair test
    int q[kMultiTest], t[kMultiTest];  // ascending qubit number (pair: q[0..1], t[0..1])
  };
  // learned schedule: the subsystems of at least propose_min qubits (not
  // under a plain retest) send their unscored dirty qubits to the network;
  // the ones below the cutoff leave the dirty set (deferred)
  auto learned = [f](const Sub& S) {
    return f->proposer && !S.plain && S.nq >= f->propose_min;
  };
  if (f->proposer) {
    std::vector<int> cand;
    for (const Sub& S : f->subs)
      if (learned(S))
        for (int b = 0; b < S.nq; ++b)
          if (((f->dirty & ~f->prop) >> S.q[b]) & 1) cand.push_back(S.q[b]);
    if (!cand.empty()) {
      std::vector<float> X(cand.size() * QS_MLP_INPUTS), score(cand.size());
      for (size_t i = 0; i < cand.size(); ++i)
        fact_features(f, cand[i], f->p, &X[i * QS_MLP_INPUTS]);
      if (int rc = mlp_scores(f->proposer, X.data(), cand.size(), score.data())) return rc;
      for (size_t i = 0; i < cand.size(); ++i) {
        const uint64_t bit = uint64_t(1) << cand[i];
        if (score[i] >= f->cutoff) {
          f->prop |= bit;
        } else {
          f->dirty &= ~bit;
          f->deferred |= bit;
          ++f->skipped;
        }
      }
    }
  }
  std::vector<Item> items;
  for (int si = 0; si < int(f->subs.size()); ++si) {
    const Sub& S = f->subs[si];
    const uint64_t want = learned(S) ? (f->dirty & f->prop) : f->dirty;
    int qd[64], td[64], nd = 0;
    for (int b = 0; b < S.nq; ++b)
      if ((want >> S.q[b]) & 1) {
        qd[nd] = S.q[b];
        td[nd++] = b;
      }
    if (!nd && S.pend_a >= 0 && !(f->dirty & sub_mask(S))) {
      // the one-qubit tests are done: the pair test its gate made due, when
      // both operands still share this subsystem of three or more qubits
      int ta = -1, tb = -1;
      for (int b = 0; b < S.nq; ++b) {
        if (S.q[b] == S.pend_a) ta = b;
        if (S.q[b] == S.pend_b) tb = b;
      }
      if (ta >= 0 && tb >= 0 && S.nq >= 3) {
        Item it{};
        it.si = si;
        it.G = 0;
        it.q[0] = S.pend_a;
        it.q[1] = S.pend_b;
        it.t[0] = ta;
        it.t[1] = tb;
        items.push_back(it);
      } else {
        f->subs[si].pend_a = f->subs[si].pend_b = -1;
      }
      continue;
    }
    if (!nd) continue;
    if (S.nq == 1) {  // nothing to separate from
      f->dirty &= ~(uint64_t(1) << S.q[0]);
      f->deferred &= ~(uint64_t(1) << S.q[0]);
      continue;
    }
    int ord[64];
    for (int i = 0; i < nd; ++i) ord[i] = i;
    std::sort(ord, ord + nd, [&](int x, int y) { return qd[x] < qd[y]; });
    Item it{};
    it.si = si;
    it.G = std::min(nd, g_multi_test ? kMultiTest : 1);
    for (int i = 0; i < it.G; ++i) {
      it.q[i] = qd[ord[i]];
      it.t[i] = td[ord[i]];
    }
    items.push_back(it);
  }
  *any = !items.empty();
  if (items.empty()) return QS_OK;
  constexpr int kRow = 4 * kMultiTest;  // stat doubles per item
  if (int(items.size()) * kRow > FactorState::kStatDoubles)
    return ffail(QS_E_UNSUPPORTED, "too many pending subsystems (%zu)", items.size());
  // kernel bit order (ascending local bit) of every item
  int bits[64][kMultiTest], pos[64][kMultiTest];
  for (size_t i = 0; i < items.size(); ++i) {
    const Item& it = items[i];
    if (it.G == 0) continue;
    int o[kMultiTest];
    for (int j = 0; j < it.G; ++j) o[j] = j;
    std::sort(o, o + it.G, [&](int x, int y) { return it.t[x] < it.t[y]; });
    for (int j = 0; j < it.G; ++j) {
      bits[i][j] = it.t[o[j]];
      pos[i][o[j]] = j;  // row of qubit j in the kernel's output
    }
  }
  // small subsystems: one launch over a table in a pinned slot; when that
  // launch is the whole round, its completion flag replaces the stream sync
  bool only_small = true, all_small = true;  // (only_small: and no pair test)
  int npair = 0;
  for (const Item& it : items) {
    if (f->subs[it.si].nq > kBlochBatchQubits) all_small = false;
    if (it.G == 0) {
      only_small = false;
      ++npair;
    }
  }
  only_small = only_small && all_small;
  // one-workgroup launches only: each workgroup counts itself, the last one
  // raises the flag
  const bool signal = all_small && g_done_flag && signal_ready(f);
  // The queued operations (the merges and projections that produced the
  // subsystems about to be swept) run in the sweep's launch when every one of
  // them writes a small subsystem of this round, which it then precedes in
  // its workgroup; otherwise they are launched first.
  constexpr size_t kOpsAt = 2048;  // byte offset of the operations in the slot
  static_assert(kOpsAt >= size_t(kMaxSweepItems) * sizeof(BlochItem<R>), "slot layout");
  std::vector<int> op_of(items.size(), -1);
  bool fuse = g_fuse_ops && only_small && !f->qops.empty() &&
              f->qops.size() <= (FactorState::kSlotBytes - kOpsAt) / sizeof(FactOp<R>);
  for (size_t k = 0; fuse && k < f->qops.size(); ++k) {
    const FactorState::QOp& q = f->qops[k];
    int hit = -1;
    for (size_t i = 0; i < items.size() && hit < 0; ++i)
      if (f->subs[items[i].si].amps == q.c) hit = int(i);
    if (q.na + q.nb > kFactOpQubits || hit < 0 || op_of[hit] >= 0) {
      fuse = false;
      break;
    }
    op_of[hit] = int(k);
  }
  if (!fuse) {
    if (int rc = launch_queue(f)) return rc;  // the sweeps read the queued results
    std::fill(op_of.begin(), op_of.end(), -1);
  }
  void *host = nullptr, *dev = nullptr;
  int slot = -1, nsmall = 0;
  for (size_t i = 0; i < items.size(); ++i) {
    const Sub& S = f->subs[items[i].si];
    if (items[i].G == 0 || S.nq > kBlochBatchQubits) continue;
    if (slot < 0) {
      slot = ring_slot(f, &host, &dev);
      if (slot < 0) return slot;
    }
    BlochItem<R>& b = static_cast<BlochItem<R>*>(host)[nsmall++];
    b.amps = static_cast<const R*>(S.amps);
    b.nq = S.nq;
    b.G = items[i].G;
    for (int j = 0; j < kMultiTest; ++j) b.bits[j] = j < b.G ? bits[i][j] : 0;
    b.out = int(i) * kRow;
    b.op = op_of[i];
  }
  FactOp<R>* hops = nullptr;
  if (fuse) {
    hops = reinterpret_cast<FactOp<R>*>(static_cast<char*>(host) + kOpsAt);
    for (size_t k = 0; k < f->qops.size(); ++k) fill_op(f->qops[k], &hops[k]);
  }
  hipError_t e = hipSuccess;
  unsigned seq = 0, target = 0;
  unsigned* counter = nullptr;
  if (signal) {
    seq = ++f->sig_seq;
    f->sig_total += unsigned(nsmall + npair);
    counter = f->sig_count;
    target = f->sig_total;
  }
  if (nsmall) {
    e = fuse ? launch_ops_bloch(static_cast<const BlochItem<R>*>(host),
                                static_cast<const BlochItem<R>*>(dev), nsmall, hops,
                                reinterpret_cast<const FactOp<R>*>(static_cast<char*>(dev) + kOpsAt),
                                int(f->qops.size()), f->dstat, counter, f->sig_dev, target, seq,
                                f->stream)
             : launch_bloch_batch(static_cast<const BlochItem<R>*>(host),
                                  static_cast<const BlochItem<R>*>(dev), nsmall, f->dstat, counter,
                                  f->sig_dev, target, seq, f->stream);
    if (e == hipSuccess) e = hipEventRecord(f->ring_ev[slot], f->stream);
    if (e == hipSuccess) f->ring_used[slot] = true;
    if (fuse) finish_queue(f);  // launched; buffers freed meanwhile go back
  }
  for (size_t i = 0; i < items.size() && e == hipSuccess; ++i) {
    const Sub& S = f->subs[items[i].si];
    const R* a = static_cast<const R*>(S.amps);
    if (items[i].G == 0) {
      e = launch_pair_rho(a, S.nq, items[i].t[0], items[i].t[1], f->scratch, f->dstat + i * kRow,
                          counter, f->sig_dev, target, seq, f->stream);
      continue;
    }
    if (S.nq <= kBlochBatchQubits) continue;
    e = items[i].G == 1
            ? launch_bloch(a, S.nq, bits[i][0], f->scratch, f->dstat + i * kRow, f->stream)
            : launch_bloch_multi(a, S.nq, bits[i], items[i].G, f->scratch, f->dstat + i * kRow,
                                 f->stream);
  }
  if (int rc = dev_err(e, "bloch")) return rc;
  if (signal) {
    if (int rc = wait_signal(f, seq)) return rc;
  } else if (int rc = dev_err(hipStreamSynchronize(f->stream), "bloch")) {
    return rc;
  }
  // decisions per subsystem, ascending qubit number, stopping at a rounding
  for (size_t i = 0; i < items.size(); ++i) {
    const Item& it = items[i];
    f->cur_phase = f->subs[it.si].phase;
    f->cur_gates = f->subs[it.si].phase_gates;
    if (it.G == 0) {
      f->subs[it.si].pend_a = f->subs[it.si].pend_b = -1;
      bool rounded = false;
      if (int rc = decide_pair(f, it.si, it.q[0], it.q[1], it.t[0], it.t[1], f->hstat + i * kRow,
                               f->p, &rounded))
        return rc;
      continue;
    }
    for (int j = 0; j < it.G; ++j) {
      const double* st = f->hstat + i * kRow + 4 * pos[i][j];
      const double sums[4] = {st[0], st[1], st[2], st[3]};
      begin_test(f, it.q[j], f->p);
      bool rounded = false;
      if (int rc = decide_qubit(f, it.q[j], it.si, it.t[j], sums, f->p, &rounded)) return rc;
      if (rounded) {  // the subsystem's remaining qubits are dirty and unscored again
        const Sub& S = f->subs[it.si];
        for (int b = 0; b < S.nq; ++b) f->prop &= ~(uint64_t(1) << S.q[b]);
        break;
      }
    }
  }
  return QS_OK;
}

template <typename R>
void fill_op(const FactorState::QOp& q, FactOp<R>* o) {
  o->a = static_cast<const R*>(q.a);
  o->b = static_cast<const R*>(q.b);
  o->c = static_cast<R*>(q.c);
  o->single = static_cast<R*>(q.single);
  o->kind = q.kind;
  o->na = q.na;
  o->nb = q.nb;
  o->t0 = q.t0;
  o->t1 = q.t1;
  o->pad = 0;
  for (int k = 0; k < 4; ++k) o->phi[k] = q.phi[k];
  o->scale = q.scale;
  for (int k = 0; k < 32; ++k) o->m[k] = R(q.m[k]);
}

// The queue has been launched: forget it, and return the buffers freed while
// it was pending.
void finish_queue(FactorState* f) {
  f->qops.clear();
  std::vector<std::pair<int, void*>> late;
  late.swap(f->late_free);
  for (const auto& b : late) sub_free(f, b.first, b.second);
}

template <typename R>
int launch_queue_t(FactorState* f) {
  constexpr size_t kPerSlot = FactorState::kSlotBytes / sizeof(FactOp<R>);
  std::vector<const FactorState::QOp*> small, large;
  for (const auto& op : f->qops)
    (op.na + op.nb <= kFactOpQubits ? small : large).push_back(&op);
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < small.size() && e == hipSuccess; i += kPerSlot) {
    void *host = nullptr, *dev = nullptr;
    const int slot = ring_slot(f, &host, &dev);
    if (slot < 0) return slot;
    const size_t cnt = std::min(kPerSlot, small.size() - i);
    auto* ops = static_cast<FactOp<R>*>(host);
    for (size_t j = 0; j < cnt; ++j) fill_op(*small[i + j], &ops[j]);
    e = launch_fact_ops(static_cast<const FactOp<R>*>(host), static_cast<const FactOp<R>*>(dev),
                        int(cnt), f->stream);
    if (e == hipSuccess) e = hipEventRecord(f->ring_ev[slot], f->stream);
    if (e == hipSuccess) f->ring_used[slot] = true;
  }
  for (size_t i = 0; i < large.size() && e == hipSuccess; ++i) {
    const FactorState::QOp& q = *large[i];
    if (q.kind == 1) {
      e = launch_decompose(static_cast<R*>(q.c), static_cast<const R*>(q.a), q.na, q.t0, q.phi,
                           q.scale, f->stream);
      if (e == hipSuccess) e = launch_store_single(static_cast<R*>(q.single), q.phi, f->stream);
      continue;
    }
    e = launch_merge_gate(static_cast<R*>(q.c), static_cast<const R*>(q.a), q.na,
                          static_cast<const R*>(q.b), q.nb, q.t0, q.t1, q.m, f->stream);
  }
  return dev_err(e, "queued subsystem operations");
}

// Launches the queued operations, then returns the buffers freed meanwhile.
int launch_queue(FactorState* f) {
  if (f->qops.empty()) return QS_OK;
  const int rc = f->dtype == QS_C64 ? launch_queue_t<float>(f) : launch_queue_t<double>(f);
  finish_queue(f);
  return rc;
}

// Runs every deferred test, then logs the attempts and applies the fidelity
// factors in the order of the gates that caused them.
int flush_pending(FactorState* f) {
  f->flushing = true;
  int rc = QS_OK;
  for (bool any = true; any && rc == QS_OK;)  // until no test (one-qubit or pair) is due
    rc = f->dtype == QS_C64 ? flush_round<float>(f, &any) : flush_round<double>(f, &any);
  if (rc == QS_OK) rc = launch_queue(f);  // the last projections
  f->flushing = false;
  for (auto& S : f->subs) S.plain = false;
  std::vector<size_t> order(f->pend.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [f](size_t a, size_t b) { return f->pend[a].phase < f->pend[b].phase; });
  const bool feats = f->feat_log && f->pend_feat.size() == f->pend.size() * QS_MLP_INPUTS;
  for (size_t i : order) {
    const FactorState::Decision& d = f->pend[i];
    if (feats && f->log_count && *f->log_count < f->feat_cap)
      std::memcpy(f->feat_log + *f->log_count * QS_MLP_INPUTS, &f->pend_feat[i * QS_MLP_INPUTS],
                  QS_MLP_INPUTS * sizeof(float));
    if (d.rounded) f->F *= (1.0 - d.eps);
    log_attempt(f, d.q, d.nsub, d.eps, d.rounded, d.partner, d.gates);
  }
  f->pend.clear();
  f->pend_feat.clear();
  return rc;
}

// The one-qubit gates `list` (indices into qubits/m, in order) on the large
// subsystem si: as tile passes when it holds a whole tile (each pass reads
// and writes the subsystem once for all the gates on its 12 tile bits), else
// one launch per gate. Plan tables go to a device buffer of the state through
// a pinned slot.
template <typename R>
int large_1q_run(FactorState* f, int si, const int* qubits, const double* m,
                 const std::vector<int>& list) {
  const Sub& S = f->subs[si];
  R* amps = static_cast<R*>(S.amps);
  constexpr int kLow = 5;  // tile low bits (both precisions)
  auto local_bit = [&S](int q) {
    for (int b = 0; b < S.nq; ++b)
      if (S.q[b] == q) return b;
    return -1;
  };
  if (g_tile_1q && list.size() >= 2 && S.nq >= kLow + kTileRowBits) {
    std::vector<Gate> gl(list.size());
    for (size_t i = 0; i < list.size(); ++i) {
      Gate& g = gl[i];
      g.k = 1;
      g.q[0] = local_bit(qubits[list[i]]);
      g.m.resize(4);
      for (int e = 0; e < 4; ++e)
        g.m[e] = cd(m[8 * list[i] + 2 * e], m[8 * list[i] + 2 * e + 1]);
    }
    const TilePlan pl = plan_tiles(gl, S.nq, kLow, kTileRowBits, 4, false);
    std::vector<unsigned char> tab;
    size_t goff = 0, moff = 0, eoff = 0;
    tile_tables(pl, sizeof(R) == 4, &tab, &goff, &moff, &eoff);
    if (tab.size() <= FactorState::kSlotBytes) {
      if (tab.size() > f->tile_cap) {
        if (int rc = dev_err(hipStreamSynchronize(f->stream), "tile tables")) return rc;
        device_free(f->tile_dev);
        f->tile_cap = 0;
        f->tile_dev = device_alloc(FactorState::kSlotBytes);
        if (!f->tile_dev) return ffail(QS_E_NOMEM, "tile tables");
        f->tile_cap = FactorState::kSlotBytes;
      }
      void *host = nullptr, *dev = nullptr;
      const int slot = ring_slot(f, &host, &dev);
      if (slot < 0) return slot;
      std::memcpy(host, tab.data(), tab.size());
      hipError_t e =
          hipMemcpyAsync(f->tile_dev, host, tab.size(), hipMemcpyHostToDevice, f->stream);
      if (e == hipSuccess) e = hipEventRecord(f->ring_ev[slot], f->stream);
      if (e == hipSuccess) f->ring_used[slot] = true;
      const char* base = static_cast<const char*>(f->tile_dev);
      for (const TileStep& st : pl.steps) {
        if (e != hipSuccess) break;
        if (st.block) {  // not made from one-qubit gates
          e = hipErrorInvalidValue;
          break;
        }
        TileRows rows;
        for (int j = 0; j < kTileRowBits; ++j) rows.b[j] = st.hb[j];
        e = launch_tile_pass(amps, S.nq, kLow, rows, base + size_t(st.r0) * 4 * sizeof(int32_t),
                             st.nr, base + goff, reinterpret_cast<const R*>(base + moff),
                             f->stream);
      }
      return dev_err(e, "one-qubit tile passes");
    }
  }
  for (int i : list) {
    Mat2<R> mm;
    for (int e = 0; e < 4; ++e) {
      mm.re[e] = R(m[8 * i + 2 * e]);
      mm.im[e] = R(m[8 * i + 2 * e + 1]);
    }
    if (int rc = dev_err(launch_apply_1q(amps, S.nq, local_bit(qubits[i]), mm, f->stream),
                         "factorized gate"))
      return rc;
  }
  return QS_OK;
}

template <typename R>
int apply_1q_run(FactorState* f, const int* qubits, const double* m, int count) {
  // the gates of each small subsystem, in circuit order
  std::vector<int> item_of(f->subs.size(), -1);
  std::vector<std::vector<int>> per_item;
  std::vector<int> item_sub;
  std::vector<int> large_of(f->subs.size(), -1);
  std::vector<std::vector<int>> per_large;  // the gates of each large subsystem
  std::vector<int> large_sub;
  for (int i = 0; i < count; ++i) {
    int t = 0;
    const int si = find(f, qubits[i], &t);
    if (si < 0) return ffail(QS_E_INVAL, "qubit %d not found", qubits[i]);
    if (!f->mirrors_ahead) mirror_1q(f->subs[si], m + 8 * i);
    if (f->subs[si].nq > kFact1qMaxQubits) {
      if (large_of[si] < 0) {
        large_of[si] = int(per_large.size());
        per_large.emplace_back();
        large_sub.push_back(si);
      }
      per_large[large_of[si]].push_back(i);
      continue;
    }
    if (item_of[si] < 0) {
      item_of[si] = int(per_item.size());
      per_item.emplace_back();
      item_sub.push_back(si);
    }
    per_item[item_of[si]].push_back(i);
  }
  // Tables in slots: up to kItems items at the start, their gates after. An
  // item whose gates do not all fit continues in the next launch, which the
  // stream runs after this one, so every subsystem sees its gates in order.
  constexpr size_t kItems = 512;
  constexpr size_t kGatesAt = kItems * sizeof(Fact1qItem<R>);
  constexpr size_t kGates = (FactorState::kSlotBytes - kGatesAt) / sizeof(Fact1qGate<R>);
  static_assert(kGatesAt % 64 == 0 && kGates >= 64, "slot layout");
  size_t j = 0, o = 0;  // next item, and how many of its gates are already out
  while (j < per_item.size()) {
    void *host = nullptr, *dev = nullptr;
    const int slot = ring_slot(f, &host, &dev);
    if (slot < 0) return slot;
    auto* items = static_cast<Fact1qItem<R>*>(host);
    auto* gates = reinterpret_cast<Fact1qGate<R>*>(static_cast<char*>(host) + kGatesAt);
    size_t nit = 0, ng = 0;
    int max_nq = 1;
    while (j < per_item.size() && nit < kItems && ng < kGates) {
      const Sub& S = f->subs[item_sub[j]];
      max_nq = std::max(max_nq, S.nq);
      const std::vector<int>& list = per_item[j];
      const size_t take = std::min(list.size() - o, kGates - ng);
      Fact1qItem<R>& it = items[nit++];
      it.amps = static_cast<R*>(S.amps);
      it.nq = S.nq;
      it.g0 = int(ng);
      it.ng = int(take);
      it.pad = 0;
      for (size_t x = 0; x < take; ++x) {
        const int gi = list[o + x];
        int t = 0;
        find(f, qubits[gi], &t);
        Fact1qGate<R>& gt = gates[ng++];
        for (int e = 0; e < 8; ++e) gt.m[e] = R(m[8 * gi + e]);
        gt.t = t;
        gt.pad = 0;
      }
      o += take;
      if (o == list.size()) {
        ++j;
        o = 0;
      }
    }
    hipError_t e = launch_fact_1q_batch(
        items, static_cast<const Fact1qItem<R>*>(dev), int(nit), gates,
        reinterpret_cast<const Fact1qGate<R>*>(static_cast<char*>(dev) + kGatesAt), int(ng),
        max_nq, f->stream);
    if (e == hipSuccess) e = hipEventRecord(f->ring_ev[slot], f->stream);
    if (int rc = dev_err(e, "batched one-qubit gates")) return rc;
    f->ring_used[slot] = true;
  }
  for (size_t l = 0; l < per_large.size(); ++l)
    if (int rc = large_1q_run<R>(f, large_sub[l], qubits, m, per_large[l])) return rc;
  return QS_OK;
}

}  // namespace

int fact_apply_1q_run(FactorState* f, const int* qubits, const double* m, int count) {
  if (f->defer && f->dirty && touches_dirty(f, qubits, count))
    if (int rc = flush_pending(f)) return rc;
  if (int rc = launch_queue(f)) return rc;
  if (!g_batch_1q || count < 2) {
    for (int i = 0; i < count; ++i)
      if (int rc = fact_apply(f, qubits + i, 1, m + 8 * i)) return rc;
    return QS_OK;
  }
  return f->dtype == QS_C64 ? apply_1q_run<float>(f, qubits, m, count)
                            : apply_1q_run<double>(f, qubits, m, count);
}

int fact_block(const FactorState* f, int start, int len, int* t0, bool* descending) {
  if (len < 2) return -1;
  int ta = 0, tb = 0;
  const int si = find(f, start, &ta);
  if (si < 0 || find(f, start + len - 1, &tb) != si) return -1;
  const Sub& S = f->subs[si];
  const bool up = tb == ta + len - 1, down = ta == tb + len - 1;
  if (!up && !down) return -1;
  const int lo = up ? ta : tb;
  for (int i = 0; i < len; ++i)
    if (S.q[lo + i] != (up ? start + i : start + len - 1 - i)) return -1;
  *t0 = lo;
  *descending = down;
  return si;
}

int fact_sync(FactorState* f) { return launch_queue(f); }

void fact_begin_run(FactorState* f) {
  f->defer = g_defer_sep &&
             (f->policy == QS_SEP_AFTER_2Q || f->policy == QS_SEP_AFTER_2Q_PAIRS) && !f->dirty;
  f->prop = 0;
}

int fact_end_run(FactorState* f, int rc) {
  int frc = QS_OK;
  if (f->defer && rc != QS_E_DEVICE) {
    if (f->dirty) frc = flush_pending(f);
    if (frc == QS_OK) frc = launch_queue(f);
  }
  if (!f->qops.empty()) {  // a device error: nothing more runs on this state
    f->qops.clear();
    std::vector<std::pair<int, void*>> late;
    late.swap(f->late_free);
    for (const auto& b : late) sub_free(f, b.first, b.second);
  }
  f->defer = false;
  return rc != QS_OK ? rc : frc;
}

int fact_swap(FactorState* f, int a, int b) {
  if (f->defer && f->dirty)
    if (int rc = flush_pending(f)) return rc;
  for (auto& s : f->subs)
    for (int t = 0; t < s.nq; ++t) {
      if (s.q[t] == a) s.q[t] = b;
      else if (s.q[t] == b) s.q[t] = a;
    }
  for (uint64_t* mask : {&f->dirty, &f->deferred}) {
    const uint64_t da = (*mask >> a) & 1, db = (*mask >> b) & 1;
    *mask &= ~((uint64_t(1) << a) | (uint64_t(1) << b));
    *mask |= (da << b) | (db << a);
  }
  std::swap(f->eps_last[a], f->eps_last[b]);
  std::swap(f->eps_prev[a], f->eps_prev[b]);
  std::swap(f->rounded_last[a], f->rounded_last[b]);
  std::swap(f->tests[a], f->tests[b]);
  std::swap(f->gates_since[a], f->gates_since[b]);
  std::swap(f->merged_last[a], f->merged_last[b]);
  std::swap(f->partner[a], f->partner[b]);
  for (int& pq : f->partner) pq = pq == a ? b : (pq == b ? a : pq);
  return QS_OK;
}

int fact_relabel(FactorState* f, const int* pos) {
  if (f->defer && f->dirty)
    if (int rc = flush_pending(f)) return rc;
  int inv[64];
  for (int q = 0; q < f->n; ++q) inv[pos[q]] = q;
  uint64_t nd = 0, nf = 0;
  for (int q = 0; q < f->n; ++q) {
    if ((f->dirty >> pos[q]) & 1) nd |= uint64_t(1) << q;
    if ((f->deferred >> pos[q]) & 1) nf |= uint64_t(1) << q;
  }
  for (auto& s : f->subs)
    for (int t = 0; t < s.nq; ++t) s.q[t] = inv[s.q[t]];
  f->dirty = nd;
  f->deferred = nf;
  // per-qubit history follows its qubit: label v becomes inv[v]
  auto moved = [&](auto& v) {
    auto old = v;
    for (int q = 0; q < f->n; ++q) v[q] = old[pos[q]];
  };
  moved(f->eps_last);
  moved(f->eps_prev);
  moved(f->rounded_last);
  moved(f->tests);
  moved(f->gates_since);
  moved(f->merged_last);
  moved(f->partner);
  for (int& pq : f->partner) pq = pq >= 0 ? inv[pq] : pq;
  return QS_OK;
}

int fact_try_separate(FactorState* f, double p, int* n_separated) {
  int count = 0;
  const int rc = f->proposer ? proposed_separate(f, p, &count) : plain_separate(f, p, &count);
  if (n_separated) *n_separated = count;
  return rc;
}

int fact_gather(FactorState* f, const uint64_t* idx, uint64_t m, double* out) {
  uint64_t* didx = static_cast<uint64_t*>(device_alloc(m * sizeof(uint64_t)));
  double* dout = static_cast<double*>(device_alloc(m * 2 * sizeof(double)));
  if (!didx || !dout) {
    device_free(didx);
    device_free(dout);
    return ffail(QS_E_NOMEM, "staging allocation failed");
  }
  std::vector<double> ones(2 * m, 0.0);
  for (uint64_t j = 0; j < m; ++j) ones[2 * j] = 1.0;
  hipError_t e = hipMemcpyAsync(didx, idx, m * sizeof(uint64_t), hipMemcpyHostToDevice, f->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(dout, ones.data(), m * 2 * sizeof(double), hipMemcpyHostToDevice, f->stream);
  for (size_t s = 0; s < f->subs.size() && e == hipSuccess; ++s) {
    Perm64 bits{};
    bits.n = f->subs[s].nq;
    for (int t = 0; t < bits.n; ++t) bits.p[t] = int8_t(f->subs[s].q[t]);
    e = f->dtype == QS_C64
            ? launch_gather_mul(static_cast<const float*>(f->subs[s].amps), didx, m, bits, dout, f->stream)
            : launch_gather_mul(static_cast<const double*>(f->subs[s].amps), didx, m, bits, dout, f->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, dout, m * 2 * sizeof(double), hipMemcpyDeviceToHost, f->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
  device_free(didx);
  device_free(dout);
  return dev_err(e, "factorized gather");
}

int fact_norm(FactorState* f, double* out) {
  double prod = 1.0;
  for (auto& s : f->subs) {
    hipError_t e = f->dtype == QS_C64
                       ? launch_inner(static_cast<const float*>(s.amps), static_cast<const float*>(s.amps),
                                      uint64_t(1) << s.nq, f->scratch, f->stream)
                       : launch_inner(static_cast<const double*>(s.amps), static_cast<const double*>(s.amps),
                                      uint64_t(1) << s.nq, f->scratch, f->stream);
    double v[2];
    if (e == hipSuccess) e = hipMemcpyAsync(v, f->scratch, sizeof v, hipMemcpyDeviceToHost, f->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
    if (int rc = dev_err(e, "norm")) return rc;
    prod *= v[0];
  }
  *out = prod;
  return QS_OK;
}

int fact_expand(FactorState* f, void* dense, int* perm_out) {
  const size_t ab = amp_bytes(f);
  void* tmp = device_alloc((size_t(1) << f->n) * ab);
  if (!tmp) return ffail(QS_E_NOMEM, "expansion buffer");
  // compose subsystems one after another, alternating between two buffers so
  // that the last compose lands in `dense`
  const int ns = int(f->subs.size());
  void* bufs[2] = {dense, tmp};
  int cur = (ns - 1) % 2;  // buffer holding the running product
  hipError_t e = hipMemcpyAsync(bufs[cur], f->subs[0].amps, (size_t(1) << f->subs[0].nq) * ab,
                                hipMemcpyDeviceToDevice, f->stream);
  int nq = f->subs[0].nq, bit = 0;
  for (int t = 0; t < f->subs[0].nq; ++t) perm_out[f->subs[0].q[t]] = bit++;
  for (int s = 1; s < ns && e == hipSuccess; ++s) {
    const Sub& B = f->subs[s];
    void* dst = bufs[1 - cur];
    e = f->dtype == QS_C64
            ? launch_compose(static_cast<float*>(dst), static_cast<const float*>(bufs[cur]), nq,
                             static_cast<const float*>(B.amps), B.nq, f->stream)
            : launch_compose(static_cast<double*>(dst), static_cast<const double*>(bufs[cur]), nq,
                             static_cast<const double*>(B.amps), B.nq, f->stream);
    for (int t = 0; t < B.nq; ++t) perm_out[B.q[t]] = bit++;
    nq += B.nq;
    cur = 1 - cur;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(f->stream);
  device_free(tmp);
  return dev_err(e, "expand");
}

}  // namespace qs
