// Circuit object and gate-fusion planner (host C++, float64).
//
// A random-circuit layer (Sec. III-C) is U(theta, phi, lambda) on every qubit
// followed by two-qubit couplers; applying each gate as its own HBM sweep costs
// one read and write of the whole ket per gate. The planner groups consecutive
// gates that act on at most kmax distinct qubits into one dense block whose
// matrix (the product of its gates, float64) is applied in a single sweep.
// SWAP gates never move data: they rename the positions later gates act on,
// and the circuit ends with that renaming applied to the state's labels
// (Table I: SWAP by qubit label swap).
#include <algorithm>
#include <cstring>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "circuit.h"
#include "qs_internal.h"

namespace qs {

namespace {

std::vector<cd> eye(int k) {
  const int d = 1 << k;
  std::vector<cd> m(size_t(d) * d, cd(0, 0));
  for (int i = 0; i < d; ++i) m[size_t(i) * d + i] = 1.0;
  return m;
}

// U(theta, phi, lambda) of Sec. III-C.
std::vector<cd> u3(double t, double p, double l) {
  const double c = std::cos(t / 2), s = std::sin(t / 2);
  return {cd(c, 0), -std::polar(1.0, l) * s, std::polar(1.0, p) * s, std::polar(1.0, p + l) * c};
}

// Two-qubit controlled 2x2: local bit 0 = control, bit 1 = target; acts when
// the control equals `cv`.
std::vector<cd> controlled(const std::vector<cd>& u, int cv) {
  std::vector<cd> m = eye(2);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) m[size_t(cv + 2 * i) * 4 + (cv + 2 * j)] = u[size_t(i) * 2 + j];
  return m;
}

}  // namespace

bool gate_matrix(int kind, int nq, const double* p, std::vector<cd>* m, int* k_out) {
  const double r2 = 1.0 / std::sqrt(2.0);
  const std::vector<cd> X = {0.0, 1.0, 1.0, 0.0};
  const std::vector<cd> Y = {0.0, cd(0, -1), cd(0, 1), 0.0};
  const std::vector<cd> Z = {1.0, 0.0, 0.0, -1.0};
  int k = 0;
  switch (kind) {
    case QS_GATE_H: k = 1; *m = {r2, r2, r2, -r2}; break;
    case QS_GATE_X: k = 1; *m = X; break;
    case QS_GATE_Y: k = 1; *m = Y; break;
    case QS_GATE_Z: k = 1; *m = Z; break;
    case QS_GATE_U3: k = 1; *m = u3(p[0], p[1], p[2]); break;
    case QS_GATE_CZ: k = 2; *m = eye(2); (*m)[15] = -1.0; break;
    case QS_GATE_CP: k = 2; *m = eye(2); (*m)[15] = std::polar(1.0, p[0]); break;
    case QS_GATE_ISWAP:
      k = 2;
      *m = eye(2);
      (*m)[1 * 4 + 1] = 0.0; (*m)[2 * 4 + 2] = 0.0;
      (*m)[1 * 4 + 2] = cd(0, 1); (*m)[2 * 4 + 1] = cd(0, 1);
      break;
    case QS_GATE_SWAP:
      k = 2;
      *m = eye(2);
      (*m)[1 * 4 + 1] = 0.0; (*m)[2 * 4 + 2] = 0.0;
      (*m)[1 * 4 + 2] = 1.0; (*m)[2 * 4 + 1] = 1.0;
      break;
    case QS_GATE_CX: k = 2; *m = controlled(X, 1); break;
    case QS_GATE_CY: k = 2; *m = controlled(Y, 1); break;
    case QS_GATE_AX: k = 2; *m = controlled(X, 0); break;
    case QS_GATE_AY: k = 2; *m = controlled(Y, 0); break;
    case QS_GATE_AZ: k = 2; *m = controlled(Z, 0); break;
    case QS_GATE_CU3:
      if (p[3] != 0.0 && p[3] != 1.0) return false;
      k = 2;
      *m = controlled(u3(p[0], p[1], p[2]), int(p[3]));
      break;
    default: return false;
  }
  if (nq != k) return false;
  *k_out = k;
  return true;
}

namespace {

// m <- g m, where g acts on the block-local bits lp[0..gk) of a k-bit block.
void left_apply(std::vector<cd>& m, int k, const std::vector<cd>& g, int gk, const int* lp) {
  const int d = 1 << k, gd = 1 << gk;
  int mask = 0;
  for (int j = 0; j < gk; ++j) mask |= 1 << lp[j];
  std::vector<cd> in(gd), out(gd);
  std::vector<int> idx(gd);
  for (int col = 0; col < d; ++col) {
    for (int base = 0; base < d; ++base) {
      if (base & mask) continue;
      for (int s = 0; s < gd; ++s) {
        int x = base;
        for (int j = 0; j < gk; ++j) x |= ((s >> j) & 1) << lp[j];
        idx[s] = x;
        in[s] = m[size_t(x) * d + col];
      }
      for (int r = 0; r < gd; ++r) {
        cd acc = 0.0;
        for (int s = 0; s < gd; ++s) acc += g[size_t(r) * gd + s] * in[s];
        out[r] = acc;
      }
      for (int s = 0; s < gd; ++s) m[size_t(idx[s]) * d + col] = out[s];
    }
  }
}

struct Open {
  bool live = true;
  std::vector<int> qubits;
  std::vector<int> gates;
};

Block build_block(const Open& o, const std::vector<Gate>& gates) {
  Block b;
  std::vector<int> q = o.qubits;
  std::sort(q.begin(), q.end());
  b.k = int(q.size());
  for (int j = 0; j < b.k; ++j) b.q[j] = q[j];
  b.m = eye(b.k);
  b.ngates = int(o.gates.size());
  for (int gi : o.gates) {
    const Gate& g = gates[gi];
    int lp[QS_MAX_FUSED];
    for (int j = 0; j < g.k; ++j)
      lp[j] = int(std::lower_bound(q.begin(), q.end(), g.q[j]) - q.begin());
    left_apply(b.m, b.k, g.m, g.k, lp);
  }
  return b;
}

}  // namespace

std::vector<Block> fuse(const std::vector<Gate>& gates, int n, int kmax) {
  std::vector<Open> open;
  std::vector<int> owner(n, -1);
  std::vector<Block> out;
  auto emit = [&](int b) {
    out.push_back(build_block(open[b], gates));
    for (int q : open[b].qubits) owner[q] = -1;
    open[b].live = false;
  };
  for (int gi = 0; gi < int(gates.size()); ++gi) {
    const Gate& g = gates[gi];
    std::vector<int> touched;
    std::vector<int> uni(g.q, g.q + g.k);
    for (int j = 0; j < g.k; ++j) {
      const int b = owner[g.q[j]];
      if (b >= 0 && std::find(touched.begin(), touched.end(), b) == touched.end()) {
        touched.push_back(b);
        for (int q : open[b].qubits)
          if (std::find(uni.begin(), uni.end(), q) == uni.end()) uni.push_back(q);
      }
    }
    Open nb;
    if (int(uni.size()) <= kmax) {
      // merge: the touched blocks act on disjoint qubits, so their gate lists
      // may be concatenated in any order before this gate
      std::sort(touched.begin(), touched.end());
      for (int b : touched) {
        nb.gates.insert(nb.gates.end(), open[b].gates.begin(), open[b].gates.end());
        open[b].live = false;
      }
      nb.qubits = uni;
    } else {
      std::sort(touched.begin(), touched.end());
      for (int b : touched) emit(b);
      nb.qubits.assign(g.q, g.q + g.k);
    }
    nb.gates.push_back(gi);
    open.push_back(nb);
    for (int q : open.back().qubits) owner[q] = int(open.size()) - 1;
  }
  for (int b = 0; b < int(open.size()); ++b)
    if (open[b].live) emit(b);
  return out;
}

namespace {

// The gates of `sel` (indices into `qb`, the qubit lists) taken in rounds of
// the dependence order: each call returns the gates of one group whose
// qubits, together with `fixed`, need at most `budget` extra qubits; `done`
// marks the gates already taken. Qubits in `fixed` are free.
struct DagCursor {
  const std::vector<std::vector<int>>* qb = nullptr;
  std::vector<std::vector<int>> per_qubit;  // gate positions (into sel) per qubit
  std::vector<size_t> next;                 // per qubit: index into per_qubit
  std::vector<char> done;
  size_t remaining = 0;

  DagCursor(const std::vector<std::vector<int>>& q, int nq) : qb(&q), per_qubit(nq), next(nq, 0) {
    for (size_t i = 0; i < q.size(); ++i)
      for (int x : q[i]) per_qubit[x].push_back(int(i));
    done.assign(q.size(), 0);
    remaining = q.size();
  }
  bool at_front(int i) const {
    for (int x : (*qb)[i])
      if (next[x] >= per_qubit[x].size() || per_qubit[x][next[x]] != i) return false;
    return true;
  }
  void take(int i) {
    done[i] = 1;
    --remaining;
    for (int x : (*qb)[i]) ++next[x];
  }
  // the front in circuit order
  std::vector<int> front() const {
    std::vector<int> f;
    for (size_t x = 0; x < per_qubit.size(); ++x)
      if (next[x] < per_qubit[x].size()) {
        const int i = per_qubit[x][next[x]];
        if (at_front(i) && std::find(f.begin(), f.end(), i) == f.end()) f.push_back(i);
      }
    std::sort(f.begin(), f.end());
    return f;
  }
};

// Greedy group: front gates (circuit order) whose qubits outside `fixed`
// fit, with the qubits already chosen, in `budget`; `eligible` filters.
template <typename Eligible>
std::vector<int> take_group(DagCursor& dag, const std::vector<char>& fixed, int budget,
                            std::vector<int>* chosen, Eligible eligible) {
  std::vector<int> out;
  bool progress = true;
  while (progress) {
    progress = false;
    for (int i : dag.front()) {
      if (!eligible(i)) continue;
      std::vector<int> need;
      for (int x : (*dag.qb)[i])
        if (!fixed[x] && std::find(chosen->begin(), chosen->end(), x) == chosen->end())
          need.push_back(x);
      if (int(chosen->size() + need.size()) > budget) continue;
      chosen->insert(chosen->end(), need.begin(), need.end());
      dag.take(i);
      out.push_back(i);
      progress = true;
    }
  }
  return out;
}

}  // namespace

TilePlan plan_tiles(const std::vector<Gate>& gates, int n, int C, int H, int W, bool dense) {
  TilePlan plan;
  plan.C = C;
  plan.H = H;
  plan.W = W;
  plan.dense = dense;
  std::vector<std::vector<int>> qb(gates.size());
  for (size_t i = 0; i < gates.size(); ++i) qb[i].assign(gates[i].q, gates[i].q + gates[i].k);
  DagCursor dag(qb, n);
  std::vector<char> low(n, 0);
  for (int q = 0; q < C && q < n; ++q) low[q] = 1;
  const int max_k = dense ? W : 2;
  auto small = [&](int i) { return gates[i].k <= max_k; };
  while (dag.remaining) {
    std::vector<int> hi;
    const std::vector<int> pass = take_group(dag, low, H, &hi, small);
    if (pass.empty()) {
      // only gates on more than two qubits at the front: the first one as a block
      const int i = dag.front().front();
      dag.take(i);
      TileStep st;
      st.block = true;
      st.ngates = 1;
      std::vector<int> q(gates[i].q, gates[i].q + gates[i].k);
      std::vector<int> order(q.size());
      for (size_t j = 0; j < q.size(); ++j) order[j] = int(j);
      std::sort(q.begin(), q.end());
      st.blk.k = gates[i].k;
      for (int j = 0; j < st.blk.k; ++j) st.blk.q[j] = q[j];
      st.blk.ngates = 1;
      st.blk.m = eye(st.blk.k);
      int lp[QS_MAX_FUSED];
      for (int j = 0; j < gates[i].k; ++j)
        lp[j] = int(std::lower_bound(q.begin(), q.end(), gates[i].q[j]) - q.begin());
      left_apply(st.blk.m, st.blk.k, gates[i].m, gates[i].k, lp);
      st.mat = plan.mats.size();
      plan.mats.insert(plan.mats.end(), st.blk.m.begin(), st.blk.m.end());
      plan.steps.push_back(std::move(st));
      continue;
    }
    // row bits: the chosen ones, completed with the lowest unused high bits
    for (int q = C; q < n && int(hi.size()) < H; ++q)
      if (std::find(hi.begin(), hi.end(), q) == hi.end()) hi.push_back(q);
    std::sort(hi.begin(), hi.end());
    std::vector<int> tbit(n, -1);  // physical bit -> tile bit
    for (int q = 0; q < C; ++q) tbit[q] = q;
    for (int j = 0; j < H; ++j) tbit[hi[j]] = C + j;
    TileStep st;
    for (int j = 0; j < H; ++j) st.hb[j] = hi[j];
    st.r0 = int(plan.rounds.size());
    st.ngates = int(pass.size());
    // rounds: the same greedy grouping on tile bits, W bits each
    std::vector<std::vector<int>> tq(pass.size());
    for (size_t i = 0; i < pass.size(); ++i)
      for (int x : qb[pass[i]]) tq[i].push_back(tbit[x]);
    DagCursor rd(tq, C + H);
    const std::vector<char> none(C + H, 0);
    while (rd.remaining) {
      std::vector<int> rb;
      const std::vector<int> grp = take_group(rd, none, W, &rb, [](int) { return true; });
      for (int b = 0; b < C + H && int(rb.size()) < W; ++b)
        if (std::find(rb.begin(), rb.end(), b) == rb.end()) rb.push_back(b);
      std::sort(rb.begin(), rb.end());
      TileRound r;
      for (int j = 0; j < W; ++j) r.bits[j] = rb[j];
      r.g0 = int(plan.gates.size());
      r.ng = int(grp.size());
      if (dense) {
        // the product of the round's gates on its W bits (local bit j = rb[j])
        std::vector<cd> u = eye(W);
        for (int gi : grp) {
          const Gate& g = gates[pass[gi]];
          int lp[QS_MAX_FUSED];
          for (int j = 0; j < g.k; ++j)
            lp[j] = int(std::find(rb.begin(), rb.end(), tq[gi][j]) - rb.begin());
          left_apply(u, W, g.m, g.k, lp);
        }
        r.mat = plan.mats.size();
        plan.mats.insert(plan.mats.end(), u.begin(), u.end());
      } else {
        // one-qubit gates folded into the round's two-qubit gates: into the
        // last two-qubit gate on their bit (from the left) when there is one,
        // else into the next (from the right); one-qubit products on bits no
        // two-qubit gate of the round touches stay one-qubit gates (they
        // commute with the rest of the round)
        struct Out { int kind, j1, j2; std::vector<cd> m; };
        std::vector<Out> outg;
        std::vector<int> last(W, -1);            // per round bit: its last two-qubit gate
        std::vector<std::vector<cd>> pend(W);    // per round bit: pending one-qubit product
        for (int gi : grp) {
          const Gate& g = gates[pass[gi]];
          const int j1 = int(std::find(rb.begin(), rb.end(), tq[gi][0]) - rb.begin());
          if (g.k == 1) {
            if (last[j1] >= 0) {
              Out& o = outg[size_t(last[j1])];
              const int at = o.j1 == j1 ? 0 : 1;
              left_apply(o.m, 2, g.m, 1, &at);
            } else {
              if (pend[j1].empty()) pend[j1] = eye(1);
              const int at = 0;
              left_apply(pend[j1], 1, g.m, 1, &at);
            }
            continue;
          }
          const int j2 = int(std::find(rb.begin(), rb.end(), tq[gi][1]) - rb.begin());
          std::vector<cd> m = eye(2);
          const int bit0 = 0, bit1 = 1, both[2] = {0, 1};
          if (!pend[j1].empty()) left_apply(m, 2, pend[j1], 1, &bit0);
          if (!pend[j2].empty()) left_apply(m, 2, pend[j2], 1, &bit1);
          left_apply(m, 2, g.m, 2, both);
          pend[j1].clear();
          pend[j2].clear();
          last[j1] = last[j2] = int(outg.size());
          outg.push_back({2, j1, j2, std::move(m)});
        }
        for (int j = 0; j < W; ++j)
          if (!pend[j].empty()) outg.push_back({1, j, 0, std::move(pend[j])});
        r.ng = int(outg.size());
        for (Out& o : outg) {
          TileGate tg;
          tg.kind = o.kind;
          tg.j1 = o.j1;
          tg.j2 = o.j2;
          tg.mat = plan.mats.size();
          plan.mats.insert(plan.mats.end(), o.m.begin(), o.m.end());
          plan.gates.push_back(tg);
        }
      }
      plan.rounds.push_back(r);
    }
    st.nr = int(plan.rounds.size()) - st.r0;
    plan.steps.push_back(st);
  }
  return plan;
}

void tile_tables(const TilePlan& pl, bool c64, std::vector<unsigned char>* out, size_t* gates_off,
                 size_t* mats_off, size_t* emb_off) {
  const bool dense = pl.dense;
  std::vector<int32_t> tab;
  for (size_t ri = 0; ri < pl.rounds.size(); ++ri) {
    const auto& r = pl.rounds[ri];
    tab.push_back(r.bits[0] | (r.bits[1] << 8) | (r.bits[2] << 16) | (r.bits[3] << 24));
    tab.push_back(dense ? int32_t(ri * kRoundOperands) : r.g0);
    tab.push_back(r.ng);
    tab.push_back(0);
  }
  const size_t gates_at = tab.size() * sizeof(int32_t);
  if (!dense)
    for (const auto& g : pl.gates) {
      tab.push_back(g.kind | (g.j1 << 4) | (g.j2 << 8));
      tab.push_back(int32_t(2 * g.mat));
    }
  const size_t esz = c64 ? sizeof(float) : sizeof(double);
  const size_t emb_at = (tab.size() * sizeof(int32_t) + 255) / 256 * 256;
  // dense rounds: each round's matrix-core operands in lane order, then the
  // matrices of the block steps; sparse rounds: every matrix as is
  const size_t emb = dense ? pl.rounds.size() * kRoundOperands * sizeof(float) : 0;
  const size_t total = emb_at + emb + 2 * pl.mats.size() * esz;
  out->assign(total, 0);
  unsigned char* host = out->data();
  std::memcpy(host, tab.data(), tab.size() * sizeof(int32_t));
  if (dense) {
    std::vector<float> A(kRoundOperands);
    for (size_t ri = 0; ri < pl.rounds.size(); ++ri) {
      embed_round(pl.mats.data() + pl.rounds[ri].mat, A.data());
      std::memcpy(host + emb_at + ri * kRoundOperands * sizeof(float), A.data(),
                  kRoundOperands * sizeof(float));
    }
  }
  for (size_t i = 0; i < pl.mats.size(); ++i) {
    if (c64) {
      const float v[2] = {float(pl.mats[i].real()), float(pl.mats[i].imag())};
      std::memcpy(host + emb_at + emb + 2 * i * esz, v, sizeof v);
    } else {
      const double v[2] = {pl.mats[i].real(), pl.mats[i].imag()};
      std::memcpy(host + emb_at + emb + 2 * i * esz, v, sizeof v);
    }
  }
  *gates_off = gates_at;
  *emb_off = emb_at;
  *mats_off = emb_at + emb;
}

void embed_round(const cd* u, float* out) {
  for (int s4 = 0; s4 < 4; ++s4)
    for (int lane = 0; lane < 64; ++lane) {
      const cd x = u[(lane % 16) * 16 + 4 * s4 + lane / 16];
      out[(3 * s4 + 0) * 64 + lane] = float(x.real());
      out[(3 * s4 + 1) * 64 + lane] = float(x.imag());
      out[(3 * s4 + 2) * 64 + lane] = float(x.real() + x.imag());
    }
}

}  // namespace qs

// ------------------------------------------------------------------ C ABI

namespace qs {
void set_last_error(const char* msg);    // capi.cpp
void circuit_invalidate(qs_circuit* c);  // frees device copies (capi.cpp)
uint64_t next_generation();              // capi.cpp
}  // namespace qs

namespace {
int cfail(int code, const char* fmt, ...) {
  char buf[256];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  qs::set_last_error(buf);
  return code;
}
}  // namespace

namespace qs {
// The block plan alone: what a dense run without tiles or a batch needs,
// without the caller's choice of run mode that qs_circuit_plan records.
int circuit_plan_blocks(qs_circuit* c, int kmax) {
  if (!c) return cfail(QS_E_INVAL, "circuit is NULL");
  if (kmax == 0) kmax = 5;
  if (kmax < 1 || kmax > QS_MAX_FUSED) return cfail(QS_E_INVAL, "kmax = %d outside [1, %d]", kmax, QS_MAX_FUSED);
  circuit_invalidate(c);
  c->kmax = kmax;
  c->blocks = fuse(c->gates, c->n, kmax);
  c->planned = true;
  return QS_OK;
}
}  // namespace qs

extern "C" {

int qs_circuit_create(int n, qs_circuit** out) {
  if (!out) return cfail(QS_E_INVAL, "out is NULL");
  if (n < 1 || n > 64) return cfail(QS_E_INVAL, "n = %d outside [1, 64]", n);
  qs_circuit* c = new qs_circuit();
  c->n = n;
  c->generation = qs::next_generation();
  c->pos.resize(n);
  for (int q = 0; q < n; ++q) c->pos[q] = q;
  *out = c;
  return QS_OK;
}

static int add_checked(qs_circuit* c, const int* qubits, int k, std::vector<qs::cd> m) {
  if (!c) return cfail(QS_E_INVAL, "circuit is NULL");
  if (!qubits) return cfail(QS_E_INVAL, "qubits is NULL");
  if (k < 1 || k > QS_MAX_FUSED) return cfail(QS_E_INVAL, "gate on %d qubits", k);
  for (int j = 0; j < k; ++j) {
    if (qubits[j] < 0 || qubits[j] >= c->n)
      return cfail(QS_E_INVAL, "qubit %d out of range [0, %d)", qubits[j], c->n);
    for (int i = 0; i < j; ++i)
      if (qubits[i] == qubits[j]) return cfail(QS_E_INVAL, "qubit %d used twice", qubits[j]);
  }
  for (const auto& v : m)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag()))
      return cfail(QS_E_INVAL, "non-finite matrix entry");
  qs::circuit_invalidate(c);
  qs::Gate g;
  g.k = k;
  for (int j = 0; j < k; ++j) g.q[j] = c->pos[qubits[j]];
  g.m = std::move(m);
  c->gates.push_back(std::move(g));
  return QS_OK;
}

int qs_circuit_add_gate(qs_circuit* c, int kind, const int* qubits, const double* params) {
  if (!c) return cfail(QS_E_INVAL, "circuit is NULL");
  if (!qubits) return cfail(QS_E_INVAL, "qubits is NULL");
  const int nq = (kind >= QS_GATE_CZ) ? 2 : 1;
  if ((kind == QS_GATE_U3 || kind == QS_GATE_CP || kind == QS_GATE_CU3) && !params)
    return cfail(QS_E_INVAL, "gate kind %d needs parameters", kind);
  if (kind == QS_GATE_U3 || kind == QS_GATE_CU3)
    for (int i = 0; i < 3; ++i)
      if (!std::isfinite(params[i])) return cfail(QS_E_INVAL, "non-finite parameter");
  if (kind == QS_GATE_CU3 && params[3] != 0.0 && params[3] != 1.0)
    return cfail(QS_E_INVAL, "control value %g is not 0 or 1", params[3]);
  if (kind == QS_GATE_CP && !std::isfinite(params[0])) return cfail(QS_E_INVAL, "non-finite parameter");
  std::vector<qs::cd> m;
  int k = 0;
  if (!qs::gate_matrix(kind, nq, params, &m, &k)) return cfail(QS_E_INVAL, "unknown gate kind %d", kind);
  if (kind == QS_GATE_SWAP) {
    for (int j = 0; j < 2; ++j)
      if (qubits[j] < 0 || qubits[j] >= c->n)
        return cfail(QS_E_INVAL, "qubit %d out of range [0, %d)", qubits[j], c->n);
    if (qubits[0] == qubits[1]) return cfail(QS_E_INVAL, "qubit %d used twice", qubits[0]);
    qs::circuit_invalidate(c);
    std::swap(c->pos[qubits[0]], c->pos[qubits[1]]);
    return QS_OK;
  }
  return add_checked(c, qubits, k, std::move(m));
}

int qs_circuit_add_matrix(qs_circuit* c, const int* qubits, int k, const double* m) {
  if (!m) return cfail(QS_E_INVAL, "matrix is NULL");
  if (k < 1 || k > QS_MAX_FUSED) return cfail(QS_E_INVAL, "gate on %d qubits", k);
  const size_t d = size_t(1) << k;
  std::vector<qs::cd> mm(d * d);
  for (size_t i = 0; i < d * d; ++i) mm[i] = qs::cd(m[2 * i], m[2 * i + 1]);
  return add_checked(c, qubits, k, std::move(mm));
}


int qs_circuit_plan(qs_circuit* c, int kmax) {
  if (int rc = qs::circuit_plan_blocks(c, kmax)) return rc;
  if (c->tiles < 0) c->tiles = 0;  // planning blocks asks for blocks
  return QS_OK;
}

int qs_circuit_use_tiles(qs_circuit* c, int on) {
  if (!c) return cfail(QS_E_INVAL, "circuit is NULL");
  c->tiles = on != 0 ? 1 : 0;
  return QS_OK;
}

int qs_circuit_tile_info(const qs_circuit* c, int dtype, int* passes, int* blocks, int* rounds) {
  if (!c) return cfail(QS_E_INVAL, "circuit is NULL");
  if (dtype != QS_C64 && dtype != QS_C128) return cfail(QS_E_INVAL, "unknown dtype %d", dtype);
  const int C = qs::tile_low_bits(dtype);
  if (c->n < C + 7) return cfail(QS_E_UNSUPPORTED, "%d qubits: fewer than one tile (%d)", c->n, C + 7);
  const qs::TilePlan pl = qs::plan_tiles(c->gates, c->n, C, 7, 4, dtype == QS_C64);
  if (passes) *passes = pl.passes();
  if (blocks) *blocks = int(pl.steps.size()) - pl.passes();
  if (rounds) *rounds = int(pl.rounds.size());
  return QS_OK;
}

int qs_circuit_info(const qs_circuit* c, int* ngates, int* nblocks, int* max_k) {
  if (!c) return cfail(QS_E_INVAL, "circuit is NULL");
  if (ngates) *ngates = int(c->gates.size());
  if (nblocks) *nblocks = c->planned ? int(c->blocks.size()) : -1;
  if (max_k) {
    int mk = 0;
    for (const auto& b : c->blocks) mk = std::max(mk, b.k);
    *max_k = mk;
  }
  return QS_OK;
}

int qs_circuit_block(const qs_circuit* c, int i, int* k, int* qubits, double* m) {
  if (!c || !k) return cfail(QS_E_INVAL, "NULL argument");
  if (!c->planned) return cfail(QS_E_INVAL, "circuit is not planned");
  if (i < 0 || i >= int(c->blocks.size())) return cfail(QS_E_INVAL, "block %d out of range", i);
  const qs::Block& b = c->blocks[i];
  *k = b.k;
  if (qubits)
    for (int j = 0; j < b.k; ++j) qubits[j] = b.q[j];
  if (m)
    for (size_t e = 0; e < b.m.size(); ++e) {
      m[2 * e] = b.m[e].real();
      m[2 * e + 1] = b.m[e].imag();
    }
  return QS_OK;
}

}  // extern "C"
