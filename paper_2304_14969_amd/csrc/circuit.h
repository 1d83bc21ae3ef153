// Host-side circuit object and gate-fusion planner (internal).
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

#include "../../include/qs.h"

namespace qs {

using cd = std::complex<double>;

// One gate: qubits[j] is bit j of the row/column index of the 2^k matrix.
struct Gate {
  int k = 0;
  int q[QS_MAX_FUSED] = {0};
  std::vector<cd> m;  // 2^k x 2^k row-major
};

// A fused block: the product of its gates, on `k` qubits (ascending).
struct Block {
  int k = 0;
  int q[QS_MAX_FUSED] = {0};
  int ngates = 0;
  std::vector<cd> m;
};

// Matrix of a named gate kind (QS_GATE_*) with its parameters; false for an
// unknown kind or a wrong qubit count.
bool gate_matrix(int kind, int nq, const double* params, std::vector<cd>* m, int* k_out);

// Greedy fusion: gates in order; open blocks on disjoint qubit sets; a gate
// joins (and merges) the open blocks it touches when the union has at most
// kmax qubits, else those blocks are emitted and the gate opens a new one.
// Blocks are emitted in an order that keeps every qubit's gates in order.
std::vector<Block> fuse(const std::vector<Gate>& gates, int n, int kmax);

// ---- tile passes
// A pass loads a tile of 2^(C+H) amplitudes: the contiguous low bits [0, C)
// and H chosen bits (rows), runs rounds of gates on it and stores it back,
// one HBM read and write for every gate it holds. A round gathers, per
// thread, the 2^W amplitudes that differ in W tile bits and applies the
// round's one- and two-qubit gates to them in registers.
struct TileGate {
  int kind = 1;      // 1: one-qubit (j1); 2: two-qubit (row bit 0 = j1, bit 1 = j2)
  int j1 = 0, j2 = 0;
  size_t mat = 0;    // offset of the matrix in TilePlan::mats (complex entries)
};
struct TileRound {
  int bits[4] = {0, 0, 0, 0};  // tile bits of the round, ascending
  int g0 = 0, ng = 0;          // its gates in TilePlan::gates (sparse rounds)
  size_t mat = 0;              // dense rounds: offset of the 16x16 product in mats
};
struct TileStep {
  bool block = false;  // a dense block (a gate on more than two qubits), not a pass
  int hb[8] = {0};     // pass: the H row bits (physical, ascending)
  int r0 = 0, nr = 0;  // pass: its rounds
  int ngates = 0;
  Block blk;           // block step, on physical bits
  size_t mat = 0;      // block step: offset of its matrix
};
struct TilePlan {
  int C = 0, H = 0, W = 0;
  bool dense = false;  // rounds are dense W-qubit blocks (any gate of <= W qubits)
  std::vector<TileStep> steps;
  std::vector<TileRound> rounds;
  std::vector<TileGate> gates;
  std::vector<cd> mats;
  int passes() const {
    int p = 0;
    for (const auto& s : steps) p += s.block ? 0 : 1;
    return p;
  }
};

// Plans `gates` (on physical bits, in circuit order) into tile passes for a
// state of n >= C + H qubits. Greedy over the gate dependence order: a pass
// takes every gate at the front whose qubits fit in the low bits plus at
// most H other bits, in circuit order, until none fits. Rounds are formed
// the same way within a pass with W bits each. Sparse rounds (dense =
// false) hold gates of one or two qubits; dense rounds hold any gate of at
// most W qubits and carry the product of their gates. Larger gates run as
// dense blocks between passes.
TilePlan plan_tiles(const std::vector<Gate>& gates, int n, int C, int H, int W, bool dense);

// The device tables of a plan, as one byte image: per round an int4 {bits
// packed by byte, first gate (sparse) or embedding offset in floats (dense),
// gate count, 0}; per gate (sparse) an int2 {kind | j1 << 4 | j2 << 8, offset
// of its matrix in reals}; at emb_off (dense) the rounds' 32 x 32 embeddings
// in lane order (float); at mats_off the plan's matrices (float or double
// pairs). Offsets are bytes from the start.
void tile_tables(const TilePlan& pl, bool c64, std::vector<unsigned char>* out, size_t* gates_off,
                 size_t* mats_off, size_t* emb_off);

// The operands a matrix-core round reads, for the three real products of
// Re U X_r, Im U X_i and (Re U + Im U)(X_r + X_i) of a 16 x 16 complex round
// matrix u (16 x 16 x 4 MFMA A-operand layout): out[(3 s + c) * 64 + lane] =
// W_c[lane % 16][4 s + lane / 16] with W_0 = Re U, W_1 = Im U,
// W_2 = Re U + Im U (summed in float64), s = 0 .. 3.
void embed_round(const cd* u, float* out);

// Fuse a circuit's gates into blocks of at most kmax qubits (0 = 5) without
// recording a choice of run mode (internal planning; qs_circuit_plan does
// record it).
int circuit_plan_blocks(qs_circuit* c, int kmax);

}  // namespace qs

struct qs_circuit {
  int n = 0;
  uint64_t generation = 0;      // bumped whenever the gate list changes
  std::vector<qs::Gate> gates;  // on virtual positions (SWAPs already folded)
  std::vector<int> pos;         // logical qubit -> virtual position after all SWAPs
  int kmax = 5;
  bool planned = false;
  std::vector<qs::Block> blocks;
  // device copies of the block matrices, per precision (owned)
  void* dmat[2] = {nullptr, nullptr};
  std::vector<size_t> off[2];   // element offset of each block's matrix
  // tile passes (dense runs), planned per precision and physical labelling:
  // 1 on, 0 off (qs_circuit_use_tiles(c, 0), or blocks planned with
  // qs_circuit_plan before any choice), -1 not chosen (on)
  int tiles = -1;
  struct TileCache {
    std::vector<int> key;  // physical bit of every virtual position
    qs::TilePlan plan;
    void* dev = nullptr;   // rounds, gates, matrices (owned)
    size_t gates_off = 0, mats_off = 0, emb_off = 0;  // byte offsets in dev
  } tcache[2];
  // host plan for batched runs (identity labelling, dense rounds); cleared
  // with the other plans when the circuit changes
  bool bplan_ok = false;
  qs::TilePlan bplan;
};
