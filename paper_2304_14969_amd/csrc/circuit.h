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

}  // namespace qs

struct qs_circuit {
  int n = 0;
  std::vector<qs::Gate> gates;  // on virtual positions (SWAPs already folded)
  std::vector<int> pos;         // logical qubit -> virtual position after all SWAPs
  int kmax = 5;
  bool planned = false;
  std::vector<qs::Block> blocks;
  // device copies of the block matrices, per precision (owned)
  void* dmat[2] = {nullptr, nullptr};
  std::vector<size_t> off[2];   // element offset of each block's matrix
};
