"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This module only draws numbers: basis indices, Gaussian amplitude vectors,
rotation angles, qubit matchings and gate-type coins. It contains none of the
simulation arithmetic (no gate matrices, no state updates), so that the FP64
oracle and the HIP path stay independent and can both consume the same input.

Gate lists are plain tuples, one per gate:

    ("h", q)                      Hadamard on qubit q
    ("u3", q, theta, phi, lam)    U(theta, phi, lambda) of Sec. III-C
    ("cp", c, t, theta)           controlled phase e^{i theta} on |11>
    ("cz", a, b)                  controlled Z
    ("iswap", a, b)               iSWAP
    ("swap", a, b)                SWAP
    ("ctrl", ctrls, cvals, t, theta, phi, lam)
                                  U3 on t, active when every ctrls[j] equals
                                  bit j of cvals (0 = anti-control)

Qubit q is bit q of the amplitude index (qubit 0 is the least significant).
All generators use numpy's PCG64 (`numpy.random.default_rng(seed)`).
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def basis_index(n: int, seed: int) -> int:
    """Uniform basis index x in [0, 2^n) for the |x> input of the QFT runs."""
    return int(rng(seed).integers(0, 2 ** n))


def gaussian_state(n: int, seed: int) -> np.ndarray:
    """i.i.d. complex Gaussian amplitudes, unit norm, complex128, length 2^n."""
    g = rng(seed)
    re = g.standard_normal(2 ** n)
    im = g.standard_normal(2 ** n)
    a = re + 1j * im
    a /= np.sqrt(np.vdot(a, a).real)
    return a


def haar_product_angles(n: int, seed: int) -> np.ndarray:
    """Per-qubit (theta, phi, lambda) with theta = arccos(1 - 2u), phi uniform,
    lambda = 0: U3(theta, phi, 0)|0> is a Haar-random single-qubit state.
    Shape (n, 3)."""
    g = rng(seed)
    u = g.random(n)
    theta = np.arccos(1.0 - 2.0 * u)
    phi = g.uniform(0.0, TWO_PI, n)
    return np.stack([theta, phi, np.zeros(n)], axis=1)


def haar_product_gates(n: int, seed: int) -> list:
    """Gate list preparing the Haar-random product state from |0...0>."""
    ang = haar_product_angles(n, seed)
    return [("u3", q, float(ang[q, 0]), float(ang[q, 1]), float(ang[q, 2]))
            for q in range(n)]


def random_circuit(n: int, layers: int, seed: int, haar: bool = False) -> list:
    """Layered random circuit: per layer, U3 on every qubit (theta, phi, lambda
    uniform on [0, 2pi), or Haar when `haar`), then a seeded random perfect
    matching of the qubits with CZ or iSWAP (probability 1/2 each) per pair.
    With odd n the leftover qubit idles for that layer."""
    g = rng(seed)
    gates: list = []
    for _ in range(layers):
        ang = g.uniform(0.0, TWO_PI, (n, 3))
        if haar:
            ang[:, 0] = np.arccos(1.0 - 2.0 * g.random(n))
        perm = g.permutation(n)
        coin = g.random(n // 2) < 0.5
        for q in range(n):
            gates.append(("u3", q, float(ang[q, 0]), float(ang[q, 1]), float(ang[q, 2])))
        for i in range(n // 2):
            a, b = int(perm[2 * i]), int(perm[2 * i + 1])
            gates.append(("cz", a, b) if coin[i] else ("iswap", a, b))
    return gates


def random_gate_soup(n: int, count: int, seed: int, kinds=None) -> list:
    """Unstructured gate sequence over every gate kind, for parity tests."""
    g = rng(seed)
    kinds = kinds or ["h", "u3", "cp", "cz", "iswap", "swap", "ctrl"]
    gates: list = []
    for _ in range(count):
        k = kinds[int(g.integers(0, len(kinds)))]
        if k == "h":
            gates.append(("h", int(g.integers(0, n))))
        elif k == "u3":
            t, p, l = g.uniform(0.0, TWO_PI, 3)
            gates.append(("u3", int(g.integers(0, n)), float(t), float(p), float(l)))
        elif k in ("cp", "cz", "iswap", "swap"):
            a, b = (int(v) for v in g.choice(n, 2, replace=False))
            if k == "cp":
                gates.append(("cp", a, b, float(g.uniform(0.0, TWO_PI))))
            else:
                gates.append((k, a, b))
        elif k == "ctrl":
            nc = int(g.integers(1, min(3, n - 1) + 1))
            qs = [int(v) for v in g.choice(n, nc + 1, replace=False)]
            cv = int(g.integers(0, 2 ** nc))
            t, p, l = g.uniform(0.0, TWO_PI, 3)
            gates.append(("ctrl", tuple(qs[:nc]), cv, qs[nc], float(t), float(p), float(l)))
    return gates


def batch_widths(count: int, seed: int, low: int = 12, high: int = 20) -> list:
    """Widths n_i = low + U{0..high-low} of a batch of small circuits."""
    g = rng(seed)
    return [int(low + v) for v in g.integers(0, high - low + 1, count)]


def qft_gate_counts(n: int) -> dict:
    """Gate counts of the n-qubit QFT circuit: n H, n(n-1)/2 controlled
    phases and floor(n/2) SWAPs of the final bit reversal."""
    return {"h": n, "cp": n * (n - 1) // 2, "swap": n // 2}


# The coupling patterns of a rows x cols grid (qubit r*cols + c): A and B are
# the horizontal edges starting at even / odd columns, C and D the vertical
# edges starting at even / odd rows. Layer l uses pattern "ABCDCDAB"[l % 8].
GRID_SEQUENCE = "ABCDCDAB"
COUPLER_KINDS = ("cx", "cy", "cz", "ax", "ay", "az")


def grid_edges(rows: int, cols: int, pattern: str) -> list:
    edges = []
    if pattern in "AB":
        start = 0 if pattern == "A" else 1
        for r in range(rows):
            for c in range(start, cols - 1, 2):
                edges.append((r * cols + c, r * cols + c + 1))
    else:
        start = 0 if pattern == "C" else 1
        for r in range(start, rows - 1, 2):
            for c in range(cols):
                edges.append((r * cols + c, (r + 1) * cols + c))
    return edges


def grid_circuit(rows: int, cols: int, layers: int, seed: int) -> list:
    """Layered random circuit of the paper's family (Sec. III-C): U3 with
    theta, phi, lambda uniform on [0, 2pi) on every qubit, then a coupler
    drawn uniformly from CX, CY, CZ, AX, AY, AZ on every nearest-neighbour
    edge of the layer's pattern, control and target in random order."""
    g = rng(seed)
    n = rows * cols
    gates: list = []
    for layer in range(layers):
        ang = g.uniform(0.0, TWO_PI, (n, 3))
        for q in range(n):
            gates.append(("u3", q, float(ang[q, 0]), float(ang[q, 1]), float(ang[q, 2])))
        for a, b in grid_edges(rows, cols, GRID_SEQUENCE[layer % len(GRID_SEQUENCE)]):
            kind = COUPLER_KINDS[int(g.integers(0, len(COUPLER_KINDS)))]
            if g.random() < 0.5:
                a, b = b, a
            gates.append((kind, a, b))
    return gates


def pair_chain_circuit(n: int, layers: int, seed: int, theta_max: float = 0.3) -> list:
    """Entangled pairs (2k, 2k+1) weakly coupled along a chain: first H on
    every even qubit and a CNOT into its partner; then per layer a U3 on every
    qubit (angles uniform in [0, 2 pi)), the CNOT inside pair 0, and for k = 0,
    2, 4, ...: a controlled RY(theta) from qubit k+1 to k+2 (theta uniform in
    [0, theta_max)) followed by the CNOT inside the pair (k+2, k+3). The pairs
    stay strongly entangled inside and weakly with each other: the workload of
    the two-qubit rounding (n even)."""
    if n % 2:
        raise ValueError("pair chains need an even number of qubits")
    g = rng(seed)
    cx = lambda c, t: ("ctrl", [c], 1, t, math.pi, 0.0, math.pi)  # noqa: E731  U3(pi,0,pi) = X
    gates = []
    for k in range(0, n, 2):
        gates += [("h", k), cx(k, k + 1)]
    for _ in range(layers):
        ang = g.uniform(0.0, TWO_PI, (n, 3))
        gates += [("u3", q, float(ang[q, 0]), float(ang[q, 1]), float(ang[q, 2])) for q in range(n)]
        th = g.uniform(0.0, theta_max, n // 2)
        gates.append(cx(0, 1))
        for k in range(0, n - 2, 2):
            gates += [("ctrl", [k + 1], 1, k + 2, float(th[k // 2]), 0.0, 0.0), cx(k + 2, k + 3)]
    return gates


# X, Y, Z with exact entries, as "mat" gates
PAULI_MATS = (((0, 1), (1, 0)), ((0, -1j), (1j, 0)), ((1, 0), (0, -1)))


def held_gate_mix(n: int, count: int, seed: int) -> list:
    """Gate sequence dominated by the forms a factorized engine can hold back
    between subsystems (controlled phases and inversions: CZ, CX, CY, CP) and
    by the one-qubit gates that move them (H, Pauli gates, phase gates as U3
    with theta = 0), with a few general U3 and anti-controlled X gates that do
    not commute with them; for parity tests of that bookkeeping."""
    g = rng(seed)
    gates: list = []
    for _ in range(count):
        u = g.random()
        q = int(g.integers(0, n))
        if u < 0.30:
            gates.append(("h", q))
        elif u < 0.40:
            gates.append(("mat", [q], PAULI_MATS[int(g.integers(0, 3))]))
        elif u < 0.48:
            gates.append(("u3", q, 0.0, 0.0, float(g.uniform(0.0, TWO_PI))))
        elif u < 0.52:
            t, p, l = g.uniform(0.0, TWO_PI, 3)
            gates.append(("u3", q, float(t), float(p), float(l)))
        else:
            a, b = (int(v) for v in g.choice(n, 2, replace=False))
            k = ("cz", "cx", "cy", "cp", "cp", "ax")[int(g.integers(0, 6))]
            if k == "cp":
                th = float(np.pi / 4 * int(g.integers(1, 8))) if g.random() < 0.5 \
                    else float(g.uniform(0.0, TWO_PI))
                gates.append(("cp", a, b, th))
            else:
                gates.append((k, a, b))
    return gates


def phase_kickback_circuit(n: int, seed: int):
    """Bernstein-Vazirani circuit on n qubits: an ancilla (qubit n - 1) in
    |->, every data qubit in |+>, a CX from each data qubit whose secret bit
    is 1 onto the ancilla, then H on the data qubits, which then hold the
    secret. Returns (gates, secret)."""
    g = rng(seed)
    secret = [int(v) for v in g.integers(0, 2, n - 1)]
    anc = n - 1
    gates: list = [("mat", [anc], PAULI_MATS[0])] + [("h", q) for q in range(n)]
    gates += [("cx", q, anc) for q in range(n - 1) if secret[q]]
    gates += [("h", q) for q in range(n - 1)]
    return gates, secret
