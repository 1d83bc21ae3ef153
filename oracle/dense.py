"""Exact FP64 state-vector oracle (test infrastructure only).

Plain, slow and direct: a ket of n qubits is a complex128 vector of 2^n
amplitudes, qubit q is bit q of the index (qubit 0 least significant), and a
circuit is applied one gate at a time (Sec. II, the problem statement
|psi_C> = C|psi_0> with C a sequence of k-local gates).

Nothing here fuses gates, relabels qubits or reorders work: a SWAP moves
amplitudes, a "fused" block is applied as its constituent gates, and the QFT is
the H + controlled-phase circuit, gate after gate.
"""
from __future__ import annotations

import math

import numpy as np

C128 = np.complex128

# ---------------------------------------------------------------- states


def zero_state(n: int) -> np.ndarray:
    a = np.zeros(2 ** n, dtype=C128)
    a[0] = 1.0
    return a


def basis_state(n: int, x: int) -> np.ndarray:
    a = np.zeros(2 ** n, dtype=C128)
    a[x] = 1.0
    return a


def ghz_state(n: int) -> np.ndarray:
    """(|0...0> + |1...1>)/sqrt(2), Eq. ghz."""
    a = np.zeros(2 ** n, dtype=C128)
    a[0] = a[-1] = 1.0 / math.sqrt(2.0)
    return a


# ---------------------------------------------------------------- matrices


def u3(theta: float, phi: float, lam: float) -> np.ndarray:
    """The general single-qubit unitary U(theta, phi, lambda) of Sec. III-C."""
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array(
        [[c, -np.exp(1j * lam) * s],
         [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]], dtype=C128)


H = np.array([[1.0, 1.0], [1.0, -1.0]], dtype=C128) / math.sqrt(2.0)
X = np.array([[0, 1], [1, 0]], dtype=C128)
Y = np.array([[0, -1j], [1j, 0]], dtype=C128)
Z = np.array([[1, 0], [0, -1]], dtype=C128)


def cphase_matrix(theta: float) -> np.ndarray:
    """Controlled phase: e^{i theta} on |11>, identity elsewhere (Sec. II-E)."""
    return np.diag([1.0, 1.0, 1.0, np.exp(1j * theta)]).astype(C128)


CZ = np.diag([1.0, 1.0, 1.0, -1.0]).astype(C128)
PAULI = {"x": X, "y": Y, "z": Z}
COUPLERS = ("cx", "cy", "cz", "ax", "ay", "az")
ISWAP = np.array([[1, 0, 0, 0], [0, 0, 1j, 0], [0, 1j, 0, 0], [0, 0, 0, 1]], dtype=C128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=C128)


def controlled_matrix(nctrl: int, cvals: int, m: np.ndarray) -> np.ndarray:
    """(nctrl+1)-qubit matrix: local bits 0..nctrl-1 are the controls, local
    bit nctrl the target; m acts on the target when control bit j equals bit j
    of cvals, the identity acts otherwise."""
    d = 2 ** (nctrl + 1)
    full = np.eye(d, dtype=C128)
    base = cvals & ((1 << nctrl) - 1)
    top = 1 << nctrl
    for i in range(2):
        for j in range(2):
            full[base + i * top, base + j * top] = m[i, j]
    return full


# ---------------------------------------------------------------- application


def apply_matrix(a: np.ndarray, n: int, qubits, m: np.ndarray) -> np.ndarray:
    """Apply a 2^k x 2^k matrix m to the listed qubits of the ket a.

    Row/column bit j of m corresponds to qubits[j]. The ket is viewed as an
    n-axis tensor; numpy's axis 0 is the most significant bit, so qubit q is
    axis n-1-q. The gate's axes are moved to the front (qubits[k-1] first, so
    that the flattened front index is sum_j bit_j 2^j), multiplied by m, and
    moved back.
    """
    qubits = list(qubits)
    k = len(qubits)
    assert len(set(qubits)) == k and all(0 <= q < n for q in qubits)
    assert m.shape == (2 ** k, 2 ** k)
    t = a.reshape((2,) * n)
    axes = [n - 1 - q for q in reversed(qubits)]
    t = np.moveaxis(t, axes, list(range(k)))
    shp = t.shape
    t = (m @ t.reshape(2 ** k, -1)).reshape(shp)
    t = np.moveaxis(t, list(range(k)), axes)
    return np.ascontiguousarray(t).reshape(-1)


def apply_1q(a, n, q, m):
    return apply_matrix(a, n, [q], np.asarray(m, dtype=C128))


def apply_ctrl(a, n, ctrls, cvals, target, m):
    ctrls = list(ctrls)
    return apply_matrix(a, n, ctrls + [target],
                        controlled_matrix(len(ctrls), cvals, np.asarray(m, dtype=C128)))


def apply_cphase(a, n, c, t, theta):
    return apply_matrix(a, n, [c, t], cphase_matrix(theta))


def apply_swap(a, n, q0, q1):
    """Physical exchange of the amplitudes whose bits q0 and q1 differ."""
    return apply_matrix(a, n, [q0, q1], SWAP)


def gate_matrix(g) -> tuple:
    """(qubits, matrix) of one gate tuple of the workloads gate-list format."""
    kind = g[0]
    if kind == "h":
        return [g[1]], H
    if kind == "u3":
        return [g[1]], u3(g[2], g[3], g[4])
    if kind == "cp":
        return [g[1], g[2]], cphase_matrix(g[3])
    if kind == "cz":
        return [g[1], g[2]], CZ
    if kind == "iswap":
        return [g[1], g[2]], ISWAP
    if kind == "swap":
        return [g[1], g[2]], SWAP
    if kind == "ctrl":
        ctrls = list(g[1])
        return ctrls + [g[3]], controlled_matrix(len(ctrls), g[2], u3(g[4], g[5], g[6]))
    if kind in COUPLERS:
        # (control, target); "c*" acts when the control is |1>, "a*" when |0>
        # (the couplers of Sec. III-C)
        cv = 1 if kind[0] == "c" else 0
        return [g[1], g[2]], controlled_matrix(1, cv, PAULI[kind[1]])
    if kind == "mat":
        return list(g[1]), np.asarray(g[2], dtype=C128)
    raise ValueError(f"unknown gate {kind!r}")


def apply_gate(a, n, g):
    qubits, m = gate_matrix(g)
    return apply_matrix(a, n, qubits, m)


def run_circuit(a, n, gates):
    for g in gates:
        a = apply_gate(a, n, g)
    return a


def apply_fused(a, n, gates):
    """A fused k-qubit block is checked against its constituent gates applied
    one at a time: the oracle never forms the block's product matrix."""
    return run_circuit(a, n, gates)


# ---------------------------------------------------------------- QFT


def qft_gates(n: int, start: int = 0, length: int | None = None,
              inverse: bool = False) -> list:
    """The QFT circuit on qubits start..start+length-1 (Sec. II-E: the DFT of
    Eq. dft, omega = e^{+2 pi i/N}, decomposed into H and controlled phases).

    Little-endian qubits. Forward: for j from the top qubit down, H on j, then
    a controlled phase pi/2^(j-m) between m and j for every lower m; finally
    the bit reversal as SWAPs. The inverse is the reversed circuit with every
    phase negated (H is its own inverse).
    """
    length = n - start if length is None else length
    qs = list(range(start, start + length))
    fwd: list = []
    for jj in range(length - 1, -1, -1):
        j = qs[jj]
        fwd.append(("h", j))
        for mm in range(jj - 1, -1, -1):
            fwd.append(("cp", qs[mm], j, math.pi / 2 ** (jj - mm)))
    for i in range(length // 2):
        fwd.append(("swap", qs[i], qs[length - 1 - i]))
    if not inverse:
        return fwd
    inv = []
    for g in reversed(fwd):
        inv.append(("cp", g[1], g[2], -g[3]) if g[0] == "cp" else g)
    return inv


def qft(a, n, start=0, length=None, inverse=False):
    return run_circuit(a, n, qft_gates(n, start, length, inverse))


def dft_entries(a, n, js, chunk: int = 1 << 22) -> np.ndarray:
    """Single outputs of the transform straight from its definition, Eq. dft
    with the printed + sign: y_j = N^{-1/2} sum_k x_k e^{+2 pi i j k / N}, for
    each j in js (for spot checks at sizes where the circuit is too slow).
    The phase j k mod N is taken in exact integer arithmetic."""
    a = np.asarray(a, dtype=np.complex128)
    N = 1 << n
    out = np.empty(len(js), dtype=np.complex128)
    for t, j in enumerate(js):
        acc = 0.0 + 0.0j
        for k0 in range(0, N, chunk):
            k = np.arange(k0, min(N, k0 + chunk), dtype=np.int64)
            ph = ((int(j) * k) % N).astype(np.float64) * (2.0 * np.pi / N)
            acc += np.dot(a[k0:k0 + len(k)], np.exp(1j * ph))
        out[t] = acc / np.sqrt(N)
    return out


def qft_basis_entries(n, x, js) -> np.ndarray:
    """The transform of the basis state |x>: 2^{-n/2} e^{2 pi i x j / 2^n}.
    The phase x j mod 2^n is taken on Python integers (exact at any n; the
    product overflows 64 bits at n = 32)."""
    N = 1 << n
    ph = np.array([(int(x) * int(j)) % N for j in np.asarray(js).ravel()],
                  dtype=np.float64) * (2.0 * np.pi / N)
    return np.exp(1j * ph) / np.sqrt(N)


# ---------------------------------------------------------------- readout


def norm2(a) -> float:
    return float(np.vdot(a, a).real)


def probs(a) -> np.ndarray:
    return (a.conj() * a).real


def fidelity(a, b) -> float:
    """|<a|b>|^2, Eq. fid_exact."""
    return float(abs(np.vdot(a, b)) ** 2)
