"""Pins of the dense FP64 oracle against what the mathematics fixes.

None of these checks re-types the oracle's own formula: gates are compared with
full 2^n x 2^n unitaries built another way (index enumeration, Kronecker
products), the QFT with its closed forms and with numpy's inverse FFT.
"""
import itertools
import math

import numpy as np
import pytest

import workloads
from oracle import dense

RNG = np.random.default_rng(1234)


def haar_unitary(d, g=RNG):
    z = (g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def brute_unitary(n, qubits, m):
    """Full matrix by enumerating index pairs: U[x', x] = m[sub(x'), sub(x)]
    when x' and x agree outside the gate's qubits."""
    N = 2 ** n
    k = len(qubits)
    mask = sum(1 << q for q in qubits)
    U = np.zeros((N, N), dtype=complex)
    for x in range(N):
        for x2 in range(N):
            if (x & ~mask) != (x2 & ~mask):
                continue
            s = sum(((x >> q) & 1) << j for j, q in enumerate(qubits))
            s2 = sum(((x2 >> q) & 1) << j for j, q in enumerate(qubits))
            U[x2, x] = m[s2, s]
    return U


@pytest.mark.parametrize("n,k", [(3, 1), (4, 2), (5, 3), (4, 4), (5, 2)])
def test_apply_matrix_matches_brute_force(n, k):
    g = np.random.default_rng(n * 10 + k)
    for _ in range(3):
        qubits = [int(v) for v in g.choice(n, k, replace=False)]
        m = haar_unitary(2 ** k, g)
        a = workloads.gaussian_state(n, int(g.integers(1 << 30)))
        want = brute_unitary(n, qubits, m) @ a
        got = dense.apply_matrix(a, n, qubits, m)
        np.testing.assert_allclose(got, want, atol=1e-13)


@pytest.mark.parametrize("q", range(5))
def test_1q_gate_is_kronecker_product(q):
    n = 5
    m = haar_unitary(2)
    U = np.kron(np.kron(np.eye(2 ** (n - q - 1)), m), np.eye(2 ** q))
    a = workloads.gaussian_state(n, q)
    np.testing.assert_allclose(dense.apply_1q(a, n, q, m), U @ a, atol=1e-13)


def test_u3_special_cases():
    # U(theta, phi, lambda) of Sec. III-C reduces to textbook gates
    np.testing.assert_allclose(dense.u3(math.pi / 2, 0, math.pi), dense.H, atol=1e-15)
    np.testing.assert_allclose(dense.u3(0, 0, 0), np.eye(2), atol=1e-15)
    np.testing.assert_allclose(dense.u3(math.pi, 0, math.pi), dense.X, atol=1e-15)
    np.testing.assert_allclose(dense.u3(math.pi, math.pi / 2, math.pi / 2), dense.Y, atol=1e-15)
    # diagonal form: U(0, 0, lambda) = diag(1, e^{i lambda})
    np.testing.assert_allclose(dense.u3(0, 0, 0.7), np.diag([1, np.exp(0.7j)]), atol=1e-15)
    for t, p, l in np.random.default_rng(5).uniform(0, 2 * math.pi, (20, 3)):
        u = dense.u3(t, p, l)
        np.testing.assert_allclose(u.conj().T @ u, np.eye(2), atol=1e-14)
        # a full period of theta only flips the global sign
        np.testing.assert_allclose(dense.u3(t + 2 * math.pi, p, l), -u, atol=1e-14)


def test_two_qubit_matrices():
    np.testing.assert_allclose(dense.cphase_matrix(0.0), np.eye(4), atol=0)
    np.testing.assert_allclose(dense.cphase_matrix(math.pi), dense.CZ, atol=1e-15)
    # iSWAP = exp(i pi/4 (XX + YY)); SWAP exchanges |01> and |10>
    XX = np.kron(dense.X, dense.X)
    YY = np.kron(dense.Y, dense.Y)
    w, V = np.linalg.eigh(XX + YY)
    iswap = V @ np.diag(np.exp(1j * math.pi / 4 * w)) @ V.conj().T
    np.testing.assert_allclose(dense.ISWAP, iswap, atol=1e-14)
    e = np.eye(4)
    np.testing.assert_allclose(dense.SWAP, e[[0, 2, 1, 3]], atol=0)


def test_controlled_gate_by_index_loop():
    n = 5
    g = np.random.default_rng(7)
    for _ in range(10):
        nc = int(g.integers(1, 4))
        qs = [int(v) for v in g.choice(n, nc + 1, replace=False)]
        ctrls, t = qs[:nc], qs[nc]
        cv = int(g.integers(0, 2 ** nc))
        m = haar_unitary(2, g)
        a = workloads.gaussian_state(n, int(g.integers(1 << 30)))
        want = a.copy()
        for x in range(2 ** n):
            if (x >> t) & 1:
                continue
            if all(((x >> c) & 1) == ((cv >> j) & 1) for j, c in enumerate(ctrls)):
                x1 = x | (1 << t)
                want[x], want[x1] = m[0, 0] * a[x] + m[0, 1] * a[x1], m[1, 0] * a[x] + m[1, 1] * a[x1]
        got = dense.apply_ctrl(a, n, ctrls, cv, t, m)
        np.testing.assert_allclose(got, want, atol=1e-13)


def test_swap_exchanges_index_bits():
    n = 6
    a = workloads.gaussian_state(n, 3)
    for q0, q1 in [(0, 5), (2, 3), (4, 1)]:
        got = dense.apply_swap(a, n, q0, q1)
        for x in range(2 ** n):
            b0, b1 = (x >> q0) & 1, (x >> q1) & 1
            y = x & ~((1 << q0) | (1 << q1)) | (b1 << q0) | (b0 << q1)
            assert got[y] == a[x]


def test_cphase_by_index_loop():
    n = 4
    a = workloads.gaussian_state(n, 9)
    got = dense.apply_cphase(a, n, 3, 1, 0.3)
    for x in range(2 ** n):
        f = np.exp(0.3j) if ((x >> 3) & 1) and ((x >> 1) & 1) else 1.0
        assert abs(got[x] - f * a[x]) < 1e-15


# ------------------------------------------------------------------ QFT


@pytest.mark.parametrize("n", range(1, 8))
def test_qft_basis_state_closed_form(n):
    """QFT|x> has amplitudes 2^{-n/2} e^{2 pi i x y / 2^n} (Eq. dft)."""
    N = 2 ** n
    ys = np.arange(N)
    for x in range(N) if n <= 4 else [0, 1, N - 1, N // 3, workloads.basis_index(n, n)]:
        got = dense.qft(dense.basis_state(n, x), n)
        want = np.exp(2j * math.pi * x * ys / N) / math.sqrt(N)
        np.testing.assert_allclose(got, want, atol=1e-13)


@pytest.mark.parametrize("n", [2, 5, 8, 10])
def test_qft_equals_inverse_fft(n):
    """Eq. dft with omega = e^{+2 pi i/N} is numpy's ifft scaled by sqrt(N)."""
    a = workloads.gaussian_state(n, 100 + n)
    np.testing.assert_allclose(dense.qft(a, n), np.fft.ifft(a) * math.sqrt(2 ** n), atol=1e-12)


@pytest.mark.parametrize("n", [3, 6, 9])
def test_qft_ghz_closed_form(n):
    """QFT of Eq. ghz: y_j = (1 + e^{-2 pi i j/N}) / sqrt(2N)."""
    N = 2 ** n
    j = np.arange(N)
    want = (1.0 + np.exp(-2j * math.pi * j / N)) / math.sqrt(2 * N)
    np.testing.assert_allclose(dense.qft(dense.ghz_state(n), n), want, atol=1e-13)


@pytest.mark.parametrize("n", [3, 8, 11])
def test_dft_entries_match_fft_and_circuit(n):
    """The per-output definition used for spot checks at large n agrees with
    numpy's inverse FFT (and, for small n, with the gate circuit); the chunked
    sum and the integer phase reduction give the same entries."""
    a = workloads.gaussian_state(n, 300 + n)
    js = list(range(2 ** n)) if n <= 8 else [0, 1, 2 ** n - 1, 77, 1234]
    got = dense.dft_entries(a, n, js, chunk=64)
    want = (np.fft.ifft(a) * math.sqrt(2 ** n))[js]
    np.testing.assert_allclose(got, want, atol=1e-12)
    if n <= 8:
        np.testing.assert_allclose(got, dense.qft(a, n), atol=1e-12)
    x = workloads.basis_index(n, 9)
    np.testing.assert_allclose(dense.qft_basis_entries(n, x, js),
                               dense.dft_entries(dense.basis_state(n, x), n, js), atol=1e-13)


def test_qft_zero_is_uniform():
    n = 7
    np.testing.assert_allclose(dense.qft(dense.zero_state(n), n),
                               np.full(2 ** n, 2 ** (-n / 2)), atol=1e-14)


@pytest.mark.parametrize("n", [4, 7])
def test_qft_inverse_and_square(n):
    a = workloads.gaussian_state(n, 7 * n)
    np.testing.assert_allclose(dense.qft(dense.qft(a, n), n, inverse=True), a, atol=1e-13)
    np.testing.assert_allclose(dense.qft(dense.qft(a, n, inverse=True), n), a, atol=1e-13)
    # the DFT applied twice maps x -> -x mod N
    N = 2 ** n
    np.testing.assert_allclose(dense.qft(dense.qft(a, n), n), a[(-np.arange(N)) % N], atol=1e-13)


@pytest.mark.parametrize("start,length", [(0, 3), (2, 3), (1, 5), (3, 2)])
def test_partial_qft_is_fft_along_its_bits(start, length):
    n = 7
    a = workloads.gaussian_state(n, start * 10 + length)
    t = a.reshape(2 ** (n - start - length), 2 ** length, 2 ** start)
    want = (np.fft.ifft(t, axis=1) * math.sqrt(2 ** length)).reshape(-1)
    np.testing.assert_allclose(dense.qft(a, n, start, length), want, atol=1e-13)
    np.testing.assert_allclose(dense.qft(dense.qft(a, n, start, length), n, start, length,
                                         inverse=True), a, atol=1e-13)


def test_qft_gate_counts():
    for n in (1, 2, 7, 16, 27):
        gates = dense.qft_gates(n)
        kinds = [g[0] for g in gates]
        want = workloads.qft_gate_counts(n)
        assert kinds.count("h") == want["h"]
        assert kinds.count("cp") == want["cp"]
        assert kinds.count("swap") == want["swap"]


def test_random_circuit_brute_force_and_norm():
    n = 5
    gates = workloads.random_circuit(n, 3, 11)
    a = dense.zero_state(n)
    U = np.eye(2 ** n, dtype=complex)
    for g in gates:
        qubits, m = dense.gate_matrix(g)
        U = brute_unitary(n, qubits, m) @ U
    got = dense.run_circuit(a, n, gates)
    np.testing.assert_allclose(got, U[:, 0], atol=1e-12)
    np.testing.assert_allclose(U.conj().T @ U, np.eye(2 ** n), atol=1e-12)
    assert abs(dense.norm2(got) - 1) < 1e-13


def test_gate_soup_brute_force():
    n = 5
    gates = workloads.random_gate_soup(n, 40, 3)
    a = workloads.gaussian_state(n, 4)
    want = a.copy()
    for g in gates:
        qubits, m = dense.gate_matrix(g)
        want = brute_unitary(n, qubits, m) @ want
    np.testing.assert_allclose(dense.run_circuit(a, n, gates), want, atol=1e-12)


def test_workload_generator_shapes():
    gates = workloads.random_circuit(7, 2, 0)
    assert sum(g[0] == "u3" for g in gates) == 14
    assert sum(g[0] in ("cz", "iswap") for g in gates) == 6
    for layer in range(2):
        pairs = [g[1:3] for g in gates[layer * 10 + 7:layer * 10 + 10]]
        flat = [q for p in pairs for q in p]
        assert len(set(flat)) == 6
    ang = workloads.haar_product_angles(10000, 1)
    # Haar: cos(theta) uniform on [-1, 1]
    assert abs(np.mean(np.cos(ang[:, 0]))) < 0.03
    assert abs(np.mean(np.cos(ang[:, 0]) ** 2) - 1 / 3) < 0.02


def test_couplers_by_index_loop():
    """CX/CY/CZ act on the target when the control is 1, AX/AY/AZ when it is 0
    (Sec. III-C)."""
    n = 4
    a = workloads.gaussian_state(n, 31)
    P = {"x": dense.X, "y": dense.Y, "z": dense.Z}
    for kind in ("cx", "cy", "cz", "ax", "ay", "az"):
        c, t = 3, 1
        got = dense.apply_gate(a, n, (kind, c, t))
        want = a.copy()
        active = 1 if kind[0] == "c" else 0
        for x in range(2 ** n):
            if (x >> t) & 1 or ((x >> c) & 1) != active:
                continue
            x1 = x | (1 << t)
            m = P[kind[1]]
            want[x] = m[0, 0] * a[x] + m[0, 1] * a[x1]
            want[x1] = m[1, 0] * a[x] + m[1, 1] * a[x1]
        np.testing.assert_allclose(got, want, atol=1e-15)


def test_grid_circuit_structure():
    rows, cols, layers = 3, 4, 8
    gates = workloads.grid_circuit(rows, cols, layers, 5)
    n = rows * cols
    two = [g for g in gates if g[0] != "u3"]
    assert sum(g[0] == "u3" for g in gates) == n * layers
    for g in two:
        a, b = g[1], g[2]
        ra, ca, rb, cb = a // cols, a % cols, b // cols, b % cols
        assert abs(ra - rb) + abs(ca - cb) == 1       # nearest neighbours
        assert g[0] in ("cx", "cy", "cz", "ax", "ay", "az")
