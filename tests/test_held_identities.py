"""The identities behind held gates (Table I: controlled phases and
inversions moved around H; Sec. II-B: state-preserving replacements), checked
with plain matrices on the CPU. Two-qubit operators act on (control, target)
with the control as the high index bit: C(M) = |0><0| (x) I + |1><1| (x) M."""
import numpy as np
import pytest

I2 = np.eye(2, dtype=complex)
H = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
X = np.array([[0, 1], [1, 0]], dtype=complex)
Z = np.diag([1, -1]).astype(complex)
P0 = np.diag([1, 0]).astype(complex)
P1 = np.diag([0, 1]).astype(complex)


def ctrl(m):
    return np.kron(P0, I2) + np.kron(P1, m)


def on_t(u):
    return np.kron(I2, u)


def on_c(u):
    return np.kron(u, I2)


def unitary(rng):
    q, r = np.linalg.qr(rng.normal(size=(2, 2)) + 1j * rng.normal(size=(2, 2)))
    return q * (np.diag(r) / abs(np.diag(r)))


def phase(rng):
    return np.diag(np.exp(1j * rng.uniform(0, 2 * np.pi, 2)))


def inversion(rng):
    return X @ phase(rng)


def test_h_on_the_target_turns_cz_into_cx_and_back():
    np.testing.assert_allclose(on_t(H) @ ctrl(Z), ctrl(X) @ on_t(H), atol=1e-15)
    np.testing.assert_allclose(on_t(H) @ ctrl(X), ctrl(Z) @ on_t(H), atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
def test_a_target_gate_passes_by_conjugation(seed):
    rng = np.random.default_rng(seed)
    u = unitary(rng)
    for m in (phase(rng), inversion(rng)):
        np.testing.assert_allclose(on_t(u) @ ctrl(m), ctrl(u @ m @ u.conj().T) @ on_t(u),
                                   atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_control_passes_only_diagonal_gates(seed):
    rng = np.random.default_rng(seed)
    m = inversion(rng)
    d = phase(rng)
    np.testing.assert_allclose(on_c(d) @ ctrl(m), ctrl(m) @ on_c(d), atol=1e-15)
    u = unitary(rng)
    assert np.abs(on_c(u) @ ctrl(m) - ctrl(m) @ on_c(u)).max() > 1e-3


def test_a_phase_with_d0_one_is_symmetric():
    d1 = np.exp(0.7j)
    m = np.diag([1, d1])
    swap = np.eye(4)[[0, 2, 1, 3]]
    np.testing.assert_allclose(swap @ ctrl(m) @ swap, ctrl(m), atol=0)
    # but diag(d0, d1) with d0 != 1 is not
    m2 = np.diag([np.exp(0.3j), d1])
    assert np.abs(swap @ ctrl(m2) @ swap - ctrl(m2)).max() > 0.1


@pytest.mark.parametrize("seed", range(5))
def test_commutation_rules(seed):
    rng = np.random.default_rng(seed)

    def comm(a, b):
        return np.abs(a @ b - b @ a).max()

    # three qubits (a, b, c), high bit first; controlled gates between pairs
    def c3(cq, tq, m):
        out = np.zeros((8, 8), dtype=complex)
        for col in range(8):
            bits = [(col >> (2 - i)) & 1 for i in range(3)]
            if not bits[cq]:
                out[col, col] = 1
                continue
            for v in range(2):
                row = bits.copy()
                row[tq] = v
                r = sum(b << (2 - i) for i, b in enumerate(row))
                out[r, col] += m[v, bits[tq]]
        return out

    p1, p2 = phase(rng), phase(rng)
    v1, v2 = inversion(rng), inversion(rng)
    assert comm(c3(0, 1, p1), c3(2, 1, p2)) < 1e-14       # phases always
    assert comm(c3(0, 1, v1), c3(0, 2, v2)) < 1e-14       # one control
    assert comm(c3(1, 2, v1), c3(0, 1, p1)) < 1e-14       # a phase on an inversion's control
    assert comm(c3(0, 1, v1), c3(1, 2, p1)) > 1e-3        # an inversion on a phase's control
    assert comm(c3(0, 1, v1), c3(2, 1, p2)) > 1e-3        # inversion vs phase, one target
    assert comm(c3(0, 1, v1), c3(1, 2, v2)) > 1e-3        # inversion into a control
    # two inversions on one target commute iff a0 b1 = b0 a1
    a0, a1, b0 = np.exp(1j * rng.uniform(0, 6, 3))
    va = np.array([[0, a0], [a1, 0]])
    vb_yes = np.array([[0, b0], [b0 * a1 / a0, 0]])
    vb_no = np.array([[0, b0], [-b0 * a1 / a0, 0]])
    assert comm(c3(0, 1, va), c3(2, 1, vb_yes)) < 1e-14
    assert comm(c3(0, 1, va), c3(2, 1, vb_no)) > 1e-3


@pytest.mark.parametrize("seed", range(5))
def test_kickback_onto_an_eigenstate(seed):
    """C(M) on |c> (x) |v> with M v = l v equals diag(1, l) |c> (x) |v>."""
    rng = np.random.default_rng(seed)
    c = unitary(rng)[:, 0]
    for m in (X, inversion(rng), unitary(rng)):
        w, vecs = np.linalg.eig(m)
        for k in range(2):
            v = vecs[:, k]
            got = ctrl(m) @ np.kron(c, v)
            want = np.kron(np.diag([1, w[k]]) @ c, v)
            np.testing.assert_allclose(got, want, atol=1e-14)
    # |-> is X's eigenstate of eigenvalue -1: a CX onto it is a Z on the control
    minus = H @ X @ np.array([1, 0])
    np.testing.assert_allclose(ctrl(X) @ np.kron(c, minus), np.kron(Z @ c, minus), atol=1e-15)
