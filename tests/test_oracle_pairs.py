"""Pins of the oracle's two-qubit rounding (the generalization the paper
mentions after Fig. 2; the reading is in oracle/factor.py): the reduced
density against its definition summed term by term, its spectrum against the
singular values of the amplitude matrix, a closed-form state with a known
dominant weight, the overlap left by the projection, and the reduction to the
one-qubit formula when one qubit of the pair is in a product state."""
import math

import numpy as np
import pytest

from oracle import dense, factor

C = np.complex128


def rand_state(n, seed):
    g = np.random.default_rng(seed)
    a = g.normal(size=2 ** n) + 1j * g.normal(size=2 ** n)
    return (a / np.linalg.norm(a)).astype(C)


def rho_by_definition(a, n, t1, t2):
    """rho[m, m'] = sum over i, j that agree outside bits t1, t2 of a_i conj(a_j)."""
    rho = np.zeros((4, 4), dtype=C)
    mask = (1 << t1) | (1 << t2)
    for i in range(2 ** n):
        for j in range(2 ** n):
            if (i & ~mask) != (j & ~mask):
                continue
            mi = ((i >> t1) & 1) + 2 * ((i >> t2) & 1)
            mj = ((j >> t1) & 1) + 2 * ((j >> t2) & 1)
            rho[mi, mj] += a[i] * np.conj(a[j])
    return rho


@pytest.mark.parametrize("t1,t2", [(0, 1), (1, 0), (3, 1), (0, 4), (4, 2)])
def test_pair_density_by_definition(t1, t2):
    n = 5
    a = rand_state(n, 10 + t1 + 7 * t2)
    got = factor.pair_density(a, n, t1, t2)
    want = rho_by_definition(a, n, t1, t2)
    np.testing.assert_allclose(got, want, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_pair_spectrum_is_schmidt_weights(seed):
    """The eigenvalues of rho_B are the squared singular values of the 4 x
    2^(n-2) matrix M[m, rest] = a[index with bits t1, t2 = m]."""
    n, t1, t2 = 6, 2, 5
    a = rand_state(n, seed)
    others = [k for k in range(n) if k not in (t1, t2)]
    M = np.zeros((4, 2 ** (n - 2)), dtype=C)
    for i in range(2 ** n):
        m = ((i >> t1) & 1) + 2 * ((i >> t2) & 1)
        r = sum(((i >> k) & 1) << j for j, k in enumerate(others))
        M[m, r] = a[i]
    sv2 = np.sort(np.linalg.svd(M, compute_uv=False) ** 2)
    w = np.linalg.eigvalsh(factor.pair_density(a, n, t1, t2))
    np.testing.assert_allclose(w, sv2, atol=1e-13)
    eps, phi = factor.pair_dominant(factor.pair_density(a, n, t1, t2))
    assert abs(eps - (1.0 - sv2[-1])) < 1e-13
    assert abs(np.linalg.norm(phi) - 1.0) < 1e-13


@pytest.mark.parametrize("e", [0.0, 0.02, 0.2, 0.45])
def test_closed_form_dominant_weight(e):
    """sqrt(1-e)|Phi+>_{ab}|0>_c + sqrt(e)|Psi->_{ab}|1>_c on a = bit 0,
    b = bit 2, c = bit 1, times |+> on bit 3: rho_ab has eigenvalues 1-e and
    e, so eps_B = e; rounding at p = 2e keeps |Phi+> on the pair, |0> on c,
    and F = 1 - e."""
    n = 4
    a = np.zeros(2 ** n, dtype=C)
    for x in range(2 ** n):
        qa, qc, qb, qd = (x >> 0) & 1, (x >> 1) & 1, (x >> 2) & 1, (x >> 3) & 1
        plus = 1 / math.sqrt(2)
        if qc == 0 and qa == qb:
            a[x] = math.sqrt(1 - e) / math.sqrt(2) * plus
        if qc == 1 and qa != qb:
            a[x] = math.sqrt(e) * (1 if qa == 0 else -1) / math.sqrt(2) * plus
    eps, phi = factor.pair_dominant(factor.pair_density(a, n, 0, 2))
    assert abs(eps - min(e, 1 - e)) < 1e-13
    st = factor.FactorizedState(n)
    st.subs = [factor.Sub([0, 1, 2, 3], a.copy())]
    assert st.test_pair(0, 2, max(2 * e, 1e-9))
    assert abs(st.F - (1 - e)) < 1e-13
    pair = [s for s in st.subs if s.qubits == [0, 2]][0]
    bell = np.array([1, 0, 0, 1], dtype=C) / math.sqrt(2)
    assert abs(abs(np.vdot(bell, pair.amps)) - 1) < 1e-12
    rest = [s for s in st.subs if s.qubits == [1, 3]][0]
    want = np.kron(np.array([1, 1]) / math.sqrt(2), np.array([1, 0]))  # bit 0 = c, bit 1 = d
    assert abs(abs(np.vdot(want, rest.amps)) - 1) < 1e-12


@pytest.mark.parametrize("seed", range(3))
def test_projection_overlap_is_dominant_weight(seed):
    """|<psi|psi'>|^2 = 1 - eps_B for the projected state psi' (the kept
    Schmidt term has weight lambda_max)."""
    n = 6
    a = rand_state(n, 40 + seed)
    st = factor.FactorizedState(n)
    st.subs = [factor.Sub(list(range(n)), a.copy())]
    before = st.expand()
    assert st.test_pair(4, 1, 2.0)  # p large enough that any pair rounds
    after = st.expand()
    eps = st.log[-1].eps
    assert st.log[-1].pair == 1 and st.log[-1].rounded
    assert abs(abs(np.vdot(before, after)) ** 2 - (1 - eps)) < 1e-12
    assert abs(np.linalg.norm(after) - 1) < 1e-12


def test_pair_with_a_product_qubit_reduces_to_the_one_qubit_test():
    """If b is in a product state with the rest, rho_ab = rho_a (x) rho_b with
    rho_b pure, so eps_B equals the one-qubit eps of a, (1 - |r_a|)/2."""
    g = np.random.default_rng(3)
    rest = rand_state(4, 77)                                  # a at bit 0, others 1..3
    u = dense.u3(*g.uniform(0, 2 * math.pi, 3))
    b = u @ np.array([1, 0], dtype=C)                         # b at bit 4
    a = np.kron(b, rest)
    eps_b, _ = factor.pair_dominant(factor.pair_density(a, 5, 0, 4))
    eps_a = factor.epsilon(factor.bloch(a, 5, 0))
    assert abs(eps_b - eps_a) < 1e-12


def test_pair_policy_run_invariants():
    """A random circuit with the pair policy: F is the product of 1 - eps over
    every rounding (one- and two-qubit), the ket stays normalized, pair
    pair attempts occur, and with p = 0 the run is exact."""
    import workloads
    gates = workloads.random_circuit(10, 6, 5)
    st = factor.FactorizedState(10).run(gates, 0.3, pairs=True)
    assert any(x.pair >= 0 for x in st.log)
    prod = 1.0
    for x in st.log:
        if x.rounded:
            prod *= 1 - x.eps
    assert abs(st.F - prod) < 1e-12
    assert abs(np.linalg.norm(st.expand()) - 1) < 1e-12
    st0 = factor.FactorizedState(10).run(gates, 0.0, pairs=True)
    exact = dense.run_circuit(dense.zero_state(10), 10, gates)
    assert abs(abs(np.vdot(st0.expand(), exact)) - 1) < 1e-10


def test_pair_chain_is_what_pairs_are_for():
    """Entangled pairs weakly coupled along a chain (workloads.pair_chain_circuit):
    each pair qubit is far from a product state, so the one-qubit rounding at
    p = 0.05 lets the chain merge into one subsystem, while the two-qubit
    rounding splits every pair off; F stays the product of 1 - eps."""
    import workloads
    gates = workloads.pair_chain_circuit(12, 5, 3)
    single = factor.FactorizedState(12).run(gates, 0.05)
    pairs = factor.FactorizedState(12).run(gates, 0.05, pairs=True)
    assert max(single.sizes()) == 12
    assert pairs.sizes() == [2] * 6
    assert sum(1 for a in pairs.log if a.pair >= 0 and a.rounded) > 0
    prod = 1.0
    for a in pairs.log:
        if a.rounded:
            prod *= 1 - a.eps
    assert abs(pairs.F - prod) < 1e-12 and 0.9 < pairs.F < 1.0
