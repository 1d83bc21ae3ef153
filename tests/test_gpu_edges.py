"""Degenerate and boundary cases on the GPU: the smallest states, empty
inputs, p = 1 with a maximally mixed qubit (|r| = 0), the capacity bound
reached exactly, single-ket batches."""
import math

import numpy as np
import pytest

import workloads
from oracle import dense, factor
from parity import C64, C128, assert_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [C64, C128])
def test_one_qubit_state(qs_lib, dtype):
    qs = qs_lib
    with qs.State(1, dtype) as st:
        st.qft()  # QFT on one qubit is H
        assert_parity(st.amplitudes(), dense.qft(dense.zero_state(1), 1), dtype, "qft n=1")
        st.apply_1q(0, dense.u3(0.3, 0.2, 0.1))
        want = dense.apply_1q(dense.qft(dense.zero_state(1), 1), 1, 0, dense.u3(0.3, 0.2, 0.1))
        assert_parity(st.amplitudes(), want, dtype, "u3 n=1")
    st = qs.State(1, dtype, factorized=True)
    st.set_policy(qs.SEP_AFTER_2Q, 1.0)
    st.apply_1q(0, dense.H)
    assert st.try_separate(1.0) == 0  # nothing to separate from
    assert st.fidelity_estimate() == 1.0
    st.free()


def test_empty_inputs(qs_lib):
    qs = qs_lib
    n = 6
    with qs.State(n, C64) as st:
        st.set_basis(5)
        c = qs.Circuit(n).plan(4)  # no gates
        assert c.info()["blocks"] == 0
        st.run(c)
        assert st.gather([]).size == 0
        np.testing.assert_array_equal(st.amplitudes(), dense.basis_state(n, 5))
        c.free()
    b = qs.Batch([5], C64)  # one ket, one empty circuit
    c = qs.Circuit(5)
    b.run([c], 3)
    np.testing.assert_array_equal(b.amplitudes(0), dense.zero_state(5))
    b.free()
    c.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_bell_pair_at_p_one(qs_lib, dtype):
    """A Bell pair has |r| = 0 for both qubits (eps = 1/2): rounding happens
    only at p = 1, projects on |0> (the tie-break of the dominant eigenvector),
    and leaves F = 1/2; the oracle takes the same steps."""
    qs = qs_lib
    gates = [("h", 0), ("cx", 0, 1)]
    for p, rounds in ((0.999, 0), (1.0, 1)):
        st = qs.State(2, dtype, factorized=True)
        st.record_attempts()
        st.set_policy(qs.SEP_AFTER_2Q, p)
        st.run(qs.Circuit(2).add_gates(gates))
        att = st.attempts()
        assert sum(a[3] for a in att) == rounds
        assert abs(att[0][2] - 0.5) < 1e-7
        ost = factor.FactorizedState(2)
        ost.run(gates, p)
        assert abs(st.fidelity_estimate() - ost.F) < 1e-12
        assert_parity(st.amplitudes(), ost.expand(), dtype, f"bell p={p}")
        if rounds:
            assert abs(st.fidelity_estimate() - 0.5) < 1e-12
            np.testing.assert_allclose(np.abs(st.amplitudes()), [1, 0, 0, 0], atol=1e-6)
        st.free()


def test_capacity_bound_reached_exactly(qs_lib):
    """A merge to exactly max_amps amplitudes succeeds; one qubit more fails."""
    qs = qs_lib
    st = qs.State(5, C64, factorized=True, max_amps=2 ** 4)
    for q in range(5):
        st.apply_1q(q, dense.H)
    for a, b in ((0, 1), (1, 2), (2, 3)):
        st.apply_cphase(a, b, 1.1)
    assert max(len(s) for s in st.subsystems()) == 4
    with pytest.raises(qs.CapacityError):
        st.apply_cphase(3, 4, 1.1)
    want = dense.zero_state(5)
    for q in range(5):
        want = dense.apply_1q(want, 5, q, dense.H)
    for a, b in ((0, 1), (1, 2), (2, 3)):
        want = dense.apply_cphase(want, 5, a, b, 1.1)
    assert_parity(st.amplitudes(), want, C64, "at the cap")
    st.free()


def test_ragged_batch_widths(qs_lib):
    """Kets of every width from 1 to 12 in one arena, each with its own depth."""
    qs = qs_lib
    widths = list(range(1, 13))
    gl = [workloads.random_circuit(n, 1 + n % 4, 70 + n) for n in widths]
    circs = [qs.Circuit(n).add_gates(g) for n, g in zip(widths, gl)]
    b = qs.Batch(widths, C128)
    b.run(circs, 3)
    for i, (n, g) in enumerate(zip(widths, gl)):
        assert_parity(b.amplitudes(i), dense.run_circuit(dense.zero_state(n), n, g), C128,
                      f"ket n={n}")
    b.free()
    for c in circs:
        c.free()


def test_out_of_range_arguments(qs_lib):
    qs = qs_lib
    with pytest.raises(qs.QSError):
        qs.State(qs.MAX_QUBITS + 1, C64)
    with qs.State(4, C64) as st:
        with pytest.raises(qs.QSError):
            st.qft(2, 3)  # range past the last qubit
        with pytest.raises(qs.QSError):
            st.apply_fused([0, 0], np.eye(4))  # repeated qubit
        with pytest.raises(qs.QSError):
            st.apply_1q(0, np.array([[math.nan, 0], [0, 1]]))  # not finite
        with pytest.raises(qs.QSError):
            st.gather([16])  # index beyond 2^n
