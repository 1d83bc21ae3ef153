"""The unobservable shortcuts of the factorized mode (Sec. II-B) and the QFT on
factorized states, against the FP64 oracle and the QFT's closed forms: gates
whose control is in a Z eigenstate are dropped or made local without a merge,
so the QFT of a basis state stays a product state at 40+ qubits (the
factorized-input runs of Fig. 1a)."""
import math

import numpy as np
import pytest

import workloads
from oracle import dense
from parity import C64, C128, assert_parity

pytestmark = pytest.mark.gpu


def _knob(qs, value):
    saved = qs.tune_get("factor.unobservable")
    qs.tune_set("factor.unobservable", value)
    return saved


@pytest.mark.parametrize("dtype", [C64, C128])
def test_controls_in_z_eigenstates(qs_lib, dtype):
    """CX with control |0> (dropped), with control |1> (a local X), CP on
    |1>|+> (a phase gate), an anti-controlled Y on |0> (a local Y), a
    controlled U3 on |1>, and a CX whose *target* is |0> (no shortcut): the
    same ket as with the shortcut off, fewer merges."""
    qs = qs_lib
    n = 6
    gates = [("h", 1), ("u3", 4, 0.3, 0.2, 0.9), ("u3", 5, math.pi, 0.0, math.pi),  # q5 = |1>
             ("cx", 0, 1), ("cx", 5, 2), ("cp", 5, 1, 0.7), ("ay", 3, 4),
             ("ctrl", [5], 1, 0, 0.4, 0.1, 0.2), ("cx", 1, 3)]
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    sizes = {}
    for on in (1, 0):
        saved = _knob(qs, on)
        try:
            st = qs.State(n, dtype, factorized=True)
            st.run(qs.Circuit(n).add_gates(gates))
            assert_parity(st.amplitudes(), want, dtype, f"shortcuts={on}")
            sizes[on] = sorted(len(s) for s in st.subsystems())
            if on:
                assert st.shortcut_count() == 5
            st.free()
        finally:
            qs.tune_set("factor.unobservable", saved)
    # only the last CX (target |0>, control |+>) merges with the shortcut on
    assert sizes[1] == [1, 1, 1, 1, 2] and max(sizes[0]) > 2


@pytest.mark.parametrize("n", [10, 40, 63])
def test_qft_of_zero_state_stays_a_product(qs_lib, n):
    """QFT|0...0> = the uniform superposition: every controlled phase meets a
    control still in |0>, so the state stays n one-qubit subsystems."""
    qs = qs_lib
    st = qs.State(n, C64, factorized=True)
    st.qft()
    assert len(st.subsystems()) == n
    assert st.shortcut_count() == n * (n - 1) // 2
    idx = np.random.default_rng(n).integers(0, 2 ** min(n, 62), 256).astype(np.uint64)
    got = st.gather(idx)
    np.testing.assert_allclose(got, np.full(idx.size, 2.0 ** (-n / 2)), rtol=1e-5, atol=0)
    assert st.fidelity_estimate() == 1.0
    st.free()


@pytest.mark.parametrize("dtype,n", [(C64, 36), (C128, 24)])
def test_qft_of_basis_states_closed_form(qs_lib, dtype, n):
    """QFT|x> has the amplitudes 2^{-n/2} e^{2 pi i x y / 2^n}: sampled entries
    against the oracle's closed form; the state stays a product; the inverse
    QFT returns |x>."""
    qs = qs_lib
    for seed in (1, 2):
        x = workloads.basis_index(n, seed)
        st = qs.State(n, dtype, factorized=True)
        st.set_basis(x)
        st.qft()
        assert len(st.subsystems()) == n
        js = np.random.default_rng(seed).integers(0, 2 ** n, 512)
        want = dense.qft_basis_entries(n, x, js)
        got = st.gather(js.astype(np.uint64))
        tol = 1e-5 * 2.0 ** (-n / 2) * n if dtype == C64 else 1e-12
        assert np.abs(got - want).max() <= tol
        # the inverse meets no Z eigenstate and merges; its intermediate states
        # are products again, which exact separations (p = 0) split back off
        st.set_policy(qs.SEP_AFTER_2Q, 0.0)
        st.qft(inverse=True)
        assert max(len(s) for s in st.subsystems()) <= 2
        got = st.gather(np.array([x, (x + 1) % 2 ** n], dtype=np.uint64))
        assert abs(abs(got[0]) - 1.0) < 1e-4 and abs(got[1]) < 1e-4
        st.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_qft_of_entangled_factorized_states(qs_lib, dtype):
    """An entangled input (a random circuit at p = 0, and a GHZ state, the
    input of Fig. 1b): the factorized QFT (gate by gate, merging as needed)
    matches the oracle's dense QFT of the same ket; a sub-range too."""
    qs = qs_lib
    n = 11
    for gates in (workloads.random_circuit(n, 2, 4),
                  [("h", 0)] + [("cx", q, q + 1) for q in range(n - 1)]):
        ket = dense.run_circuit(dense.zero_state(n), n, gates)
        for start, length, inverse in ((0, n, False), (3, 6, True)):
            st = qs.State(n, dtype, factorized=True)
            st.run(qs.Circuit(n).add_gates(gates))
            st.qft(start, length, inverse)
            want = dense.run_circuit(ket, n, dense.qft_gates(n, start, length, inverse))
            assert_parity(st.amplitudes(), want, dtype, f"qft [{start},{start + length}) inv={inverse}")
            st.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_qft_twice_on_a_ghz_subsystem(qs_lib, dtype):
    """GHZ built by a CNOT chain lies in one subsystem with its qubits at
    ascending local bits: the factorized QFT runs the dense passes on that
    buffer; the second transform finds the block descending (the relabelled
    reversal of the first) and runs the passes in the other orientation."""
    qs = qs_lib
    n = 14
    gates = [("h", 0)] + [("cx", q, q + 1) for q in range(n - 1)]
    ket = dense.run_circuit(dense.zero_state(n), n, gates)
    st = qs.State(n, dtype, factorized=True)
    st.run(qs.Circuit(n).add_gates(gates))
    st.profile_start()
    st.qft()
    want = dense.qft(ket, n)
    assert_parity(st.amplitudes(), want, dtype, "qft of ghz")
    st.qft(2, 9, inverse=True)
    prof = st.profile_stop()
    assert any(k.startswith("qft_") for k in prof), prof
    want = dense.run_circuit(want, n, dense.qft_gates(n, 2, 9, True))
    assert_parity(st.amplitudes(), want, dtype, "inverse qft on a sub-range")
    st.free()


@pytest.mark.parametrize("defer", [0, 1])
def test_shortcut_after_a_deferred_rounding(qs_lib, defer):
    """An iSWAP on |00> merges two qubits that stay |00>; the (deferred) test
    splits qubit 2 back off as exactly |0>, an X makes it |1>, and the CX it
    then controls must act on its target: the host copy of the split-off
    qubit has to include the X although the rounding and the X were queued
    in the same run."""
    qs = qs_lib
    n = 5
    gates = [("iswap", 2, 3), ("u3", 2, math.pi, 0.0, math.pi), ("cx", 2, 4), ("h", 0),
             ("cx", 0, 1), ("u3", 3, 0.4, 0.1, 0.2), ("cz", 3, 2)]
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    saved = qs.tune_get("factor.defer")
    try:
        qs.tune_set("factor.defer", defer)
        st = qs.State(n, C64, factorized=True)
        st.set_policy(qs.SEP_AFTER_2Q, 0.1)
        st.run(qs.Circuit(n).add_gates(gates))
        assert_parity(st.amplitudes(), want, C64, f"defer={defer}")
        assert st.shortcut_count() >= 2
        st.free()
    finally:
        qs.tune_set("factor.defer", saved)
