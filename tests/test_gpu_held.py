"""Held gates of the factorized mode (Table I: controlled phases and
inversions buffered and moved around H; Sec. II-B: any transformation that
leaves the state unchanged is allowed), against the FP64 oracle: the ket is
the circuit's whether gates are held or not, and held gates that cancel, fold
or kick back onto an eigenstate never merge their subsystems."""
import math

import numpy as np
import pytest

import workloads
from oracle import dense
from parity import C64, C128, assert_parity, compare

pytestmark = pytest.mark.gpu


def _run(qs, n, dtype, gates, hold):
    saved = qs.tune_get("factor.hold")
    qs.tune_set("factor.hold", hold)
    try:
        st = qs.State(n, dtype, factorized=True)
        st.run(qs.Circuit(n).add_gates(gates))
        return st
    finally:
        qs.tune_set("factor.hold", saved)


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_held_gate_mix_matches_the_oracle(qs_lib, dtype, seed):
    """300 gates of CZ/CX/CY/CP/anti-controlled X with H, Paulis, phases and
    a few general U3 on 10 qubits: the same ket as the oracle with gates held
    and without, and some gates held."""
    qs = qs_lib
    n = 10
    gates = workloads.held_gate_mix(n, 300, seed)
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    for hold in (1, 0):
        st = _run(qs, n, dtype, gates, hold)
        assert_parity(st.amplitudes(), want, dtype, f"hold={hold} seed={seed}")
        held, removed = st.held_count()
        if hold:
            assert held > 0 and removed <= held
        else:
            assert held == 0
        st.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_cancelling_and_conjugated_pairs(qs_lib, dtype):
    """|+>^6; CZ(0,1) twice cancels; CZ(2,3), H(3), CX(2,3): H turns the held
    CZ into a CX, which the second CX cancels; CP(4,5, pi/4) then
    CP(5,4, -pi/4) (the same phase read from the other side) cancels; no
    subsystem ever merges."""
    qs = qs_lib
    n = 6
    gates = [("h", q) for q in range(n)]
    gates += [("cz", 0, 1), ("cz", 0, 1), ("cz", 2, 3), ("h", 3), ("cx", 2, 3),
              ("cp", 4, 5, math.pi / 4), ("cp", 5, 4, -math.pi / 4)]
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    st = _run(qs, n, dtype, gates, 1)
    assert_parity(st.amplitudes(), want, dtype, "held pairs")
    assert sorted(len(s) for s in st.subsystems()) == [1] * n
    assert st.held_count() == (6, 6)
    st.free()
    st = _run(qs, n, dtype, gates, 0)
    assert_parity(st.amplitudes(), want, dtype, "not held")
    assert max(len(s) for s in st.subsystems()) == 2
    st.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_a_held_gate_meets_a_noncommuting_one(qs_lib, dtype):
    """A held CX(0->1) then a general U3 on its control (no pass): the CX is
    applied first and the ket equals the oracle's; a held CZ then a diagonal
    phase on either qubit passes."""
    qs = qs_lib
    n = 4
    gates = [("h", 0), ("u3", 1, 0.4, 0.3, 0.2), ("cx", 0, 1), ("u3", 0, 0.7, 0.1, 0.5),
             ("h", 2), ("h", 3), ("cz", 2, 3), ("u3", 2, 0.0, 0.0, 0.9),
             ("u3", 3, 0.0, 0.0, -0.4)]
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    st = _run(qs, n, dtype, gates, 1)
    assert_parity(st.amplitudes(), want, dtype, "noncommuting")
    assert st.held_count() == (2, 0)
    assert sorted(len(s) for s in st.subsystems()) == [2, 2]
    st.free()


@pytest.mark.parametrize("n", [12, 55])
def test_phase_kickback_keeps_a_product(qs_lib, n):
    """Bernstein-Vazirani on n qubits: each CX onto the ancilla in |-> acts as
    a Z on its control (the kickback shortcut), so the state stays n one-qubit
    subsystems at any width, and the data qubits read the secret. At 12 qubits
    the same without holding merges, with the same ket as the oracle."""
    qs = qs_lib
    gates, secret = workloads.phase_kickback_circuit(n, n)
    assert sum(secret) > 2
    st = _run(qs, n, C128, gates, 1)
    assert sorted(len(s) for s in st.subsystems()) == [1] * n
    s = sum(b << q for q, b in enumerate(secret))
    got = st.gather(np.array([s, s | (1 << (n - 1))], dtype=np.uint64))
    np.testing.assert_allclose(got, [2 ** -0.5, -(2 ** -0.5)], rtol=0, atol=1e-12)
    assert st.held_count()[0] == 0 and st.shortcut_count() >= sum(secret)
    if n <= 12:
        want = dense.run_circuit(dense.zero_state(n), n, gates)
        assert_parity(st.amplitudes(), want, C128, "kickback")
        st.free()
        st = _run(qs, n, C128, gates, 0)
        assert max(len(x) for x in st.subsystems()) == sum(secret) + 1
        assert_parity(st.amplitudes(), want, C128, "kickback off")
    st.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_qft_of_product_states_with_holding(qs_lib, dtype):
    """The factorized QFT (gate by gate) of a random product state and of a
    GHZ state with holding on: the oracle's ket."""
    qs = qs_lib
    n = 9
    prod = workloads.haar_product_gates(n, 4)
    ghz = [("h", 0)] + [("cx", 0, q) for q in range(1, n)]
    for pre in (prod, ghz):
        gates = pre + dense.qft_gates(n)
        want = dense.run_circuit(dense.zero_state(n), n, gates)
        st = _run(qs, n, dtype, pre, 1)
        st.qft()
        assert_parity(st.amplitudes(), want, dtype, "qft")
        st.free()


def test_holding_is_off_under_a_separation_policy(qs_lib):
    """With a separation policy the gates are applied as they come (no held
    gates), so the tests see every gate's effect; at p = 0 only roundings of
    eps <= tau (1e-6) happen, so the ket stays within their sum of the
    oracle's."""
    qs = qs_lib
    n = 8
    gates = workloads.held_gate_mix(n, 120, 9)
    st = qs.State(n, C128, factorized=True)
    st.set_policy(qs.SEP_AFTER_2Q, 0.0)
    st.run(qs.Circuit(n).add_gates(gates))
    assert st.held_count() == (0, 0)
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    assert compare(st.amplitudes(), want, C128)["infidelity"] <= 1e-3
    st.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_held_gates_with_relabels_and_wider_gates(qs_lib, dtype):
    """The gate mix with SWAPs (relabels of the circuit's positions), iSWAPs
    (two-qubit gates that are neither phase nor inversion) and random
    three-qubit unitaries (which apply the held gates on all three qubits
    first) interleaved: the oracle's ket."""
    qs = qs_lib
    n = 9
    g = np.random.default_rng(17)
    gates = []
    for i, gate in enumerate(workloads.held_gate_mix(n, 240, 17)):
        gates.append(gate)
        if i % 15 == 7:
            a, b = (int(v) for v in g.choice(n, 2, replace=False))
            gates.append(("swap", a, b))
        if i % 40 == 20:
            a, b = (int(v) for v in g.choice(n, 2, replace=False))
            gates.append(("iswap", a, b))
        if i % 60 == 30:
            qs3 = [int(v) for v in g.choice(n, 3, replace=False)]
            z = g.normal(size=(8, 8)) + 1j * g.normal(size=(8, 8))
            u, _ = np.linalg.qr(z)
            gates.append(("mat", qs3, u))
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    st = _run(qs, n, dtype, gates, 1)
    assert_parity(st.amplitudes(), want, dtype, "relabels and wider gates")
    assert st.held_count()[0] > 0
    st.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_kickback_onto_y_eigenstates(qs_lib, dtype):
    """A CY onto |+i> (eigenvalue +1) disappears, a CY onto |-i> (eigenvalue
    -1) is a Z on its control: no merge, the oracle's ket."""
    qs = qs_lib
    n = 4
    gates = [("h", 0), ("h", 1), ("u3", 1, 0.0, 0.0, math.pi / 2), ("cy", 0, 1),
             ("h", 3), ("h", 2), ("u3", 2, 0.0, 0.0, -math.pi / 2), ("cy", 3, 2), ("h", 3)]
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    st = _run(qs, n, dtype, gates, 1)
    assert_parity(st.amplitudes(), want, dtype, "cy kickback")
    assert sorted(len(s) for s in st.subsystems()) == [1] * n
    assert st.shortcut_count() == 2 and st.held_count() == (0, 0)
    st.free()


def test_kickback_has_its_own_switch(qs_lib):
    """factor.kickback = 0 keeps holding on but turns the kickback shortcut
    off: Bernstein-Vazirani then merges the ancilla with the qubits of the
    secret, and the ket is still the oracle's."""
    qs = qs_lib
    n = 12
    gates, secret = workloads.phase_kickback_circuit(n, n)
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    saved = qs.tune_get("factor.kickback")
    qs.tune_set("factor.kickback", 0)
    try:
        st = _run(qs, n, C128, gates, 1)
    finally:
        qs.tune_set("factor.kickback", saved)
    assert max(len(x) for x in st.subsystems()) == sum(secret) + 1
    assert_parity(st.amplitudes(), want, C128, "hold on, kickback off")
    st.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_failed_run_applies_the_held_gates(qs_lib, dtype):
    """A run that fails (a merge past the cap) with a gate held back leaves
    the prefix of the circuit before the failing gate, the held gate
    included; the state stays usable."""
    qs = qs_lib
    n = 6
    prefix = ([("h", q) for q in range(n)] + [("iswap", 0, 1), ("iswap", 1, 2),
                                               ("cp", 3, 4, 0.7)])
    gates = prefix + [("iswap", 2, 5), ("h", 0)]
    saved = qs.tune_get("factor.hold")
    qs.tune_set("factor.hold", 1)
    try:
        st = qs.State(n, dtype, factorized=True, max_amps=2 ** 3)
        c = qs.Circuit(n).add_gates(gates)
        with pytest.raises(qs.CapacityError):
            st.run(c)
        c.free()
    finally:
        qs.tune_set("factor.hold", saved)
    assert sorted(sorted(s) for s in st.subsystems()) == [[0, 1, 2], [3, 4], [5]]
    want = dense.run_circuit(dense.zero_state(n), n, prefix)
    assert_parity(st.amplitudes(), want, dtype, "prefix with the held gate")
    assert st.fidelity_estimate() == 1.0
    st.free()


def test_failed_run_whose_held_gate_cannot_merge_poisons_the_state(qs_lib):
    """If a held gate cannot be applied after the failure either (its merge
    is past the cap too), the state is none of the circuit's: every later call
    but qs_free is refused."""
    qs = qs_lib
    n = 6
    gates = ([("h", q) for q in range(n)] + [("iswap", 0, 1), ("iswap", 1, 2),
                                             ("cp", 2, 3, 0.7), ("iswap", 0, 4)])
    saved = qs.tune_get("factor.hold")
    qs.tune_set("factor.hold", 1)
    try:
        st = qs.State(n, C64, factorized=True, max_amps=2 ** 3)
        c = qs.Circuit(n).add_gates(gates)
        with pytest.raises(qs.CapacityError):
            st.run(c)
        c.free()
    finally:
        qs.tune_set("factor.hold", saved)
    with pytest.raises(qs.QSError) as e:
        st.norm()
    assert e.value.code == -4
    with pytest.raises(qs.QSError):
        st.amplitudes()
    st.free()
