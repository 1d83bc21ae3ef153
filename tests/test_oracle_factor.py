"""Pins of the approximate-mode (SDRP) oracle.

Checked against constructions independent of the oracle's own formulas:
Pauli expectations from Kronecker-built operators, the SVD of the 2 x 2^{n-1}
reshaped ket (epsilon is the smaller squared Schmidt coefficient, Eq. schmidt
read with sqrt(1 - eps)), the per-rounding fidelity 1 - eps (Sec. III-B), and
hand-solvable states.
"""
import math
import os

import numpy as np
import pytest

import workloads
from oracle import dense, factor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pauli_on(n, q, P):
    return np.kron(np.kron(np.eye(2 ** (n - q - 1)), P), np.eye(2 ** q))


def svd_eps(a, n, q):
    """Smaller squared singular value of the qubit-q / rest bipartition."""
    t = np.moveaxis(a.reshape((2,) * n), n - 1 - q, 0).reshape(2, -1)
    s = np.linalg.svd(t, compute_uv=False)
    return float(s[-1] ** 2)


def random_entangled(n, seed):
    gates = workloads.random_circuit(n, 2, seed)
    return dense.run_circuit(dense.zero_state(n), n, gates)


@pytest.mark.parametrize("n", [2, 4, 6])
def test_bloch_vector_is_pauli_expectation(n):
    a = random_entangled(n, n)
    for q in range(n):
        want = [np.vdot(a, pauli_on(n, q, P) @ a).real for P in (dense.X, dense.Y, dense.Z)]
        np.testing.assert_allclose(factor.bloch(a, n, q), want, atol=1e-13)


@pytest.mark.parametrize("n", [2, 3, 5, 7])
def test_epsilon_is_smaller_schmidt_weight(n):
    for seed in range(3):
        a = random_entangled(n, 10 * n + seed)
        for q in range(n):
            eps = factor.epsilon(factor.bloch(a, n, q))
            assert abs(eps - svd_eps(a, n, q)) < 1e-12


def test_projection_fidelity_is_one_minus_eps():
    n = 6
    for seed in range(4):
        a = random_entangled(n, 50 + seed)
        for t in range(n):
            r = factor.bloch(a, n, t)
            eps = factor.epsilon(r)
            phi = factor.dominant_state(r)
            rest = factor.project_out(a, n, t, phi)
            # the product ket phi at bit t, rest on the other bits, by index loop
            out = np.empty(2 ** n, dtype=complex)
            for x in range(2 ** n):
                lo, hi = x & ((1 << t) - 1), x >> (t + 1)
                out[x] = phi[(x >> t) & 1] * rest[lo | (hi << t)]
            assert abs(np.vdot(out, out).real - 1.0) < 1e-12
            assert abs(abs(np.vdot(out, a)) ** 2 - (1.0 - eps)) < 1e-12
            # phi is the dominant eigenvector of rho_q = (I + r.sigma)/2
            rho = 0.5 * (np.eye(2) + r[0] * dense.X + r[1] * dense.Y + r[2] * dense.Z)
            assert abs(np.vdot(phi, rho @ phi).real - (1 + np.linalg.norm(r)) / 2) < 1e-12


def load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    return rows


def test_golden_weakly_entangled_pair():
    """sqrt(1-e)|00> + sqrt(e)|11>: eps = e; rounding at p >= 2e leaves |00>
    with fidelity 1-e (Eq. schmidt, Eq. sdrp, Sec. III-B)."""
    for e, p, rounds, F_want in load_golden("sdrp_pair.txt"):
        st = factor.FactorizedState(2)
        amps = np.zeros(4, dtype=complex)
        amps[0], amps[3] = math.sqrt(1 - e), math.sqrt(e)
        st.subs = [factor.Sub([0, 1], amps)]
        st.dirty = {0, 1}
        n_sep = st.try_separate(p)
        assert st.log[0].eps == pytest.approx(e, abs=1e-14)
        assert n_sep == int(rounds)
        assert st.F == pytest.approx(F_want, abs=1e-14)
        if rounds:
            np.testing.assert_allclose(st.expand(), [1, 0, 0, 0], atol=1e-14)
            assert abs(dense.fidelity(st.expand(), amps) - (1 - e)) < 1e-14
        else:
            np.testing.assert_allclose(st.expand(), amps, atol=1e-15)


def test_product_state_separates_without_loss():
    n = 5
    st = factor.FactorizedState(n)
    for q in range(n):
        st.apply_gate(("u3", q, 0.3 + q, 1.1 * q, 0.2))
    # merge everything with CZ then undo it: a product state in one subsystem
    for q in range(n - 1):
        st.apply_gate(("cz", q, q + 1))
    for q in range(n - 2, -1, -1):
        st.apply_gate(("cz", q, q + 1))
    assert max(st.sizes()) == n
    exact = st.expand().copy()
    st.dirty = set(range(n))
    assert st.try_separate(0.0) == n - 1
    assert st.sizes() == [1] * n
    assert abs(st.F - 1.0) < 1e-12
    assert abs(dense.fidelity(st.expand(), exact) - 1.0) < 1e-12


def test_bell_rounds_only_at_p_one():
    for p, want in [(0.0, 0), (0.5, 0), (0.99, 0), (1.0, 1)]:
        st = factor.FactorizedState(2)
        st.apply_gate(("h", 0))
        st.apply_gate(("ctrl", (0,), 1, 1, math.pi, 0.0, math.pi))  # CNOT
        assert st.try_separate(p) == want
        if want:
            assert st.F == pytest.approx(0.5, abs=1e-14)


def test_fidelity_model_exact_for_disjoint_pairs():
    """Disjoint pairs each rounded once: the neglected branches stay orthogonal,
    so F = prod(1 - eps_j) equals |<approx|exact>|^2 (Eq. fid_model)."""
    n = 8
    g = np.random.default_rng(3)
    st = factor.FactorizedState(n)
    gates = []
    for q in range(0, n, 2):
        th = float(g.uniform(0.05, 0.4))
        gates += [("u3", q, th, 0.0, 0.0), ("ctrl", (q,), 1, q + 1, math.pi, 0.0, math.pi),
                  ("u3", q, 0.7, 0.2, 0.1), ("u3", q + 1, 1.3, 0.4, 0.9)]
    exact = dense.run_circuit(dense.zero_state(n), n, gates)
    st.run(gates, p=0.2)
    assert len([a for a in st.log if a.rounded]) == n // 2
    F_exact = dense.fidelity(st.expand(), exact)
    assert st.F == pytest.approx(F_exact, abs=1e-12)
    assert st.F < 0.99


@pytest.mark.parametrize("seed", range(3))
def test_exact_mode_matches_dense(seed):
    """At p = 0 only numerically exact separations happen: the factorized run
    reproduces the dense ket."""
    n = 7
    gates = workloads.random_circuit(n, 4, seed)
    st = factor.FactorizedState(n).run(gates, p=0.0)
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    assert abs(st.F - 1.0) < 1e-9
    assert dense.fidelity(st.expand(), want) > 1 - 1e-10


def test_merge_is_kron_and_keeps_reduced_states():
    st = factor.FactorizedState(4)
    for q in range(4):
        st.apply_gate(("u3", q, 0.4 * (q + 1), 0.3, 0.2 * q))
    st.apply_gate(("iswap", 0, 1))
    st.apply_gate(("iswap", 2, 3))
    before = st.expand()
    rs = []
    for q in range(4):
        si, t = st.where(q)
        S = st.subs[si]
        rs.append(factor.bloch(S.amps, len(S.qubits), t))
    si = st.merge(1, 3)
    S = st.subs[si]
    assert sorted(S.qubits) == [0, 1, 2, 3]
    np.testing.assert_allclose(st.expand(), before, atol=1e-14)
    for q in range(4):
        t = S.qubits.index(q)
        np.testing.assert_allclose(factor.bloch(S.amps, 4, t), rs[q], atol=1e-13)


def test_eps_invariant_under_local_gates():
    n = 5
    a = random_entangled(n, 77)
    eps0 = [factor.epsilon(factor.bloch(a, n, q)) for q in range(n)]
    b = dense.apply_1q(a, n, 2, dense.u3(0.9, 0.1, 2.0))
    b = dense.apply_matrix(b, n, [0, 4], dense.ISWAP)
    eps1 = [factor.epsilon(factor.bloch(b, n, q)) for q in range(n)]
    for q in (1, 2, 3):
        assert abs(eps0[q] - eps1[q]) < 1e-12


def test_capacity_error_leaves_state_unchanged():
    st = factor.FactorizedState(6, max_amps=2 ** 3)
    st.apply_gate(("h", 0))
    st.apply_gate(("cz", 0, 1))
    st.apply_gate(("h", 2))
    st.apply_gate(("cz", 1, 2))
    before = st.expand().copy()
    sizes = st.sizes()
    with pytest.raises(factor.CapacityError):
        st.apply_gate(("cz", 2, 3))
    assert st.sizes() == sizes
    np.testing.assert_allclose(st.expand(), before, atol=0)


def test_decisions_obey_rule_and_F_nonincreasing():
    n = 10
    gates = workloads.random_circuit(n, 5, 21)
    st = factor.FactorizedState(n)
    Fs = []
    for g in gates:
        st.apply_gate(g)
        if g[0] in ("cz", "iswap"):
            st.try_separate(0.1)
        Fs.append(st.F)
    assert all(b <= a + 1e-15 for a, b in zip(Fs, Fs[1:]))
    for att in st.log:
        assert att.rounded == (att.eps <= 0.05 + factor.TAU)
    assert abs(dense.norm2(st.expand()) - 1) < 1e-12


def load_schedule_cases(name):
    """Parse the hand-worked schedule cases (format in the file's header)."""
    cases, cur = [], None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if not line:
                continue
            kind, args = line[0], line[1:]
            if kind == "case":
                cur = {"name": args[0], "n": int(args[1]), "p": float(args[2]),
                       "amps": {}, "atts": [], "F": None}
                cases.append(cur)
            elif kind == "amp":
                cur["amps"][int(args[0])] = float(args[1])
            elif kind == "att":
                cur["atts"].append((int(args[0]), int(args[1]), bool(int(args[2])), float(args[3])))
            elif kind == "F":
                cur["F"] = float(args[0])
    return cases


@pytest.mark.parametrize("case", load_schedule_cases("sdrp_schedule.txt"), ids=lambda c: c["name"])
def test_golden_schedule_order(case):
    """The attempt sequence (qubit, n_S, rounded, eps) of the dirty-set
    schedule inside one subsystem, worked by hand (Sec. III-A, Eq. sdrp)."""
    n = case["n"]
    amps = np.zeros(2 ** n, dtype=complex)
    for idx, w in case["amps"].items():
        amps[idx] = math.sqrt(w)
    st = factor.FactorizedState(n)
    st.subs = [factor.Sub(list(range(n)), amps)]
    st.dirty = set(range(n))
    st.try_separate(case["p"])
    got = [(a.qubit, a.n_sub, a.rounded) for a in st.log]
    assert got == [(q, ns, r) for q, ns, r, _ in case["atts"]]
    for a, (_, _, _, e) in zip(st.log, case["atts"]):
        assert a.eps == pytest.approx(e, abs=1e-12)
    assert st.F == pytest.approx(case["F"], abs=1e-12)
    assert not st.dirty


def fixed_point_violations(family, seeds=range(40),
                           ps=(0.05, 0.15, 0.25, 0.35, 0.45, 0.55, 0.65, 0.75, 0.85, 0.95)):
    """Runs whose end state still holds a testable qubit: one with eps <= p/2
    inside a multi-qubit subsystem. eps is taken from the SVD of the qubit /
    rest bipartition, not from the oracle's Bloch vector."""
    bad = []
    for seed in seeds:
        gates = (workloads.random_circuit(8, 4, 1000 + seed) if family == "matching"
                 else workloads.grid_circuit(2, 4, 4, 1000 + seed))
        for p in ps:
            st = factor.FactorizedState(8).run(gates, p)
            for S in st.subs:
                nq = len(S.qubits)
                if nq < 2:
                    continue
                for t in range(nq):
                    if svd_eps(S.amps, nq, t) <= p / 2.0 + factor.TAU - 1e-10:
                        bad.append((seed, p, S.qubits[t]))
    return bad


@pytest.mark.parametrize("family", ["matching", "grid"])
def test_schedule_reaches_fixed_point(family):
    """After a run no rounding is left undone: every qubit that shares a
    subsystem with others has eps > p/2 (Eq. sdrp). The dirty-set schedule is
    exhaustive only if every co-member of a rounded qubit is retested."""
    assert fixed_point_violations(family) == []


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_logged_schedule_replays_itself(seed):
    """Replaying a plain run's own attempts (their gate counts and qubits)
    with run_tests_as_logged repeats the run: the same attempts, the same
    fidelity estimate and the same ket."""
    n, p = 8, 0.3
    gates = workloads.random_circuit(n, 5, 40 + seed)
    a = factor.FactorizedState(n).run(gates, p)
    assert any(x.rounded for x in a.log) and len(a.log) > 10
    sched = [(x.gates, x.qubit) for x in a.log]
    # the counts are those of the multi-qubit gates that preceded each attempt
    assert all(0 < k <= sum(1 for g in gates if len(dense.gate_matrix(g)[0]) >= 2)
               for k, _ in sched)
    assert [k for k, _ in sched] == sorted(k for k, _ in sched)
    b = factor.FactorizedState(n).run_tests_as_logged(gates, p, sched)
    assert [(x.qubit, x.n_sub, x.eps, x.rounded, x.gates) for x in b.log] == \
        [(x.qubit, x.n_sub, x.eps, x.rounded, x.gates) for x in a.log]
    assert b.F == a.F
    assert np.array_equal(b.expand(), a.expand())


@pytest.mark.parametrize("seed", [3, 4])
def test_any_logged_schedule_is_exact_at_p_zero(seed):
    """At p = 0 only exactly separable qubits are rounded, so any choice of
    tests (here a random subset of qubits after each multi-qubit gate, in
    random order, including qubits not touched by the gate) leaves the
    circuit's ket (Sec. II-A: the factorized form is exact); testing nothing
    keeps F = 1 and the ket too, at any p."""
    n = 8
    gates = workloads.random_circuit(n, 4, seed)
    # an early CZ between freshly rotated qubits leaves many separable moments
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    g = np.random.default_rng(seed)
    k_total = sum(1 for gg in gates if len(dense.gate_matrix(gg)[0]) >= 2)
    sched = []
    for k in range(1, k_total + 1):
        for q in g.permutation(n)[: int(g.integers(0, 4))]:
            sched.append((k, int(q)))
    s = factor.FactorizedState(n, tau=1e-12).run_tests_as_logged(gates, 0.0, sched)
    assert abs(abs(np.vdot(s.expand(), want)) - 1.0) < 1e-10
    assert s.F > 1 - 1e-10
    none = factor.FactorizedState(n).run_tests_as_logged(gates, 0.9, [])
    assert none.F == 1.0 and not none.log
    assert np.abs(none.expand() - want).max() < 1e-12


def test_logged_schedule_outside_the_list_is_refused():
    n = 4
    gates = [("h", 0), ("cz", 0, 1), ("h", 2), ("cz", 2, 3)]
    with pytest.raises(ValueError):
        factor.FactorizedState(n).run_tests_as_logged(gates, 0.1, [(3, 0)])
    with pytest.raises(ValueError):  # counts must not go back
        factor.FactorizedState(n).run_tests_as_logged(gates, 0.1, [(2, 0), (1, 1)])
