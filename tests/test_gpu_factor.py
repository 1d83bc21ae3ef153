"""Approximate (SDRP) mode on the GPU against the FP64 oracle.

Decisions are compared by replay: the oracle recomputes eps on its own state
for every attempt; the two decisions must agree unless the oracle's eps lies
within 1e-5 of the threshold p/2 (complex64 rounding can move eps by ~1e-7),
in which case the oracle follows the GPU's decision. Then the attempt
sequences, the fidelity estimates and the expanded kets must match."""
import math
import os

import numpy as np
import pytest

import workloads
from oracle import dense, factor
from parity import C64, C128, assert_parity

pytestmark = pytest.mark.gpu
NEAR = 1e-5


def gpu_run(qs, n, gates, p, dtype=C64, max_amps=2 ** 30):
    st = qs.State(n, dtype, factorized=True, max_amps=max_amps)
    st.set_policy(qs.SEP_AFTER_2Q, p)
    st.record_attempts()
    c = qs.Circuit(n).add_gates(gates)
    st.run(c)
    return st


def replay(n, gates, p, attempts, eps_tol):
    it = iter(attempts)
    seen = []

    def decide(q, nsub, eps, rule):
        gq, gn, geps, grounded = next(it)
        assert (gq, gn) == (q, nsub), f"attempt {len(seen)}: gpu {(gq, gn)} oracle {(q, nsub)}"
        assert abs(geps - eps) <= eps_tol, (len(seen), geps, eps)
        seen.append(q)
        if abs(eps - p / 2) < NEAR:
            return grounded
        assert grounded == rule, (len(seen), q, eps, p)
        return rule

    ost = factor.FactorizedState(n, decide=decide)
    ost.run(gates, p)
    assert next(it, None) is None, "GPU made more attempts than the oracle"
    return ost


@pytest.mark.parametrize("dtype", [C64, C128])
def test_exact_mode_matches_dense(qs_lib, dtype):
    qs = qs_lib
    n = 12
    gates = workloads.random_circuit(n, 5, 3)
    st = gpu_run(qs, n, gates, 0.0, dtype)
    assert st.fidelity_estimate() > 1 - 1e-5
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    assert_parity(st.amplitudes(), want, dtype, "factorized p=0")
    st.free()


@pytest.mark.parametrize("n,layers,p,seed", [(10, 6, 0.05, 1), (10, 6, 0.2, 2), (14, 5, 0.1, 3),
                                             (14, 7, 0.3, 4), (16, 4, 0.05, 5)])
def test_sdrp_decision_replay(qs_lib, n, layers, p, seed):
    qs = qs_lib
    gates = workloads.random_circuit(n, layers, seed)
    st = gpu_run(qs, n, gates, p)
    att = st.attempts()
    ost = replay(n, gates, p, att, eps_tol=2e-5)
    assert len(att) == len(ost.log)
    # each attempt at the same place in the circuit (deferred or not)
    assert st.attempt_gates() == [a.gates for a in ost.log]
    assert sum(a[3] for a in att) == sum(a.rounded for a in ost.log)
    F = st.fidelity_estimate()
    assert abs(F - ost.F) <= 1e-5 * max(ost.F, 1e-3) + 1e-7, (F, ost.F)
    assert sorted(len(s) for s in st.subsystems()) == ost.sizes()
    got = st.amplitudes()
    want = ost.expand()
    assert_parity(got, want, C64, f"sdrp n={n} p={p}")
    st.free()


def test_sdrp_replay_complex128(qs_lib):
    qs = qs_lib
    n, p = 12, 0.15
    gates = workloads.random_circuit(n, 6, 9)
    st = gpu_run(qs, n, gates, p, C128)
    att = st.attempts()
    ost = replay(n, gates, p, att, eps_tol=1e-10)
    assert abs(st.fidelity_estimate() - ost.F) < 1e-10
    assert_parity(st.amplitudes(), ost.expand(), C128, "c128 sdrp")
    st.free()


def test_golden_pair_on_gpu(qs_lib):
    """sqrt(1-e)|00> + sqrt(e)|11> (tests/golden/sdrp_pair.txt): eps = e, the
    rule eps <= p/2, fidelity 1 - e."""
    qs = qs_lib
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "sdrp_pair.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    # the state is built by gates; at e = 0 the CX control is exactly |0>,
    # which the Z-eigenstate shortcut would drop (no merge, nothing to test)
    saved = qs.tune_get("factor.unobservable")
    qs.tune_set("factor.unobservable", 0)
    try:
        _golden_rows(qs, rows)
    finally:
        qs.tune_set("factor.unobservable", saved)


def _golden_rows(qs, rows):
    for e, p, rounds, F_want in rows:
        st = qs.State(2, C128, factorized=True)
        st.record_attempts()
        th = 2 * math.acos(math.sqrt(1 - e))
        st.apply_1q(0, np.array([[math.cos(th / 2), -math.sin(th / 2)],
                                 [math.sin(th / 2), math.cos(th / 2)]]))
        st.apply_ctrl([0], 1, 1, np.array([[0, 1], [1, 0]]))
        assert st.try_separate(p) == int(rounds)
        a = st.attempts()[0]
        assert abs(a[2] - e) < 1e-12
        assert abs(st.fidelity_estimate() - F_want) < 1e-12
        if rounds:
            np.testing.assert_allclose(st.amplitudes(), [1, 0, 0, 0], atol=1e-12)
        st.free()


def test_capacity_leaves_state_unchanged(qs_lib):
    qs = qs_lib
    st = qs.State(6, C64, factorized=True, max_amps=2 ** 3)
    for q in range(4):
        st.apply_1q(q, dense.H)
    st.apply_cphase(0, 1, 0.7)
    st.apply_cphase(1, 2, 0.4)
    before = st.amplitudes()
    sizes = sorted(len(s) for s in st.subsystems())
    with pytest.raises(qs.CapacityError):
        st.apply_cphase(2, 3, 0.9)
    assert sorted(len(s) for s in st.subsystems()) == sizes
    np.testing.assert_array_equal(st.amplitudes(), before)
    st.apply_1q(5, dense.H)  # still usable
    st.free()


def test_factorized_gate_kinds_and_relabels(qs_lib):
    qs = qs_lib
    n = 9
    g = np.random.default_rng(2)
    st = qs.State(n, C64, factorized=True)
    want = dense.zero_state(n)
    for it in range(60):
        kind = int(g.integers(0, 5))
        if kind == 0:
            q = int(g.integers(0, n))
            m = dense.u3(*g.uniform(0, 2 * math.pi, 3))
            st.apply_1q(q, m)
            want = dense.apply_1q(want, n, q, m)
        elif kind == 1:
            a, b = (int(v) for v in g.choice(n, 2, replace=False))
            st.apply_cphase(a, b, 0.37 * it)
            want = dense.apply_cphase(want, n, a, b, 0.37 * it)
        elif kind == 2:
            a, b = (int(v) for v in g.choice(n, 2, replace=False))
            st.apply_swap(a, b)
            want = dense.apply_swap(want, n, a, b)
        elif kind == 3:
            qq = [int(v) for v in g.choice(n, 3, replace=False)]
            m = dense.u3(*g.uniform(0, 2 * math.pi, 3))
            st.apply_ctrl(qq[:2], 2, qq[2], m)
            want = dense.apply_ctrl(want, n, qq[:2], 2, qq[2], m)
        else:
            qq = [int(v) for v in g.choice(n, 2, replace=False)]
            st.apply_fused(qq, dense.ISWAP)
            want = dense.apply_matrix(want, n, qq, dense.ISWAP)
        if it % 10 == 9:
            st.mark_dirty((1 << n) - 1)
            st.try_separate(0.0)
    assert_parity(st.amplitudes(), want, C64, "gate kinds")
    idx = np.random.default_rng(0).integers(0, 2 ** n, 64)
    np.testing.assert_allclose(st.gather(idx), want[idx], atol=2e-6)
    assert abs(st.norm() - 1) < 1e-5
    st.free()


def test_fidelity_exact_pipeline(qs_lib):
    """F_exact = |<approx|exact>|^2 (Eq. fid_exact) from GPU states equals the
    oracle's value for the same decisions."""
    qs = qs_lib
    n, p = 16, 0.1
    gates = workloads.random_circuit(n, 6, 11)
    st = gpu_run(qs, n, gates, p)
    ost = replay(n, gates, p, st.attempts(), eps_tol=2e-5)
    approx = qs.State(n, C64)
    st.expand_into(approx)
    exact = qs.State(n, C64)
    exact.run(qs.Circuit(n).add_gates(gates))
    F_gpu = abs(approx.inner(exact)) ** 2
    F_orc = dense.fidelity(ost.expand(), dense.run_circuit(dense.zero_state(n), n, gates))
    assert abs(F_gpu - F_orc) < 2e-5, (F_gpu, F_orc)
    assert 0 < st.fidelity_estimate() <= 1
    for s in (st, approx, exact):
        s.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_multi_qubit_sweeps_keep_the_decisions(qs_lib, dtype):
    """Measuring several dirty qubits of a subsystem in one sweep gives the
    attempt sequence of one sweep per qubit (same qubits, sizes and decisions;
    eps equal up to summation order)."""
    qs = qs_lib
    n = 16
    saved = qs.tune_get("factor.multi_test")
    logs, fs = [], []
    try:
        for multi in (0, 1):
            qs.tune_set("factor.multi_test", multi)
            for gates, p in ((workloads.grid_circuit(4, 4, 6, 2), 0.3),
                             (workloads.random_circuit(n, 6, 8), 0.2)):
                st = gpu_run(qs, n, gates, p, dtype)
                logs.append(st.attempts())
                fs.append(st.fidelity_estimate())
                st.free()
    finally:
        qs.tune_set("factor.multi_test", saved)
    tol = 1e-9 if dtype == C128 else 1e-6
    for a, b in zip(logs[:2], logs[2:]):
        assert len(a) == len(b) and len(a) > 20
        assert [(x[0], x[1], x[3]) for x in a] == [(x[0], x[1], x[3]) for x in b]
        assert max(abs(x[2] - y[2]) for x, y in zip(a, b)) <= tol
    for fa, fb in zip(fs[:2], fs[2:]):
        assert abs(fa - fb) <= 1e-9 * max(1.0, fa) + tol


@pytest.mark.parametrize("dtype", [C64, C128])
def test_batched_one_qubit_runs(qs_lib, dtype):
    """Runs of one-qubit gates in one launch over the small subsystems (held in
    LDS) and per-gate launches on the large ones: the ket of a state with a
    13-qubit subsystem and three one-qubit ones after a run of 2000 one-qubit
    gates (more than one table slot holds, so items continue in a second
    launch) matches the dense oracle; decisions of SDRP runs, whose many short
    runs cycle through every table slot, are those of one launch per gate."""
    qs = qs_lib
    n = 16
    g = np.random.default_rng(21)
    gates = [("h", 0)] + [("cx", q, q + 1) for q in range(12)]
    for _ in range(2000):
        gates.append(("u3", int(g.integers(0, n)), *g.uniform(0, 2 * math.pi, 3)))
    saved = qs.tune_get("factor.batch_1q")
    try:
        qs.tune_set("factor.batch_1q", 1)
        st = gpu_run(qs, n, gates, 0.0, dtype)
        assert sorted(len(s) for s in st.subsystems()) == [1, 1, 1, 13]
        want = dense.run_circuit(dense.zero_state(n), n, gates)
        assert_parity(st.amplitudes(), want, dtype, "2000 one-qubit gates")
        st.free()
        logs, amps = [], []
        for batch in (0, 1):
            qs.tune_set("factor.batch_1q", batch)
            for gl, p in ((workloads.grid_circuit(4, 4, 8, 3), 0.3),
                          (workloads.random_circuit(n, 8, 12), 0.2)):
                st = gpu_run(qs, n, gl, p, dtype)
                logs.append(st.attempts())
                amps.append(st.amplitudes())
                st.free()
    finally:
        qs.tune_set("factor.batch_1q", saved)
    tol = 1e-9 if dtype == C128 else 2e-5
    for a, b in zip(logs[:2], logs[2:]):
        assert len(a) == len(b) and len(a) > 20
        assert [(x[0], x[1], x[3]) for x in a] == [(x[0], x[1], x[3]) for x in b]
        assert max(abs(x[2] - y[2]) for x, y in zip(a, b)) <= tol
    for x, y in zip(amps[:2], amps[2:]):
        assert np.abs(x - y).max() <= (1e-12 if dtype == C128 else 1e-5)


def _run_mode(qs, n, gates, p, dtype, defer, max_amps=2 ** 30, dirty=0):
    saved = qs.tune_get("factor.defer")
    qs.tune_set("factor.defer", defer)
    try:
        st = qs.State(n, dtype, factorized=True, max_amps=max_amps)
        st.set_policy(qs.SEP_AFTER_2Q, p)
        st.record_attempts()
        if dirty:
            st.mark_dirty(dirty)
        err = None
        try:
            st.run(qs.Circuit(n).add_gates(gates))
        except qs.CapacityError as e:
            err = e
        out = (st.attempts(), st.fidelity_estimate(), sorted(sorted(s) for s in st.subsystems()),
               st.amplitudes(), err is not None)
        st.free()
        return out
    finally:
        qs.tune_set("factor.defer", saved)


@pytest.mark.parametrize("dtype", [C64, C128])
def test_deferred_tests_keep_the_sequence(qs_lib, dtype):
    """Tests that wait until a gate touches their subsystem (and then share one
    launch with the tests pending elsewhere) give the attempt log of testing
    right after every gate: same qubits, sizes, eps (the same sums) and
    decisions in the same order, the same F and the same subsystems."""
    qs = qs_lib
    n = 16
    cases = [(workloads.grid_circuit(4, 4, 8, 3), 0.3), (workloads.random_circuit(n, 8, 12), 0.2),
             (workloads.random_circuit(n, 6, 5), 0.05)]
    for gates, p in cases:
        a = _run_mode(qs, n, gates, p, dtype, 0)
        b = _run_mode(qs, n, gates, p, dtype, 1)
        assert len(a[0]) > 20 and a[0] == b[0]
        assert a[1] == b[1] and a[2] == b[2]
        assert np.abs(a[3] - b[3]).max() <= (1e-12 if dtype == C128 else 1e-6)
        ost = replay(n, gates, p, b[0], eps_tol=2e-5 if dtype == C64 else 1e-10)
        assert abs(b[1] - ost.F) <= 1e-5 * max(ost.F, 1e-3) + 1e-7


def test_deferred_tests_capacity_and_leftover_dirty(qs_lib):
    """A merge refused for capacity in the middle of a run, and a run that
    starts with dirty qubits left from before (which turns deferral off for
    that run): the same log, F and subsystems as testing at once."""
    qs = qs_lib
    n = 12
    gates = workloads.random_circuit(n, 8, 31)
    a = _run_mode(qs, n, gates, 0.02, C64, 0, max_amps=2 ** 6)
    b = _run_mode(qs, n, gates, 0.02, C64, 1, max_amps=2 ** 6)
    assert a[4] and b[4], "the cap should be reached"
    assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2]
    assert np.abs(a[3] - b[3]).max() <= 1e-6
    pre = [("h", q) for q in range(n)] + [("cz", 0, 1), ("cz", 2, 3)]
    for defer in (0, 1):
        a = _run_mode(qs, n, pre + gates, 0.3, C64, 0, dirty=(1 << n) - 1)
        b = _run_mode(qs, n, pre + gates, 0.3, C64, defer, dirty=(1 << n) - 1)
        assert a[0] == b[0] and a[1] == b[1] and a[2] == b[2]


@pytest.mark.parametrize("dtype", [C64, C128])
def test_large_subsystem_paths(qs_lib, dtype):
    """Subsystems past the one-workgroup bounds: merges with their gate over a
    grid (17 and 18 qubits), and one-qubit runs on a 17-qubit subsystem as tile
    passes or one sweep per gate; both ways match the dense oracle."""
    qs = qs_lib
    n = 18
    g = np.random.default_rng(33)
    layer = lambda: [("u3", q, *g.uniform(0, 2 * math.pi, 3)) for q in range(n)]
    gates = [("h", q) for q in range(n)] + [("cz", q, q + 1) for q in range(16)]
    gates += layer() + layer() + layer() + [("cz", 16, 17)] + layer() + [("iswap", 3, 11)] + layer()
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    saved = qs.tune_get("factor.tile_1q")
    try:
        for tile in (1, 0):
            qs.tune_set("factor.tile_1q", tile)
            st = gpu_run(qs, n, gates, 0.0, dtype)
            assert sorted(len(s) for s in st.subsystems()) == [18]
            assert_parity(st.amplitudes(), want, dtype, f"tile_1q={tile}")
            st.free()
    finally:
        qs.tune_set("factor.tile_1q", saved)


@pytest.mark.parametrize("dtype", [C64, C128])
def test_tables_in_kernel_arguments_or_host_memory(qs_lib, dtype):
    """Small operation tables (batched sweeps, merges, projections, one-qubit
    runs) travel in the kernel arguments or are read from mapped host memory:
    the same kernels' arithmetic either way, so identical logs and kets."""
    qs = qs_lib
    n = 16
    gates = workloads.grid_circuit(4, 4, 8, 5)
    saved = qs.tune_get("factor.kernarg_tables")
    out = []
    try:
        for k in (0, 1):
            qs.tune_set("factor.kernarg_tables", k)
            st = gpu_run(qs, n, gates, 0.3, dtype)
            out.append((st.attempts(), st.fidelity_estimate(), st.amplitudes()))
            st.free()
    finally:
        qs.tune_set("factor.kernarg_tables", saved)
    assert len(out[0][0]) > 20 and out[0][0] == out[1][0] and out[0][1] == out[1][1]
    np.testing.assert_array_equal(out[0][2], out[1][2])


def test_completion_flag_or_stream_sync(qs_lib):
    """Batched sweeps waited for by their completion flag or by a stream
    synchronization: the same results (the flag is set only after every sum
    is visible), over many rounds in a row."""
    qs = qs_lib
    n = 16
    saved = qs.tune_get("factor.done_flag")
    out = []
    try:
        for k in (0, 1):
            qs.tune_set("factor.done_flag", k)
            rows = []
            for seed in range(3):
                st = gpu_run(qs, n, workloads.random_circuit(n, 8, 60 + seed), 0.3)
                rows.append((st.attempts(), st.fidelity_estimate(), st.amplitudes()))
                st.free()
            out.append(rows)
    finally:
        qs.tune_set("factor.done_flag", saved)
    for a, b in zip(*out):
        assert len(a[0]) > 20 and a[0] == b[0] and a[1] == b[1]
        np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("dtype", [C64, C128])
def test_operations_fused_with_their_sweeps(qs_lib, dtype):
    """Queued merges and projections run in the launch of the sweeps that
    read their results, or in a launch of their own: identical logs and kets
    (the same device functions in the same order per subsystem)."""
    qs = qs_lib
    n = 16
    saved = qs.tune_get("factor.fuse_ops")
    out = []
    try:
        for k in (0, 1):
            qs.tune_set("factor.fuse_ops", k)
            rows = []
            for gates, p in ((workloads.grid_circuit(4, 4, 8, 6), 0.3),
                             (workloads.random_circuit(n, 8, 77), 0.2)):
                st = gpu_run(qs, n, gates, p, dtype)
                rows.append((st.attempts(), st.fidelity_estimate(), st.amplitudes()))
                st.free()
            out.append(rows)
    finally:
        qs.tune_set("factor.fuse_ops", saved)
    for a, b in zip(*out):
        assert len(a[0]) > 20 and a[0] == b[0] and a[1] == b[1]
        np.testing.assert_array_equal(a[2], b[2])


@pytest.mark.parametrize("dtype", [C64, C128])
def test_execution_switches_do_not_change_results(qs_lib, dtype):
    """The execution switches of the factorized mode that reuse the same
    kernels' arithmetic (deferral, fused operations, kernel-argument tables,
    flag waits) all off, each on by itself, and all on, on a circuit with
    controlled gates on basis-state qubits (the shortcut) under the pair
    policy: the same attempt log, F and ket every time. Batched one-qubit runs
    change the arithmetic on subsystems past 2^12 amplitudes (tile passes):
    the same decisions, eps to rounding."""
    qs = qs_lib
    n = 14
    g = np.random.default_rng(5)
    gates = [("u3", q, math.pi, 0.0, math.pi) for q in range(0, n, 3)]   # some |1> qubits
    for _ in range(20):  # on basis states, then on what they leave
        a, b = (int(v) for v in g.choice(n, 2, replace=False))
        gates.append(("ctrl", [a], int(g.integers(0, 2)), b, *g.uniform(0, 2 * math.pi, 3)))
    gates += workloads.pair_chain_circuit(n, 3, 11)
    gates += workloads.random_circuit(n, 3, 13)
    exact_keys = ("factor.defer", "factor.fuse_ops", "factor.kernarg_tables", "factor.done_flag")
    keys = exact_keys + ("factor.batch_1q",)
    saved = {k: qs.tune_get(k) for k in keys}
    on = dict.fromkeys(keys, 1)
    off = dict(dict.fromkeys(exact_keys, 0), **{"factor.batch_1q": 1})
    settings = [off] + [dict(off, **{k: 1}) for k in exact_keys] + [on,
                                                                     dict(on, **{"factor.batch_1q": 0})]
    runs = []
    try:
        for cfg in settings:
            for k, v in cfg.items():
                qs.tune_set(k, v)
            st = qs.State(n, dtype, factorized=True)
            st.set_policy(qs.SEP_AFTER_2Q_PAIRS, 0.15)
            st.record_attempts()
            st.run(qs.Circuit(n).add_gates(gates))
            runs.append((st.attempts(), st.fidelity_estimate(), st.amplitudes(),
                         st.shortcut_count()))
            st.free()
    finally:
        for k, v in saved.items():
            qs.tune_set(k, v)
    base = runs[0]
    assert len(base[0]) > 20 and base[3] > 0
    for r in runs[1:-1]:
        assert r[0] == base[0] and r[1] == base[1] and r[3] == base[3]
        np.testing.assert_array_equal(r[2], base[2])
    last = runs[-1]  # batched one-qubit runs off
    assert [x[:2] + x[3:] for x in last[0]] == [x[:2] + x[3:] for x in base[0]]
    assert max(abs(x[2] - y[2]) for x, y in zip(last[0], base[0])) <= (1e-10 if dtype == C128 else 1e-5)
    assert abs(last[1] - base[1]) <= 1e-6 * base[1]
    np.testing.assert_allclose(last[2], base[2], rtol=0, atol=1e-10 if dtype == C128 else 2e-6)
