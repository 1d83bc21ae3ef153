"""Parity of the dense HIP path (per-gate kernels, QFT passes, readout) with
the FP64 oracle, through the C ABI."""
import math

import numpy as np
import pytest

import workloads
from oracle import dense
from parity import C64, C128, assert_parity

pytestmark = pytest.mark.gpu
DTYPES = [C64, C128]


def haar(d, seed):
    g = np.random.default_rng(seed)
    z = (g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


def fresh(qs, n, dtype, amps=None):
    st = qs.State(n, dtype)
    if amps is not None:
        st.set_amplitudes(amps)
    return st


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 7, 13])
def test_1q_every_qubit(qs_lib, dtype, n):
    qs = qs_lib
    a = workloads.gaussian_state(n, n)
    with fresh(qs, n, dtype, a) as st:
        want = a
        for q in range(n):
            m = haar(2, 100 * n + q)
            st.apply_1q(q, m)
            want = dense.apply_1q(want, n, q, m)
        assert_parity(st.amplitudes(), want, dtype, f"1q n={n}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_controlled_and_anticontrolled(qs_lib, dtype):
    qs = qs_lib
    n = 12
    g = np.random.default_rng(5)
    a = workloads.gaussian_state(n, 5)
    with fresh(qs, n, dtype, a) as st:
        want = a
        for it in range(24):
            nc = int(g.integers(1, 5))
            qq = [int(v) for v in g.choice(n, nc + 1, replace=False)]
            if it < 2:  # bit 0 as a control, then as the target
                qq = [v for v in qq if v != 0][:nc]
                qq = ([0] + qq[:nc - 1] + [qq[-1]]) if it == 0 else (qq[:nc] + [0])
                qq = qq[:nc + 1]
            ctrls, t = qq[:nc], qq[nc]
            cv = int(g.integers(0, 2 ** nc))
            m = haar(2, it)
            st.apply_ctrl(ctrls, cv, t, m)
            want = dense.apply_ctrl(want, n, ctrls, cv, t, m)
        assert_parity(st.amplitudes(), want, dtype, "ctrl")


@pytest.mark.parametrize("dtype", DTYPES)
def test_cphase_and_swap_relabel(qs_lib, dtype):
    qs = qs_lib
    n = 11
    a = workloads.gaussian_state(n, 6)
    pairs = [(0, 1), (1, 0), (0, 10), (5, 3), (10, 9), (2, 7)]
    with fresh(qs, n, dtype, a) as st:
        want = a
        for k, (x, y) in enumerate(pairs):
            st.apply_cphase(x, y, 0.3 + k)
            want = dense.apply_cphase(want, n, x, y, 0.3 + k)
            st.apply_swap(x, (y + 3) % n) if x != (y + 3) % n else None
            if x != (y + 3) % n:
                want = dense.apply_swap(want, n, x, (y + 3) % n)
            st.apply_1q(y, haar(2, k))
            want = dense.apply_1q(want, n, y, haar(2, k))
        assert_parity(st.amplitudes(), want, dtype, "cphase+swap")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_fused_block(qs_lib, dtype, k):
    qs = qs_lib
    n = 12
    g = np.random.default_rng(k)
    a = workloads.gaussian_state(n, 40 + k)
    with fresh(qs, n, dtype, a) as st:
        want = a
        for it in range(3):
            qubits = [int(v) for v in g.choice(n, k, replace=False)]
            if it == 0:
                qubits = list(range(k))[::-1]  # block on the lowest bits
            m = haar(2 ** k, 10 * k + it)
            st.apply_fused(qubits, m)
            want = dense.apply_matrix(want, n, qubits, m)
        assert_parity(st.amplitudes(), want, dtype, f"fused k={k}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_random_circuit(qs_lib, dtype):
    qs = qs_lib
    n = 12
    gates = workloads.random_circuit(n, 6, 3)
    with fresh(qs, n, dtype) as st:
        qs.run_gates(st, gates)
        want = dense.run_circuit(dense.zero_state(n), n, gates)
        assert_parity(st.amplitudes(), want, dtype, "random circuit")


@pytest.mark.parametrize("dtype", DTYPES)
def test_gate_soup(qs_lib, dtype):
    qs = qs_lib
    n = 10
    gates = workloads.random_gate_soup(n, 200, 8)
    a = workloads.gaussian_state(n, 8)
    with fresh(qs, n, dtype, a) as st:
        qs.run_gates(st, gates)
        assert_parity(st.amplitudes(), dense.run_circuit(a, n, gates), dtype, "soup")


# ------------------------------------------------------------------ QFT

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 12, 13, 16, 17])
def test_qft_gaussian(qs_lib, dtype, n):
    qs = qs_lib
    a = workloads.gaussian_state(n, 1000 + n)
    with fresh(qs, n, dtype, a) as st:
        st.qft()
        assert_parity(st.amplitudes(), dense.qft(a, n), dtype, f"qft n={n}")


@pytest.mark.parametrize("dtype", DTYPES)
def test_qft_basis_and_haar_product(qs_lib, dtype):
    """The small-case workload: QFT n=16 on |x> and on a Haar product state."""
    qs = qs_lib
    n = 16
    for seed in range(3):
        x = workloads.basis_index(n, seed)
        with fresh(qs, n, dtype) as st:
            st.set_basis(x)
            st.qft()
            assert_parity(st.amplitudes(), dense.qft(dense.basis_state(n, x), n), dtype, "basis")
        gates = workloads.haar_product_gates(n, seed)
        with fresh(qs, n, dtype) as st:
            qs.run_gates(st, gates)
            st.qft()
            want = dense.qft(dense.run_circuit(dense.zero_state(n), n, gates), n)
            assert_parity(st.amplitudes(), want, dtype, "haar product")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("start,length", [(0, 5), (3, 6), (2, 12), (12, 4), (13, 3), (5, 11), (0, 15)])
def test_partial_qft(qs_lib, dtype, start, length):
    qs = qs_lib
    n = 16
    a = workloads.gaussian_state(n, start * 31 + length)
    with fresh(qs, n, dtype, a) as st:
        st.qft(start, length)
        assert_parity(st.amplitudes(), dense.qft(a, n, start, length), dtype, "partial")


@pytest.mark.parametrize("dtype", DTYPES)
def test_qft_inverse_roundtrip_and_relabels(qs_lib, dtype):
    qs = qs_lib
    n = 14
    a = workloads.gaussian_state(n, 77)
    with fresh(qs, n, dtype, a) as st:
        st.qft()
        st.qft(inverse=True)
        assert_parity(st.amplitudes(), a, dtype, "qft then inverse")
        st.qft(inverse=True)
        assert_parity(st.amplitudes(), dense.qft(a, n, inverse=True), dtype, "inverse")
        # a QFT after SWAP relabels must see the swapped qubits
        st.set_amplitudes(a)
        st.apply_swap(0, 13)
        st.apply_swap(4, 6)
        st.qft(2, 9)
        want = dense.apply_swap(dense.apply_swap(a, n, 0, 13), n, 4, 6)
        assert_parity(st.amplitudes(), dense.qft(want, n, 2, 9), dtype, "qft after swaps")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,start,length", [(15, 0, 15), (16, 2, 9), (16, 9, 7), (14, 5, 4)])
def test_back_to_back_qft(qs_lib, dtype, n, start, length):
    """Consecutive transforms alternate between natural and bit-reversed
    storage of the range; both pass schedules must match the oracle."""
    qs = qs_lib
    a = workloads.gaussian_state(n, 3 * n + start)
    with fresh(qs, n, dtype, a) as st:
        want = a
        for k, inv in enumerate([False, False, True, False, True, True]):
            st.qft(start, length, inverse=inv)
            want = dense.qft(want, n, start, length, inverse=inv)
            assert_parity(st.amplitudes(), want, dtype, f"step {k}")
        # four forward transforms are the identity
        st.set_amplitudes(a)
        for _ in range(4):
            st.qft(start, length)
        assert_parity(st.amplitudes(), a, dtype, "QFT^4")


@pytest.mark.parametrize("dtype", DTYPES)
def test_qft_ghz_and_zero(qs_lib, dtype):
    qs = qs_lib
    n = 18
    N = 2 ** n
    j = np.arange(N)
    with fresh(qs, n, dtype, dense.ghz_state(n)) as st:
        st.qft()
        want = (1.0 + np.exp(-2j * math.pi * j / N)) / math.sqrt(2 * N)
        assert_parity(st.amplitudes(), want, dtype, "ghz")
    with fresh(qs, n, dtype) as st:
        st.qft()
        assert_parity(st.amplitudes(), np.full(N, N ** -0.5), dtype, "zero")


# ------------------------------------------------------------------ readout

@pytest.mark.parametrize("dtype", DTYPES)
def test_norm_probs_gather(qs_lib, dtype):
    qs = qs_lib
    n = 15
    a = workloads.gaussian_state(n, 9) * 1.5
    with fresh(qs, n, dtype, a) as st:
        st.apply_swap(1, 14)
        want = dense.apply_swap(a, n, 1, 14)
        tol = 1e-6 if dtype == C64 else 1e-12
        assert abs(st.norm() - dense.norm2(want)) < tol * 2.25
        idx = np.random.default_rng(0).integers(0, 2 ** n, 500)
        np.testing.assert_allclose(st.gather(idx), want[idx], atol=1e-6 if dtype == C64 else 1e-14)
        np.testing.assert_allclose(st.probs(), dense.probs(want), atol=1e-7 if dtype == C64 else 1e-15)
        # norm is repeatable bit for bit
        assert st.norm() == st.norm()


def test_error_codes(qs_lib):
    qs = qs_lib
    with fresh(qs, 6, C64) as st:
        for bad in (lambda: st.apply_1q(6, np.eye(2)),
                    lambda: st.apply_1q(-1, np.eye(2)),
                    lambda: st.apply_ctrl([2, 2], 3, 1, np.eye(2)),
                    lambda: st.apply_ctrl([1], 1, 1, np.eye(2)),
                    lambda: st.apply_fused([0, 1, 1], np.eye(8)),
                    lambda: st.apply_1q(0, np.array([[np.nan, 0], [0, 1]])),
                    lambda: st.qft(3, 4),
                    lambda: st.set_basis(64)):
            with pytest.raises(qs.QSError) as e:
                bad()
            assert e.value.code == qs.E_INVAL
        # state still usable and unchanged by the rejected calls
        assert abs(st.norm() - 1.0) < 1e-7
        st.check(1e-6)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("high_pass,lds_bits", [(0, 0), (1, 13), (0, 9), (1, 10), (0, 12), (0, 7),
                                               (0, 13)])
def test_qft_pass_variants(qs_lib, dtype, high_pass, lds_bits):
    """Every planner variant (LDS tile size, strided-LDS or register passes
    above it) in both storage orientations."""
    qs = qs_lib
    n = 17
    a = workloads.gaussian_state(n, 555)
    saved = {k: qs.tune_get(k) for k in ("qft.high_pass", "qft.lds_bits")}
    qs.tune_set("qft.high_pass", high_pass)
    qs.tune_set("qft.lds_bits", lds_bits)
    try:
        with fresh(qs, n, dtype, a) as st:
            want = a
            for inv in (False, True, False):
                st.qft(inverse=inv)
                want = dense.qft(want, n, inverse=inv)
                assert_parity(st.amplitudes(), want, dtype, f"hp={high_pass} T={lds_bits}")
            st.qft(3, 11)
            want = dense.qft(want, n, 3, 11)
            assert_parity(st.amplitudes(), want, dtype, "partial")
    finally:
        for k, v in saved.items():
            qs.tune_set(k, v)



@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,lds_bits,col_rows", [(19, 11, 0), (20, 12, 1), (22, 11, 1), (20, 12, 2),
                                                 (21, 13, 1)])
def test_qft_eight_bit_strided_passes(qs_lib, dtype, n, lds_bits, col_rows):
    """Strided passes of 8 row bits (256-byte rows) above a smaller contiguous
    tile: sampled outputs against the oracle's DFT entries (Eq. dft), then
    QFT^2 = index negation (natural and bit-reversed storage) and the
    inverse transforms back to the input."""
    qs = qs_lib
    a = workloads.gaussian_state(n, 900 + n)
    N = 2 ** n
    js = np.random.default_rng(n).integers(0, N, 48)
    saved = {k: qs.tune_get(k) for k in ("qft.col_max", "qft.lds_bits", "qft.col_rows")}
    qs.tune_set("qft.col_max", 8)
    qs.tune_set("qft.lds_bits", lds_bits)
    qs.tune_set("qft.col_rows", col_rows)
    try:
        with fresh(qs, n, dtype, a) as st:
            st.qft()
            assert_parity(st.gather(js.astype(np.uint64)), dense.dft_entries(a, n, js), dtype,
                          f"col8 n={n} T={lds_bits}")
            st.qft()
            assert_parity(st.amplitudes(), a[(-np.arange(N)) % N], dtype, "QFT^2")
            st.qft(inverse=True)
            st.qft(inverse=True)
            assert_parity(st.amplitudes(), a, dtype, "roundtrip")
    finally:
        for k, v in saved.items():
            qs.tune_set(k, v)



@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("n,lds_bits", [(17, 0), (19, 11), (20, 12), (21, 13), (22, 10)])
def test_qft_streaming_accesses(qs_lib, dtype, n, lds_bits):
    """qft.stream = 1: the LDS tile passes with non-temporal loads and stores
    (by default only for states above 256 MiB) against the oracle, forward in
    both storage orientations and the inverse; every result bit for bit equal
    to the plain accesses' (qft.stream = 2)."""
    qs = qs_lib
    a = workloads.gaussian_state(n, 1700 + n)
    saved = {k: qs.tune_get(k) for k in ("qft.stream", "qft.lds_bits")}
    qs.tune_set("qft.lds_bits", lds_bits)
    try:
        runs = {}
        for stream in (1, 2):
            qs.tune_set("qft.stream", stream)
            with fresh(qs, n, dtype, a) as st:
                out = []
                for inv in (False, False, True, True):
                    st.qft(inverse=inv)
                    out.append(st.amplitudes(np.complex64 if dtype == C64 else np.complex128))
            runs[stream] = out
        for k in range(4):
            assert np.array_equal(runs[1][k], runs[2][k]), f"step {k}"
        want = dense.qft(a, n)
        assert_parity(runs[1][0], want, dtype, f"stream n={n} T={lds_bits}")
        assert_parity(runs[1][1], dense.qft(want, n), dtype, "second transform")
        assert_parity(runs[1][3], a, dtype, "roundtrip")
    finally:
        for k, v in saved.items():
            qs.tune_set(k, v)


@pytest.mark.parametrize("dtype", DTYPES)
def test_sweeps_streaming_accesses(qs_lib, dtype):
    """sweep.stream = 1: gate sweeps, fused blocks of 1 to 6 qubits (vector and
    matrix-core forms), planned circuits of fused blocks and tile passes with
    non-temporal loads and stores (by default only for states above 256 MiB),
    each bit for bit equal to the plain accesses' result (sweep.stream = 2)
    and against the oracle."""
    qs = qs_lib
    n = 14
    a = workloads.gaussian_state(n, 1900)
    soup = workloads.random_gate_soup(n, 300, 9)
    circ = workloads.random_circuit(n, 6, 5)
    g = np.random.default_rng(77)
    blocks = [([int(v) for v in g.choice(n, k, replace=False)], haar(2 ** k, 60 + k))
              for k in range(1, 7)] + [([3, 2, 1, 0], haar(16, 70))]
    saved = qs.tune_get("sweep.stream")
    try:
        out = {}
        for stream in (1, 2):
            qs.tune_set("sweep.stream", stream)
            res = []
            with fresh(qs, n, dtype, a) as st:
                qs.run_gates(st, soup)
                res.append(st.amplitudes())
                for qubits, m in blocks:
                    st.apply_fused(qubits, m)
                res.append(st.amplitudes())
            for mode in ("blocks3", "blocks5", "tiles"):
                c = qs.Circuit(n).add_gates(circ)
                if mode == "tiles":
                    c.use_tiles()
                else:
                    c.plan(int(mode[-1]))
                with fresh(qs, n, dtype) as st:
                    st.run(c)
                    res.append(st.amplitudes())
                c.free()
            out[stream] = res
        for k, (x, y) in enumerate(zip(out[1], out[2])):
            assert np.array_equal(x, y), f"result {k} differs between the access forms"
        want = dense.run_circuit(a, n, soup)
        assert_parity(out[1][0], want, dtype, "soup")
        for qubits, m in blocks:
            want = dense.apply_matrix(want, n, qubits, m)
        assert_parity(out[1][1], want, dtype, "fused blocks")
        want = dense.run_circuit(dense.zero_state(n), n, circ)
        for k in (2, 3, 4):
            assert_parity(out[1][k], want, dtype, f"circuit form {k}")
    finally:
        qs.tune_set("sweep.stream", saved)


@pytest.mark.parametrize("n", [7, 8, 12, 15])
def test_1q_wavefront_shuffles(qs_lib, n):
    """gate.shuffle_bits = 6: complex64 one-qubit gates on bits 1-6 with each
    lane holding contiguous amplitudes and the partners (target bit flipped)
    exchanged by cross-lane shuffles, in the plain and the streaming access
    form: bit for bit equal to the strided pairs' result, and against the
    oracle, for every target bit (7 qubits: exactly one wavefront)."""
    qs = qs_lib
    a = workloads.gaussian_state(n, 2100 + n)
    g = np.random.default_rng(n)
    gates = [(t, haar(2, 80 + t)) for t in range(1, 7)] * 2
    g.shuffle(gates)
    saved = {k: qs.tune_get(k) for k in ("gate.shuffle_bits", "sweep.stream")}
    try:
        out = {}
        for shuffle, stream in ((0, 2), (6, 2), (6, 1)):
            qs.tune_set("gate.shuffle_bits", shuffle)
            qs.tune_set("sweep.stream", stream)
            with fresh(qs, n, C64, a) as st:
                for t, m in gates:
                    st.apply_1q(t, m)
                out[(shuffle, stream)] = st.amplitudes(np.complex64)
        assert np.array_equal(out[(0, 2)], out[(6, 2)]), "shuffles differ from strided pairs"
        assert np.array_equal(out[(6, 2)], out[(6, 1)]), "streaming form differs"
        want = a
        for t, m in gates:
            want = dense.apply_1q(want, n, t, m)
        assert_parity(out[(6, 1)].astype(np.complex128), want, C64, f"shuffles n={n}")
    finally:
        for k, v in saved.items():
            qs.tune_set(k, v)


@pytest.mark.parametrize("n", [7, 9, 13])
def test_ctrl_dense_low_bits(qs_lib, n):
    """gate.dense_ctrl = 1: singly controlled complex64 gates whose control is
    below bit 3 swept densely (the whole state, the matrix applied where the
    control matches; targets on bit 0, by shuffles, or strided), in both
    access forms, among gates with high controls that keep the sparse sweep:
    bit for bit equal to the sparse sweeps and against the oracle, for
    controls and anti-controls."""
    qs = qs_lib
    a = workloads.gaussian_state(n, 2300 + n)
    cases = [(0, 1, 5), (1, 1, n - 1), (2, 0, 4), (1, 0, 0), (0, 1, 3), (n - 1, 1, 1),
             (n - 2, 0, 0), (2, 1, 6), (0, 0, n - 1)]
    mats = [haar(2, 90 + k) for k in range(len(cases))]
    saved = {k: qs.tune_get(k) for k in ("gate.dense_ctrl", "sweep.stream")}
    try:
        out = {}
        for dense_on, stream in ((0, 2), (1, 2), (1, 1)):
            qs.tune_set("gate.dense_ctrl", dense_on)
            qs.tune_set("sweep.stream", stream)
            with fresh(qs, n, C64, a) as st:
                for (c, cv, t), m in zip(cases, mats):
                    st.apply_ctrl([c], cv, t, m)
                out[(dense_on, stream)] = st.amplitudes(np.complex64)
        assert np.array_equal(out[(0, 2)], out[(1, 2)]), "dense and sparse sweeps differ"
        assert np.array_equal(out[(1, 2)], out[(1, 1)]), "streaming form differs"
        want = a
        for (c, cv, t), m in zip(cases, mats):
            want = dense.apply_ctrl(want, n, [c], cv, t, m)
        assert_parity(out[(1, 1)].astype(np.complex128), want, C64, f"dense ctrl n={n}")
    finally:
        for k, v in saved.items():
            qs.tune_set(k, v)
