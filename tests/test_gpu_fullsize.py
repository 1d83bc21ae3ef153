"""Checks at the benchmark's full sizes, in the launch configuration bench.py
times: QFT on 27 qubits (complex64) against single outputs of the oracle's
direct definition and the basis-state closed form; the QFT on 28 to 32 qubits
(up to 32 GiB) against the closed form in both stored orientations, and at 28
against single outputs of the direct definition; the QFT on 24 qubits against
the oracle's whole vector with the benchmark's pass kinds; the 32-qubit
random circuit followed by its inverse; 54-qubit approximate runs against the
invariants that hold at any size."""
import math

import numpy as np
import pytest

import workloads
from oracle import dense
from parity import C64, C128

pytestmark = pytest.mark.gpu
N27 = 27


def sample_indices(n, count, seed):
    g = np.random.default_rng(seed)
    idx = g.integers(0, 2 ** n, count, dtype=np.int64)
    return np.concatenate([[0, 1, 2 ** n - 1, 2 ** (n - 1)], idx]).astype(np.uint64)


@pytest.mark.parametrize("high_pass", [0, 1])
def test_qft27_basis_state_closed_form(qs_lib, high_pass):
    """Strided-LDS passes above the contiguous tile (bench.py's configuration)
    and register passes."""
    qs = qs_lib
    saved = qs.tune_get("qft.high_pass")
    qs.tune_set("qft.high_pass", high_pass)
    try:
        x = workloads.basis_index(N27, 0)
        with qs.State(N27, C64) as st:
            st.set_basis(x)
            st.qft()
            idx = sample_indices(N27, 4096, 1)
            got = st.gather(idx)
            want = dense.qft_basis_entries(N27, x, idx)
            err = np.abs(got - want)
            assert err.max() <= 1e-5
            assert err.max() / np.abs(want).max() <= 1e-4, err.max()
            assert abs(st.norm() - 1.0) < 1e-5
    finally:
        qs.tune_set("qft.high_pass", saved)


def test_qft27_gaussian_spot_checks_and_roundtrip(qs_lib):
    """The benchmark's input (complex Gaussian, seed 0): a few outputs against
    the direct sum of Eq. dft, then QFT^-1 brings the input back."""
    qs = qs_lib
    a = workloads.gaussian_state(N27, 0)
    js = [0, 1, 12345, 2 ** 26 + 3, 2 ** 27 - 1]
    want = dense.dft_entries(a, N27, js)
    with qs.State(N27, C64) as st:
        st.set_amplitudes(a)
        st.qft()
        got = st.gather(np.array(js, dtype=np.uint64))
        assert np.abs(got - want).max() <= 1e-5
        assert np.abs(got - want).max() / np.abs(want).max() <= 1e-4
        st.qft(inverse=True)
        idx = sample_indices(N27, 4096, 2)
        back = st.gather(idx)
        assert np.abs(back - a[idx.astype(np.int64)]).max() <= 1e-5
        assert abs(st.norm() - 1.0) < 1e-5


def test_qft24_gaussian_full_vector(qs_lib):
    """Every output of the QFT of a 24-qubit complex Gaussian state against
    the oracle's gate-by-gate circuit (Sec. II-E), with the default pass plan
    (12-bit contiguous tile, then two 6-bit strided passes) and with a 9-bit
    tile, which leaves the benchmark's 8- and 7-bit strided passes (the same
    kernels bench.py times at 27 qubits)."""
    from parity import assert_parity
    qs = qs_lib
    n = 24
    a = workloads.gaussian_state(n, 0)
    want = dense.qft(a, n)
    saved = qs.tune_get("qft.lds_bits")
    try:
        for lds_bits in (saved, 9):
            qs.tune_set("qft.lds_bits", lds_bits)
            with qs.State(n, C64) as st:
                st.set_amplitudes(a)
                st.qft()
                got = st.amplitudes()
            r = assert_parity(got, want, C64, f"qft24 lds_bits={lds_bits}")
            assert r["max_rel"] <= 1e-4, r
    finally:
        qs.tune_set("qft.lds_bits", saved)


@pytest.mark.parametrize("n,dtype", [(28, C64), (29, C64), (30, C64), (31, C64), (32, C64),
                                     (25, C128), (26, C128), (29, C128), (30, C128)])
def test_qft_large_basis_closed_form_both_orientations(qs_lib, n, dtype):
    """QFT|x> = 2^{-n/2} e^{2 pi i x y / 2^n} at 28-32 qubits (complex64, up
    to 32 GiB) and 25-30 qubits in complex128 (the plans with 10- and 11-bit
    tiles the library takes above 256 MiB, up to 16 GiB), sampled at 4,100
    outputs. The transform leaves the range stored bit-reversed, so the
    second forward transform runs the reversed-order passes; QFT^2 |x> =
    |-x mod 2^n> exactly. The two inverse transforms then return to QFT|x>
    (natural order) and to |x>."""
    qs = qs_lib
    N = 1 << n
    x = workloads.basis_index(n, n)
    idx = sample_indices(n, 4096, n)
    want = dense.qft_basis_entries(n, x, idx)
    tol = 1e-5 if dtype == C64 else 1e-12

    def check_closed_form(st, what):
        got = st.gather(idx)
        err = np.abs(got - want)
        assert err.max() <= tol, (what, err.max())
        assert err.max() / np.abs(want).max() <= 10 * tol, (what, err.max())

    def check_basis(st, y, what):
        probe = np.concatenate([[y], idx[idx != y]]).astype(np.uint64)
        got = st.gather(probe)
        assert abs(got[0] - 1.0) <= tol, (what, got[0])
        assert np.abs(got[1:]).max() <= tol, (what, np.abs(got[1:]).max())

    with qs.State(n, dtype) as st:
        st.set_basis(x)
        st.qft()
        check_closed_form(st, "QFT|x>")
        assert abs(st.norm() - 1.0) < tol
        st.qft()
        check_basis(st, (N - x) % N, "QFT^2|x>")
        st.qft(inverse=True)
        check_closed_form(st, "QFT^-1 QFT^2|x>")
        st.qft(inverse=True)
        check_basis(st, x, "QFT^-2 QFT^2|x>")
        assert abs(st.norm() - 1.0) < tol


def test_qft28_gaussian_spot_checks_and_roundtrip(qs_lib):
    """28 qubits, complex Gaussian input: 8 outputs against the direct sum
    of Eq. dft, then QFT^-1 brings the input back (4,100 sampled entries)."""
    qs = qs_lib
    n = 28
    a = workloads.gaussian_state(n, 1)
    js = [0, 1, 2, 3, 777777, 2 ** 27 + 5, 2 ** 28 - 2, 2 ** 28 - 1]
    want = dense.dft_entries(a, n, js)
    with qs.State(n, C64) as st:
        st.set_amplitudes(a)
        st.qft()
        got = st.gather(np.array(js, dtype=np.uint64))
        assert np.abs(got - want).max() <= 1e-5
        assert np.abs(got - want).max() / np.abs(want).max() <= 1e-4
        st.qft(inverse=True)
        idx = sample_indices(n, 4096, 3)
        back = st.gather(idx)
        assert np.abs(back - a[idx.astype(np.int64)]).max() <= 1e-5
        assert abs(st.norm() - 1.0) < 1e-5


def test_random_circuit_n32_then_inverse(qs_lib):
    """32 qubits (32 GiB): C then C^-1 returns |0...0>, norm 1, both circuits
    on the fused kernels with the default block width of bench.py (4)."""
    from test_gpu_circuit import inverse_gates
    qs = qs_lib
    n = 32
    gates = workloads.random_circuit(n, 10, 0)
    c = qs.Circuit(n).add_gates(gates).plan(4)
    ci = qs.Circuit(n).add_gates(inverse_gates(gates)).plan(4)
    with qs.State(n, C64) as st:
        st.run(c)
        assert abs(st.norm() - 1.0) < 1e-5
        assert abs(st.gather([0])[0]) < 1e-2
        st.run(ci)
        amp0 = st.gather([0])[0]
        assert abs(abs(amp0) - 1.0) < 1e-5, amp0
    c.free()
    ci.free()


@pytest.mark.parametrize("family", ["grid", "matching"])
def test_approx54_invariants(qs_lib, family):
    """54 qubits x 7 layers at p = 0.6: completes under the 2^30 cap, every
    rounding obeys eps <= p/2 (+ the complex64 tolerance), the fidelity
    estimate is the product of (1 - eps) over the roundings, the norm is 1."""
    from paper_2304_14969_amd import protocol
    gates = (workloads.grid_circuit(6, 9, 7, 0) if family == "grid"
             else workloads.random_circuit(54, 7, 0))
    p = 0.6
    r = protocol.approx_run(54, gates, p, record=True, keep=True)
    st = r["state"]
    try:
        assert r["ok"] and r["max_sub"] <= 30
        F = 1.0
        for q, nsub, eps, rounded in r["log"]:
            assert 0.0 <= eps <= 0.5 and 2 <= nsub <= 30
            if rounded:
                assert eps <= p / 2 + 1e-6
                F *= 1.0 - eps
            else:
                assert eps > p / 2
        assert math.isclose(F, r["F"], rel_tol=1e-12)
        assert abs(st.norm() - 1.0) < 1e-4
        sizes = [len(s) for s in st.subsystems()]
        assert sum(sizes) == 54
    finally:
        st.free()
