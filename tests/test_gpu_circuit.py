"""Fused random circuits on the GPU (planner + block kernels, MFMA for
complex64 blocks of 4-5 qubits) against the oracle applying each gate."""
import math

import numpy as np
import pytest

import workloads
from oracle import dense
from parity import C64, C128, assert_parity

pytestmark = pytest.mark.gpu


def haar(d, seed):
    g = np.random.default_rng(seed)
    z = (g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))) / math.sqrt(2)
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("kmax", [2, 4, 5, 6])
@pytest.mark.parametrize("n", [12, 15])
def test_random_circuit_fused(qs_lib, dtype, kmax, n):
    qs = qs_lib
    gates = workloads.random_circuit(n, 6, 100 * kmax + n)
    c = qs.Circuit(n).add_gates(gates).plan(kmax)
    with qs.State(n, dtype) as st:
        st.run(c)
        want = dense.run_circuit(dense.zero_state(n), n, gates)
        assert_parity(st.amplitudes(), want, dtype, f"n={n} kmax={kmax}")


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("mfma", [0, 1])
def test_mfma_blocks_every_position(qs_lib, mfma, dtype):
    """k = 4, 5 blocks on low, high, mixed and bit-0 positions; the matrix-core
    kernel (mfma=1: FP32 or FP64 matrix cores) and the vector-FMA kernel
    (mfma=0) both match."""
    qs = qs_lib
    n = 14
    a = workloads.gaussian_state(n, 21)
    qs.tune_set("fused.mfma", mfma)
    try:
        with qs.State(n, dtype) as st:
            st.set_amplitudes(a)
            want = a
            sets = [[0, 1, 2, 3], [13, 12, 11, 10], [3, 9, 0, 12], [1, 5, 8, 11, 13],
                    [4, 3, 2, 1, 0], [13, 6, 0, 7, 2], [7, 8, 9, 10, 11]]
            for i, qq in enumerate(sets):
                m = haar(2 ** len(qq), i)
                st.apply_fused(qq, m)
                want = dense.apply_matrix(want, n, qq, m)
            prof_want = "fused5_mfma" if mfma else "fused5"
            st.profile_start()
            st.apply_fused([2, 4, 6, 8, 10], haar(32, 99))
            want = dense.apply_matrix(want, n, [2, 4, 6, 8, 10], haar(32, 99))
            assert prof_want in st.profile_stop()
            assert_parity(st.amplitudes(), want, dtype, f"mfma={mfma}")
    finally:
        qs.tune_set("fused.mfma", 1)


@pytest.mark.parametrize("dtype", [C64, C128])
def test_mfma_blocks_random_positions(qs_lib, dtype):
    """4- and 5-qubit matrix-core blocks on 40 random qubit sets of a 13-qubit
    state, each against the oracle: where the block's bits fall decides the
    tile's LDS layout, and for complex64 5-qubit blocks with conflicting reads
    the swizzled form and its shift (4-7 among these sets)."""
    qs = qs_lib
    n = 13
    rng = np.random.default_rng(5)
    a = workloads.gaussian_state(n, 22)
    rel = 1e-5 if dtype == C64 else 1e-12
    with qs.State(n, dtype) as st:
        for i in range(40):
            k = 4 + (i % 2)
            qq = [int(x) for x in rng.choice(n, size=k, replace=False)]
            m = haar(2 ** k, 100 + i)
            st.set_amplitudes(a)
            st.profile_start()
            st.apply_fused(qq, m)
            assert f"fused{k}_mfma" in st.profile_stop(), qq
            r = assert_parity(st.amplitudes(), dense.apply_matrix(a, n, qq, m), dtype, f"block {i} on {qq}")
            assert r["max_rel"] < rel, (qq, r)



def test_swaps_in_circuit_and_relabel(qs_lib):
    qs = qs_lib
    n = 13
    gates = workloads.random_circuit(n, 3, 5)
    gates = gates[:20] + [("swap", 0, 12), ("swap", 3, 7)] + gates[20:] + [("swap", 1, 2)]
    c = qs.Circuit(n).add_gates(gates).plan(5)
    with qs.State(n, C64) as st:
        st.run(c)
        st.run(c)
        want = dense.run_circuit(dense.zero_state(n), n, gates)
        want = dense.run_circuit(want, n, gates)
        assert_parity(st.amplitudes(), want, C64, "swaps")
        # the state's labels carry the renaming: a QFT afterwards still matches
        st.qft(2, 8)
        assert_parity(st.amplitudes(), dense.qft(want, n, 2, 8), C64, "qft after circuit")


def test_paper_couplers(qs_lib):
    """The anti-controlled couplers of Sec. III-C (AX, AY, AZ) and CX, CY."""
    qs = qs_lib
    n = 12
    g = np.random.default_rng(4)
    gates = []
    for layer in range(4):
        for q in range(n):
            t, p, l = g.uniform(0, 2 * math.pi, 3)
            gates.append(("u3", q, float(t), float(p), float(l)))
        perm = g.permutation(n)
        for i in range(n // 2):
            kind = ["cx", "cy", "cz", "ax", "ay", "az"][int(g.integers(0, 6))]
            gates.append((kind, int(perm[2 * i]), int(perm[2 * i + 1])))
    ctrl = {"x": (math.pi, 0.0, math.pi), "y": (math.pi, math.pi / 2, math.pi / 2),
            "z": (0.0, 0.0, math.pi)}
    ogates = [("ctrl", (gg[1],), 0 if gg[0][0] == "a" else 1, gg[2]) + ctrl[gg[0][1]]
              if gg[0] in ("cx", "cy", "ax", "ay", "az") else gg for gg in gates]
    c = qs.Circuit(n).add_gates(gates).plan(5)
    with qs.State(n, C64) as st:
        st.run(c)
        assert_parity(st.amplitudes(), dense.run_circuit(dense.zero_state(n), n, ogates), C64,
                      "couplers")


def inverse_gates(gates):
    """Gate list of the inverse circuit (reversed, each gate inverted)."""
    out = []
    for g in reversed(gates):
        if g[0] == "u3":
            # U(t, p, l)^-1 = U(-t, -l, -p)
            out.append(("u3", g[1], -g[2], -g[4], -g[3]))
        elif g[0] == "iswap":
            qs_, m = [g[1], g[2]], dense.ISWAP.conj().T
            out.append(("mat", qs_, m))
        else:
            out.append(g)
    return out


@pytest.mark.timeout(1500)
def test_random_circuit_n26_full_vector_against_oracle(qs_lib):
    """The exact random-circuit workload (10 layers of U3 on every qubit, then
    CZ or iSWAP on a seeded random matching; the generator of the 32-qubit
    benchmark) at 26 qubits, every amplitude against the oracle run gate by
    gate (about 5 minutes on one host core; 28 qubits would take about 20):
    tile passes (the benchmark's mode), blocks of at most 4 qubits (its
    comparison) and blocks of at most 5 (matrix cores for 4-5 qubits)."""
    qs = qs_lib
    n = 26
    gates = workloads.random_circuit(n, 10, 0)
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    for mode in ("tiles", 4, 5):
        c = qs.Circuit(n).add_gates(gates)
        if mode == "tiles":
            c.use_tiles()
        else:
            c.plan(mode)
        with qs.State(n, C64) as st:
            st.run(c)
            got = st.amplitudes()
        c.free()
        r = assert_parity(got, want, C64, f"n=26 {mode}")
        print(f"n=26 {mode}: {r}")
        del got


@pytest.mark.parametrize("n", [28])
def test_large_random_circuit_then_inverse(qs_lib, n):
    """At a size the oracle cannot run whole: C followed by C^-1 returns |0...0>
    (amplitude 1 within float32 rounding) and the norm stays 1. Every block of
    both circuits runs on the fused kernels (MFMA for 4-5 qubits)."""
    qs = qs_lib
    gates = workloads.random_circuit(n, 10, 7)
    c = qs.Circuit(n).add_gates(gates).plan(5)
    ci = qs.Circuit(n).add_gates(inverse_gates(gates)).plan(5)
    with qs.State(n, C64) as st:
        st.profile_start()
        st.run(c)
        prof = st.profile_stop()
        assert "fused5_mfma" in prof and "fused4_mfma" in prof
        assert abs(st.norm() - 1.0) < 1e-5
        amp0 = st.gather([0])[0]
        assert abs(amp0) < 1e-2  # a deep random circuit spreads the weight
        st.run(ci)
        amp0 = st.gather([0])[0]
        assert abs(abs(amp0) - 1.0) < 1e-5, amp0
        assert abs(st.norm() - 1.0) < 1e-5
