"""Tile passes (several gates per HBM sweep) against the FP64 oracle."""
import numpy as np
import pytest

import workloads
from oracle import dense
from parity import C64, C128, assert_parity

pytestmark = pytest.mark.gpu


@pytest.fixture(params=[(1, 6), (1, 5), (0, 6), (0, 5)],
                ids=["mfma-rows64", "mfma-rows32", "registers-rows64", "registers-rows32"])
def tile_mode(request, qs_lib):
    """Complex64 passes with dense rounds on the matrix cores or one- and
    two-qubit gates in registers, on tiles with 64- or 32-amplitude rows.
    Yields whether the matrix-core rounds are on."""
    mfma, low = request.param
    keys = ("tile.mfma", "tile.low_bits")
    saved = [qs_lib.tune_get(k) for k in keys]
    for k, v in zip(keys, (mfma, low)):
        qs_lib.tune_set(k, v)
    yield mfma
    for k, v in zip(keys, saved):
        qs_lib.tune_set(k, v)


@pytest.mark.parametrize("dtype,n", [(C64, 13), (C64, 14), (C64, 17), (C128, 12), (C128, 15)])
@pytest.mark.parametrize("family", ["matching", "grid"])
def test_tiled_random_circuits(qs_lib, tile_mode, dtype, n, family):
    qs = qs_lib
    if dtype == C128 and tile_mode == 0:
        pytest.skip("complex128 always runs register rounds")
    if family == "matching":
        gates = workloads.random_circuit(n, 8, 40 + n)
    else:
        rows = 3 if n % 3 == 0 else 1  # 3 x 4, 3 x 5, or one row
        gates = workloads.grid_circuit(rows, n // rows, 8, 40 + n)
    c = qs.Circuit(n).add_gates(gates).use_tiles()
    with qs.State(n, dtype) as st:
        st.profile_start()
        st.run(c)
        prof = st.profile_stop()
        name = "tile_mfma" if (dtype == C64 and tile_mode) else "tile_pass"
        assert name in prof
        if dtype == C128 or tile_mode:
            assert prof[name]["launches"] == c.tile_info(dtype)["passes"]
        assert_parity(st.amplitudes(), dense.run_circuit(dense.zero_state(n), n, gates), dtype,
                      f"tiles n={n}")
    c.free()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_tiles_with_swaps_blocks_and_relabels(qs_lib, tile_mode, dtype):
    """SWAP renaming, gates on three qubits (dense blocks between passes),
    controlled gates, and a state whose labelling is not the identity (after a
    QFT, whose bit reversal is a relabelling; the plan is made on physical
    bits and remade when the labelling changes)."""
    qs = qs_lib
    n = 15
    g3 = dense.u3(0.3, 0.5, 0.7)
    m3 = np.kron(np.kron(dense.H, g3), dense.u3(1.1, 0.2, 0.4))
    m4 = np.kron(m3, dense.u3(0.9, 0.1, 0.6)) @ np.diag(np.exp(1j * np.arange(16) * 0.3))
    m5 = np.kron(m4, g3)
    gates = (workloads.random_circuit(n, 3, 5) + [("swap", 0, 14), ("swap", 3, 9)]
             + workloads.random_circuit(n, 2, 6) + [("mat", [1, 8, 13], m3), ("cx", 12, 2),
                                                     ("ay", 4, 11), ("cp", 5, 10, 0.77),
                                                     ("mat", [14, 0, 9, 6], m4),
                                                     ("mat", [3, 12, 7, 1, 10], m5)]
             + workloads.grid_circuit(3, 5, 2, 7))
    c = qs.Circuit(n).add_gates(gates).use_tiles()
    a = workloads.gaussian_state(n, 12)
    with qs.State(n, dtype) as st:
        st.set_amplitudes(a)
        st.run(c)
        want = dense.run_circuit(a, n, gates)
        assert_parity(st.amplitudes(), want, dtype, "identity labelling")
        st.qft()  # leaves the state bit-reversed
        want = dense.qft(want, n)
        st.run(c)
        want = dense.run_circuit(want, n, gates)
        assert_parity(st.amplitudes(), want, dtype, "after a relabelling")
        st.run(c)  # labelling changed again by the circuit's swaps
        want = dense.run_circuit(want, n, gates)
        assert_parity(st.amplitudes(), want, dtype, "third run")
    c.free()


def test_tiles_agree_with_blocks_at_28(qs_lib, tile_mode):
    """A 28-qubit circuit (2 GiB): tile passes and fused blocks give the same
    ket to float32 rounding."""
    qs = qs_lib
    n = 28
    gates = workloads.random_circuit(n, 10, 3)
    ct = qs.Circuit(n).add_gates(gates).use_tiles()
    cb = qs.Circuit(n).add_gates(gates).plan(4)
    with qs.State(n, C64) as a, qs.State(n, C64) as b:
        a.run(ct)
        b.run(cb)
        idx = np.random.default_rng(3).integers(0, 2 ** n, 20000).astype(np.uint64)
        ga, gb = a.gather(idx), b.gather(idx)
        assert np.abs(ga - gb).max() <= 1e-6
        assert abs(a.norm() - 1.0) < 1e-5
        assert abs(abs(a.inner(b)) - 1.0) < 1e-5
    ct.free()
    cb.free()


@pytest.mark.parametrize("dtype,n", [(C64, 14), (C128, 12), (C64, 9)])
def test_default_run_mode(qs_lib, dtype, n):
    """A circuit run without qs_circuit_plan or qs_circuit_use_tiles takes
    tile passes when the state holds a tile (12 qubits in complex64, 11 in
    complex128), fused blocks below that; blocks planned before any choice,
    or tiles switched off, run as blocks; switching tiles on after planning
    runs tiles; the library's own block planning (a batch run of the same
    circuit first) leaves the choice open. Every form against the oracle."""
    qs = qs_lib
    gates = workloads.random_circuit(n, 4, 60 + n)
    want = dense.run_circuit(dense.zero_state(n), n, gates)
    tiles_fit = n >= (12 if dtype == C64 else 11)
    cases = [("default", lambda c: c, tiles_fit),
             ("plan", lambda c: c.plan(4), False),
             ("tiles off", lambda c: c.use_tiles(False), False),
             ("plan then tiles", lambda c: c.plan(4).use_tiles(), tiles_fit),
             ("tiles then plan", lambda c: c.use_tiles().plan(4), tiles_fit),
             ("after a batch run", lambda c: batch_first(c), tiles_fit)]

    def batch_first(c):
        b = qs.Batch([n], dtype)
        b.run([c], 4)
        assert_parity(b.amplitudes(0), want, dtype, "batch")
        b.free()
        return c

    for name, setup, expect_tiles in cases:
        c = setup(qs.Circuit(n).add_gates(gates))
        with qs.State(n, dtype) as st:
            st.profile_start()
            st.run(c)
            prof = st.profile_stop()
            ran_tiles = any(k.startswith("tile_") for k in prof)
            assert ran_tiles == expect_tiles, (name, sorted(prof))
            assert_parity(st.amplitudes(), want, dtype, name)
        c.free()
