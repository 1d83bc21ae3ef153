"""Batched runs of many small circuits (one launch per block width per pass),
and their HIP-graph capture."""
import numpy as np
import pytest

import workloads
from oracle import dense
from parity import C64, C128, assert_parity

pytestmark = pytest.mark.gpu


def circuits_for(qs, widths, depth, seed):
    gl = [workloads.random_circuit(n, depth, seed * 1000 + i) for i, n in enumerate(widths)]
    return gl, [qs.Circuit(n).add_gates(g) for n, g in zip(widths, gl)]


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("kmax", [2, 4, 5])
def test_batch_matches_oracle(qs_lib, dtype, kmax):
    qs = qs_lib
    widths = workloads.batch_widths(12, 7, low=6, high=12)
    gl, circs = circuits_for(qs, widths, 4, kmax)
    b = qs.Batch(widths, dtype).use_tiles(False)  # blocks of at most kmax for every ket
    b.run(circs, kmax)
    for i, (n, g) in enumerate(zip(widths, gl)):
        want = dense.run_circuit(dense.zero_state(n), n, g)
        assert_parity(b.amplitudes(i), want, dtype, f"ket {i} n={n}")
    # launches scale with depth, not with the number of kets
    assert b.info()["launches"] < sum(c.info()["blocks"] for c in circs)
    b.free()


def test_batch_graph_replays(qs_lib):
    import torch
    qs = qs_lib
    widths = workloads.batch_widths(20, 3, low=8, high=13)
    gl, circs = circuits_for(qs, widths, 5, 3)
    side = torch.cuda.Stream()
    eager = qs.Batch(widths, C64, stream=side)
    eager.run(circs)
    eager.synchronize()
    want = [eager.amplitudes(i) for i in range(len(widths))]
    g = qs.Batch(widths, C64, stream=side)
    g.capture(circs)
    for rep in range(3):
        g.reset()
        g.replay()
        g.synchronize()
        # eager work between replays
        x = torch.ones(1 << 20, device="cuda").sum().item()
        assert x == float(1 << 20)
        for i in range(len(widths)):
            np.testing.assert_array_equal(g.amplitudes(i), want[i])
    for i, (n, gg) in enumerate(zip(widths, gl)):
        assert_parity(want[i], dense.run_circuit(dense.zero_state(n), n, gg), C64, f"ket {i}")
    eager.free()
    g.free()


@pytest.fixture(scope="module")
def batch1024_oracle():
    """The 1024-circuit batch (12-20 qubits, depth 8, seed 300) and the
    oracle's kets of 64 of its circuits: the first 7 of every width from 12 to
    20 and the last circuit."""
    widths = workloads.batch_widths(1024, 300)
    gl = [workloads.random_circuit(n, 8, 300 * 1000 + i) for i, n in enumerate(widths)]
    pick = []
    for w in range(12, 21):
        pick += [i for i, n in enumerate(widths) if n == w][:7]
    pick.append(1023)
    assert len(set(pick)) == 64 and {widths[i] for i in pick} == set(range(12, 21))
    want = {i: dense.run_circuit(dense.zero_state(widths[i]), widths[i], gl[i]) for i in pick}
    return widths, want


def check_batch1024(b, widths, want):
    for i, w in want.items():
        assert_parity(b.amplitudes(i), w, C64, f"ket {i} n={widths[i]}")
    for i in range(0, 1024, 61):
        a = b.amplitudes(i).astype(np.complex128)
        assert abs(np.vdot(a, a).real - 1) < 1e-4


def test_batch_1024_circuits(qs_lib, batch1024_oracle):
    """1024 random circuits of 12-20 qubits, depth 8, in one batched run with
    the default settings (tile passes for these kets: a few launches per pass
    index); 64 kets (every width) in full against the oracle, others
    normalized."""
    qs = qs_lib
    widths, want = batch1024_oracle
    gl, circs = circuits_for(qs, widths, 8, 300)
    b = qs.Batch(widths, C64)
    b.run(circs)
    b.synchronize()
    assert b.info()["launches"] <= 20
    check_batch1024(b, widths, want)
    b.free()


def test_batch_tiles_match_oracle_and_blocks(qs_lib):
    """Tile passes for the kets of >= 12 qubits, block launches for the
    smaller ones, in one arena: every ket against the oracle; a complex128
    batch with tiles on keeps its block launches."""
    qs = qs_lib
    widths = [6, 12, 13, 9, 14, 12, 15, 11, 16]
    gl, circs = circuits_for(qs, widths, 5, 61)
    b = qs.Batch(widths, C64).use_tiles()
    b.run(circs)
    tiled = b.info()["launches"]
    for i, (n, g) in enumerate(zip(widths, gl)):
        assert_parity(b.amplitudes(i), dense.run_circuit(dense.zero_state(n), n, g), C64,
                      f"ket {i} n={n}")
    b.use_tiles(False)
    b.reset()
    b.run(circs)
    assert tiled < b.info()["launches"]
    b.free()
    b2 = qs.Batch(widths, C128).use_tiles()
    b2.run(circs)
    for i, (n, g) in enumerate(zip(widths, gl)):
        assert_parity(b2.amplitudes(i), dense.run_circuit(dense.zero_state(n), n, g), C128,
                      f"c128 ket {i}")
    b2.free()


def test_batch_tiles_graph_replays(qs_lib):
    import torch
    qs = qs_lib
    widths = workloads.batch_widths(24, 5, low=12, high=16)
    gl, circs = circuits_for(qs, widths, 6, 9)
    side = torch.cuda.Stream()
    b = qs.Batch(widths, C64, stream=side).use_tiles()
    b.capture(circs)
    want = [dense.run_circuit(dense.zero_state(n), n, g) for n, g in zip(widths, gl)]
    first = None
    for rep in range(3):
        b.reset()
        b.replay()
        b.synchronize()
        x = torch.ones(1 << 20, device="cuda").sum().item()
        assert x == float(1 << 20)
        got = [b.amplitudes(i) for i in range(len(widths))]
        if first is None:
            first = got
            for i, n in enumerate(widths):
                assert_parity(got[i], want[i], C64, f"ket {i} n={n}")
        else:
            for a, c in zip(first, got):
                np.testing.assert_array_equal(a, c)
    b.free()


def test_batch_1024_circuits_tiles(qs_lib, batch1024_oracle):
    """The 1024-circuit batch with tile passes: a few launches per pass index;
    the same 64 kets in full against the oracle."""
    qs = qs_lib
    widths, want = batch1024_oracle
    gl, circs = circuits_for(qs, widths, 8, 300)
    b = qs.Batch(widths, C64).use_tiles()
    b.run(circs)
    b.synchronize()
    assert b.info()["launches"] <= 20
    check_batch1024(b, widths, want)
    b.free()


@pytest.mark.parametrize("tiles", [False, True])
def test_batch_tables_follow_circuit_changes(qs_lib, tiles):
    """A run with the same, unchanged circuits reuses the prepared tables; a
    changed circuit, or new circuits (even at a freed circuit's address), is
    prepared again."""
    qs = qs_lib
    widths = [12, 13, 10]
    gl, circs = circuits_for(qs, widths, 3, 71)
    b = qs.Batch(widths, C64).use_tiles(tiles)
    for _ in range(2):
        b.reset()
        b.run(circs)
    for i, (n, g) in enumerate(zip(widths, gl)):
        assert_parity(b.amplitudes(i), dense.run_circuit(dense.zero_state(n), n, g), C64, "same")
    extra = [("h", 2), ("cx", 2, 7), ("u3", 9, 0.4, 0.5, 0.6)]
    circs[1].add_gates(extra)
    gl[1] = gl[1] + extra
    b.reset()
    b.run(circs)
    for i, (n, g) in enumerate(zip(widths, gl)):
        assert_parity(b.amplitudes(i), dense.run_circuit(dense.zero_state(n), n, g), C64,
                      "changed")
    for c in circs:
        c.free()
    gl2, circs2 = circuits_for(qs, widths, 3, 72)
    b.reset()
    b.run(circs2)
    for i, (n, g) in enumerate(zip(widths, gl2)):
        assert_parity(b.amplitudes(i), dense.run_circuit(dense.zero_state(n), n, g), C64, "new")
    b.free()
