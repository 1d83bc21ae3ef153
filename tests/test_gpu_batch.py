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
    b = qs.Batch(widths, dtype)
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


def test_batch_1024_circuits(qs_lib):
    """1024 random circuits of 12-20 qubits, depth 8, in one batched run."""
    qs = qs_lib
    widths = workloads.batch_widths(1024, 300)
    gl, circs = circuits_for(qs, widths, 8, 300)
    b = qs.Batch(widths, C64)
    b.run(circs)
    b.synchronize()
    assert b.info()["launches"] <= 8 * 5 * 10
    small = [i for i, n in enumerate(widths) if n <= 13][:3]
    for i in small:
        n = widths[i]
        want = dense.run_circuit(dense.zero_state(n), n, gl[i])
        assert_parity(b.amplitudes(i), want, C64, f"ket {i}")
    for i in range(0, 1024, 97):
        a = b.amplitudes(i).astype(np.complex128)
        assert abs(np.vdot(a, a).real - 1) < 1e-4
    b.free()
