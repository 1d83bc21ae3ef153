"""The gate-fusion planner is host code: check its blocks without a GPU.

Applying the planner's fused block matrices (with the oracle's generic
matrix routine) must give the same ket as the oracle applying the original
gates one at a time; block widths respect kmax."""
import math

import numpy as np
import pytest

import workloads
from oracle import dense


@pytest.fixture(scope="module")
def qs():
    import paper_2304_14969_amd as m
    m.open_library()
    return m


def apply_blocks(circ, n, a):
    nb = circ.info()["blocks"]
    for i in range(nb):
        qubits, m = circ.block(i)
        a = dense.apply_matrix(a, n, qubits, m)
    return a


@pytest.mark.parametrize("kmax", [1, 2, 3, 4, 5, 6])
def test_fused_blocks_reproduce_circuit(qs, kmax):
    n = 8
    gates = workloads.random_circuit(n, 4, kmax)
    gates += [("h", 3), ("cp", 1, 6, 0.4), ("cx", 0, 7), ("ay", 5, 2), ("az", 2, 4), ("cy", 7, 1)]
    c = qs.Circuit(n).add_gates(gates).plan(kmax)
    info = c.info()
    assert info["gates"] == len(gates)
    assert 1 <= info["max_k"] <= max(kmax, 2)
    a = workloads.gaussian_state(n, kmax)
    want = dense.run_circuit(a, n, [g if g[0] not in ("cx", "cy", "ax", "ay", "az") else
                                    _ctrl(g) for g in gates])
    np.testing.assert_allclose(apply_blocks(c, n, a), want, atol=1e-12)
    if kmax >= 2:
        assert info["blocks"] < len(gates)


def _ctrl(g):
    """two-qubit controlled couplers as oracle 'ctrl' gates (U3 form)."""
    kind, c, t = g
    cv = 0 if kind[0] == "a" else 1
    ang = {"x": (math.pi, 0.0, math.pi), "y": (math.pi, math.pi / 2, math.pi / 2),
           "z": (0.0, 0.0, math.pi)}[kind[1]]
    return ("ctrl", (c,), cv, t) + ang


def test_swaps_become_relabels(qs):
    n = 6
    gates = [("h", 0), ("cz", 0, 1), ("swap", 0, 5), ("u3", 0, 0.3, 0.2, 0.1), ("iswap", 5, 2),
             ("swap", 2, 3), ("h", 3)]
    c = qs.Circuit(n).add_gates(gates).plan(5)
    # SWAPs add no gate
    assert c.info()["gates"] == len(gates) - 2
    # the blocks act on positions; logical qubit q ends at position pos[q]
    pos = list(range(n))
    for g in gates:
        if g[0] == "swap":
            pos[g[1]], pos[g[2]] = pos[g[2]], pos[g[1]]
    a = workloads.gaussian_state(n, 1)
    got_pos = apply_blocks(c, n, a)
    x = np.arange(2 ** n)
    idx = np.zeros_like(x)
    for q in range(n):
        idx |= ((x >> q) & 1) << pos[q]
    got = got_pos[idx]
    np.testing.assert_allclose(got, dense.run_circuit(a, n, gates), atol=1e-12)


def test_planner_rejects_bad_gates(qs):
    c = qs.Circuit(4)
    for bad in (lambda: c.add("cz", [1, 1]), lambda: c.add("h", [4]),
                lambda: c.add("u3", [0], [float("nan"), 0, 0]),
                lambda: c.add_matrix([0, 1], np.eye(2))):
        with pytest.raises(Exception):
            bad()
    with pytest.raises(qs.QSError):
        c.plan(7)


def test_block_count_random_layers(qs):
    """Fusion actually groups gates: a 5-qubit-wide plan of a 20-qubit,
    10-layer random circuit needs far fewer sweeps than gates."""
    n = 20
    c = qs.Circuit(n).add_gates(workloads.random_circuit(n, 10, 0)).plan(5)
    info = c.info()
    assert info["blocks"] * 3 < info["gates"]


def test_tile_plan_counts(qs):
    """Tile-pass planning is host code too: a 10-layer random circuit on 32
    qubits needs far fewer passes than gates (each pass holds every gate that
    fits a tile of the 6 low bits plus 7 others); a gate wider than a round
    (complex64 dense rounds: 4 qubits; complex128: 2) becomes a dense block
    between passes; a state smaller than a tile has no tile plan."""
    n = 32
    c = qs.Circuit(n).add_gates(workloads.random_circuit(n, 10, 0))
    info = c.tile_info(qs.C64)
    assert info["blocks"] == 0
    assert 10 <= info["passes"] <= 60
    assert info["rounds"] >= info["passes"]
    c128 = c.tile_info(qs.C128)
    assert c128["passes"] >= info["passes"]  # register rounds take gates of <= 2 qubits
    g3 = dense.u3(0.1, 0.2, 0.3)
    m3 = np.kron(np.kron(g3, g3), dense.H)
    c3 = qs.Circuit(16).add_gates(workloads.random_circuit(16, 3, 1)
                                  + [("mat", [2, 9, 14], m3)]
                                  + workloads.random_circuit(16, 2, 2))
    assert c3.tile_info(qs.C64)["blocks"] == 0
    assert c3.tile_info(qs.C128)["blocks"] == 1
    m5 = np.kron(m3, np.kron(g3, g3))
    c5 = qs.Circuit(16).add_gates(workloads.random_circuit(16, 2, 3)
                                  + [("mat", [0, 4, 7, 11, 15], m5)])
    assert c5.tile_info(qs.C64)["blocks"] == 1
    c5.free()
    small = qs.Circuit(11).add_gates(workloads.random_circuit(11, 2, 0))
    with pytest.raises(qs.QSError):
        small.tile_info(qs.C64)  # the default tile has 5 + 7 bits
    small.free()
    for x in (c, c3):
        x.free()
