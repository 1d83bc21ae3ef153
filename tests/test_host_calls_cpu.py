"""C-ABI calls that run on the host only (no GPU): the circuit objects and
their fusion and tile planners over many shapes and gate mixes, every
argument check of those calls, and every tuning knob. Run as they are here,
and again against the sanitizer build of the host code
(test_host_sanitized.py)."""
import ctypes as C
import math

import numpy as np
import pytest

import workloads


@pytest.fixture(scope="module")
def qs():
    import paper_2304_14969_amd as m
    m.open_library()
    return m


def unitary(d, seed):
    g = np.random.default_rng(seed)
    z = g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 9, 12, 13, 17, 21])
def test_planner_over_shapes(qs, n):
    """Every kmax, both tile precisions, gate mixes with swaps and dense
    matrices: the plan's blocks cover every gate and are read back whole."""
    kinds = ["h", "u3"] if n < 2 else ["h", "u3", "cp", "cz", "iswap", "swap", "ctrl"]
    gates = workloads.random_gate_soup(n, 40 + 5 * n, 7 * n, kinds)
    gates = [g for g in gates if g[0] != "ctrl" or len(g[1]) == 1]
    if n >= 3:
        gates.append(("mat", [0, n - 1, n // 2], unitary(8, n)))
    for kmax in range(0, 7):
        c = qs.Circuit(n).add_gates(gates).plan(kmax)
        info = c.info()
        # SWAPs become a renaming of positions, not gates
        assert info["gates"] == sum(g[0] != "swap" for g in gates) and info["blocks"] >= 1
        # a gate wider than kmax is a block of its own
        widest = 3 if n >= 3 else (2 if n == 2 else 1)
        assert info["max_k"] <= max(kmax if kmax else 5, widest)
        for i in range(info["blocks"]):
            qubits, m = c.block(i)
            d = 2 ** len(qubits)
            assert m.shape == (d, d)
            assert np.allclose(m.conj().T @ m, np.eye(d), atol=1e-9)
        if n >= 12:
            c.use_tiles()
            for dtype in (qs.C64, qs.C128):
                t = c.tile_info(dtype)
                assert t["passes"] >= 1 and t["rounds"] >= t["passes"]
        c.free()


def test_circuit_argument_checks(qs):
    lib = qs.open_library()
    h = C.c_void_p()
    assert lib.qs_circuit_create(0, C.byref(h)) == qs.E_INVAL
    assert lib.qs_circuit_create(65, C.byref(h)) == qs.E_INVAL
    assert lib.qs_circuit_create(4, None) == qs.E_INVAL
    c = qs.Circuit(4)
    q2 = (C.c_int * 2)(0, 1)
    bad = (C.c_int * 2)(0, 0)
    far = (C.c_int * 2)(0, 4)
    nan = (C.c_double * 4)(math.nan, 0.0, 0.0, 1.0)
    ok = (C.c_double * 4)(0.1, 0.2, 0.3, 1.0)
    assert lib.qs_circuit_add_gate(c.h, 99, q2, ok) == qs.E_INVAL       # unknown kind
    assert lib.qs_circuit_add_gate(c.h, qs.GATE["cz"], bad, ok) == qs.E_INVAL   # repeated
    assert lib.qs_circuit_add_gate(c.h, qs.GATE["cz"], far, ok) == qs.E_INVAL   # out of range
    assert lib.qs_circuit_add_gate(c.h, qs.GATE["u3"], q2, nan) == qs.E_INVAL   # not finite
    assert lib.qs_circuit_add_gate(c.h, qs.GATE["u3"], q2, None) == qs.E_INVAL  # no params
    assert lib.qs_circuit_add_gate(c.h, qs.GATE["cz"], None, ok) == qs.E_INVAL  # no qubits
    assert lib.qs_circuit_add_gate(None, qs.GATE["cz"], q2, ok) == qs.E_INVAL
    cu = (C.c_double * 4)(0.1, 0.2, 0.3, 0.5)
    assert lib.qs_circuit_add_gate(c.h, qs.GATE["cu3"], q2, cu) == qs.E_INVAL  # control value
    m = np.eye(4).astype(np.complex128).view(np.float64).ravel()
    mp = m.ctypes.data_as(C.POINTER(C.c_double))
    assert lib.qs_circuit_add_matrix(c.h, q2, 0, mp) == qs.E_INVAL
    assert lib.qs_circuit_add_matrix(c.h, q2, 7, mp) == qs.E_INVAL
    assert lib.qs_circuit_add_matrix(c.h, q2, 2, None) == qs.E_INVAL
    assert lib.qs_circuit_add_matrix(c.h, bad, 2, mp) == qs.E_INVAL
    assert lib.qs_circuit_plan(c.h, 7) == qs.E_INVAL
    assert lib.qs_circuit_plan(c.h, -1) == qs.E_INVAL
    assert len(lib.qs_last_error()) > 0
    assert lib.qs_circuit_add_gate(c.h, qs.GATE["cz"], q2, ok) == qs.OK
    c.plan(2)
    k = C.c_int()
    qq = (C.c_int * 6)()
    assert lib.qs_circuit_block(c.h, 5, C.byref(k), qq, None) == qs.E_INVAL
    assert lib.qs_circuit_tile_info(c.h, qs.C64, None, None, None) == qs.E_UNSUPPORTED
    c.free()


def test_every_knob_round_trips(qs):
    lib = qs.open_library()

    def get(key):
        v = C.c_int64()
        assert lib.qs_tune_get(key.encode(), C.byref(v)) == qs.OK
        return v.value

    keys = {"qft.lds_bits": (0, 13, 14), "qft.high_pass": (0, 1, 2), "qft.threads": (0, 512, 300),
            "qft.round_bits": (4, 5, 6), "qft.col_max": (7, 8, 9), "qft.col_rows": (0, 2, 3),
            "tile.low_bits": (4, 6, 7), "tile.mfma": (0, 1, 2), "fused.mfma": (0, 1, 2),
            "factor.multi_test": (0, 1, 2), "factor.batch_1q": (0, 1, 2),
            "factor.defer": (0, 1, 2), "factor.tile_1q": (0, 1, 2),
            "factor.unobservable": (0, 1, 2), "factor.done_flag": (0, 1, 2),
            "factor.fuse_ops": (0, 1, 2), "factor.kernarg_tables": (0, 1, 2),
            "factor.hold": (0, 1, 2), "factor.kickback": (0, 1, 2), "qft.stream": (1, 2, 3), "sweep.stream": (1, 2, 3),
            "gate.shuffle_bits": (0, 6, 7), "gate.dense_ctrl": (0, 1, 2)}
    for key, (a, b, bad) in keys.items():
        saved = get(key)
        try:
            for v in (a, b):
                assert lib.qs_tune_set(key.encode(), v) == qs.OK
                assert get(key) == v
            assert lib.qs_tune_set(key.encode(), bad) == qs.E_INVAL
            assert get(key) == b
        finally:
            assert lib.qs_tune_set(key.encode(), saved) == qs.OK
    v = C.c_int64()
    assert lib.qs_tune_set(b"no.such.knob", 1) == qs.E_INVAL
    assert lib.qs_tune_get(b"no.such.knob", C.byref(v)) == qs.E_INVAL
    assert lib.qs_tune_set(None, 1) == qs.E_INVAL
