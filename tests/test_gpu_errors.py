"""Error paths of the C ABI on the GPU and the named-gate call.

qs_apply_gate builds every named gate's matrix inside the library: each kind
against the oracle's gate. Refused arguments leave the state as it was. A
failing device allocator gives QS_E_NOMEM with the state unchanged (a dense
readout that needs staging, a factorized merge), while the no-allocation
gather still works; corrupted amplitudes make qs_check report QS_E_NUMERIC."""
import ctypes as C
import gc
import math

import numpy as np
import pytest

from oracle import dense
from parity import C64, C128, assert_parity

pytestmark = pytest.mark.gpu

E_INVAL, E_NOMEM, E_NUMERIC = -1, -2, -5


def named_gates_and_oracle_form():
    """(gate tuples for the library, the same gates for the oracle): X, Y, Z
    are given to the oracle as explicit matrices."""
    lib = [("h", 0), ("x", 1), ("y", 2), ("z", 3), ("u3", 4, 0.3, 1.1, -0.7),
           ("cz", 0, 5), ("iswap", 1, 4), ("cp", 2, 0, 0.9), ("swap", 3, 5),
           ("cx", 4, 2), ("cy", 5, 1), ("ax", 0, 3), ("ay", 2, 4), ("az", 1, 0),
           ("ctrl", (3,), 0, 2, 1.2, 0.4, 2.2),
           ("ctrl", (0, 4, 5), 0b101, 1, 0.8, -1.3, 0.5),
           ("u3", 5, 2.0, -0.3, 0.6), ("h", 3)]
    mats = {"x": dense.X, "y": dense.Y, "z": dense.Z}
    orc = [("mat", [g[1]], mats[g[0]]) if g[0] in mats else g for g in lib]
    return lib, orc


@pytest.mark.parametrize("dtype", [C64, C128])
@pytest.mark.parametrize("factorized", [False, True])
def test_apply_gate_every_kind_matches_oracle(qs_lib, dtype, factorized):
    qs = qs_lib
    n = 6
    lib, orc = named_gates_and_oracle_form()
    st = qs.State(n, dtype, factorized=factorized)
    try:
        st.apply_1q(0, dense.u3(0.5, 0.1, 0.2))  # off |0...0>
        want = dense.apply_1q(dense.zero_state(n), n, 0, dense.u3(0.5, 0.1, 0.2))
        for g in lib:
            qs.apply_gate(st, g)
        want = dense.run_circuit(want, n, orc)
        assert_parity(st.amplitudes(), want, dtype, f"named gates factorized={factorized}")
    finally:
        st.free()


def test_apply_gate_refusals_leave_the_state(qs_lib):
    qs = qs_lib
    n = 5
    with qs.State(n, C64) as st:
        st.set_amplitudes(dense.qft(dense.basis_state(n, 3), n))
        before = st.amplitudes()

        def call(kind, qubits, params):
            q = (C.c_int * max(1, len(qubits)))(*qubits)
            p = (C.c_double * max(1, len(params)))(*params) if params is not None else None
            return st.lib.qs_apply_gate(st.h, kind, q, len(qubits), p)

        G = qs.GATE
        assert call(99, [0], []) == E_INVAL                       # unknown kind
        assert call(G["h"], [0, 1], []) == E_INVAL                # wrong qubit count
        assert call(G["cx"], [2], []) == E_INVAL
        assert call(G["u3"], [0], [0.1, math.nan, 0.2]) == E_INVAL  # not finite
        assert call(G["u3"], [0], None) == E_INVAL                # missing parameters
        assert call(G["cp"], [1, 1], [0.3]) == E_INVAL            # repeated qubit
        assert call(G["cx"], [0, 5], []) == E_INVAL               # out of range
        assert call(G["cu3"], [0, 1, 2], [0.1, 0.2, 0.3, 4.0]) == E_INVAL  # mask > 2 bits
        assert call(G["cu3"], [0, 1], [0.1, 0.2, 0.3, 0.5]) == E_INVAL     # not a mask
        assert call(G["cu3"], [0, 1, 2, 0], [0.1, 0.2, 0.3, 1.0]) == E_INVAL  # repeated
        np.testing.assert_array_equal(st.amplitudes(), before)


class FailingAllocator:
    """Device allocator hooks over torch's caching allocator that can be made
    to fail (return NULL) on demand."""

    def __init__(self, qs):
        import torch
        self.fail = False

        def _alloc(nbytes, _user):
            if self.fail:
                return None
            return torch.cuda.caching_allocator_alloc(int(nbytes))

        def _free(ptr, _user):
            torch.cuda.caching_allocator_delete(ptr)
        self.alloc_cb, self.free_cb = qs._ALLOC_FN(_alloc), qs._FREE_FN(_free)


def test_failing_allocator_nomem_state_unchanged(qs_lib):
    qs = qs_lib
    lib = qs.load()
    gc.collect()  # states of earlier tests that are no longer referenced
    hooks = FailingAllocator(qs)
    rc = lib.qs_set_allocator(hooks.alloc_cb, hooks.free_cb, None)
    assert rc == 0, lib.qs_last_error()
    states = []
    try:
        # a new state: QS_E_NOMEM, nothing created
        hooks.fail = True
        with pytest.raises(qs.QSError) as e:
            qs.State(8, C64)
        assert e.value.code == E_NOMEM
        hooks.fail = False

        # dense: a readout that needs staging device memory fails; the
        # no-allocation gather does not need any
        n = 10
        a = dense.qft(dense.basis_state(n, 77), n)
        st = qs.State(n, C128)
        states.append(st)
        st.set_amplitudes(a)
        idx = np.array([0, 5, 77, 1023], dtype=np.uint64)
        hooks.fail = True
        with pytest.raises(qs.QSError) as e:
            st.amplitudes(dtype=np.complex64)
        assert e.value.code == E_NOMEM
        with pytest.raises(qs.QSError) as e:
            st.gather(idx)
        assert e.value.code == E_NOMEM
        got = st.gather_noalloc(idx)
        assert np.abs(got - a[idx.astype(np.int64)]).max() < 1e-14
        hooks.fail = False
        np.testing.assert_array_equal(st.amplitudes(), st.amplitudes())
        assert_parity(st.amplitudes(), a, C128, "dense after NOMEM")

        # factorized: a merge into a subsystem size never allocated before
        n = 8
        fs = qs.State(n, C64, factorized=True)
        states.append(fs)
        want = dense.zero_state(n)
        for q in range(n):
            fs.apply_1q(q, dense.H)
            want = dense.apply_1q(want, n, q, dense.H)
        for q in range(4):
            fs.apply_cphase(q, q + 1, 0.7 + 0.1 * q)
            want = dense.apply_cphase(want, n, q, q + 1, 0.7 + 0.1 * q)
        subs_before = fs.subsystems()
        amps_before = fs.amplitudes()
        hooks.fail = True
        with pytest.raises(qs.QSError) as e:
            fs.apply_cphase(4, 5, 1.3)  # 5 + 1 qubits: a new 2^6 buffer
        assert e.value.code == E_NOMEM
        hooks.fail = False
        assert fs.subsystems() == subs_before
        np.testing.assert_array_equal(fs.amplitudes(), amps_before)
        fs.apply_cphase(4, 5, 1.3)  # now it goes through
        want = dense.apply_cphase(want, n, 4, 5, 1.3)
        assert_parity(fs.amplitudes(), want, C64, "factorized after NOMEM")
    finally:
        hooks.fail = False
        for s in states:
            s.free()
        gc.collect()
        assert lib.qs_set_allocator(qs._alloc_cb, qs._free_cb, None) == 0, lib.qs_last_error()


@pytest.mark.parametrize("dtype", [C64, C128])
def test_check_reports_corrupted_amplitudes(qs_lib, dtype):
    qs = qs_lib
    n = 9
    a = dense.qft(dense.basis_state(n, 11), n)
    with qs.State(n, dtype) as st:
        st.set_amplitudes(a)
        st.check(1e-6)  # a normalized ket passes
        bad = a.copy()
        bad[100] *= 3.0  # one amplitude corrupted: the norm drifts
        st.set_amplitudes(bad)
        with pytest.raises(qs.QSError) as e:
            st.check(1e-6)
        assert e.value.code == E_NUMERIC
        bad[100] = complex(math.nan, 0.0)
        st.set_amplitudes(bad)
        with pytest.raises(qs.QSError) as e:
            st.check(1.0)
        assert e.value.code == E_NUMERIC
