"""The autotuner picks among equivalent launch shapes: whatever it leaves set,
the transforms still match the oracle."""
import pytest

import workloads
from oracle import dense
from parity import assert_parity

pytestmark = pytest.mark.gpu


def test_tune_qft_leaves_a_correct_choice(qs_lib):
    from paper_2304_14969_amd import autotune
    qs = qs_lib
    n = 16
    keys = autotune.QFT_KEYS
    saved = {k: qs.tune_get(k) for k in keys}
    try:
        cands = [(0, 0, 512, 4, 7), (12, 1, 256, 5, 8), (11, 0, 256, 4, 8)]
        r = autotune.tune_qft(n, reps=2, candidates=cands)
        assert len(r["tried"]) == 3
        assert tuple(r["best"][k] for k in keys) in cands
        assert r["ms"] == min(t["ms"] for t in r["tried"]) or abs(
            r["ms"] - min(t["ms"] for t in r["tried"])) < 1e-3
        for k in keys:
            assert qs.tune_get(k) == r["best"][k]
        a = workloads.gaussian_state(n, 3)
        st = qs.State(n, qs.C64)
        st.set_amplitudes(a)
        st.qft()
        assert_parity(st.amplitudes(), dense.qft(a, n), qs.C64, "tuned QFT")
        st.free()
    finally:
        for k, v in saved.items():
            qs.tune_set(k, v)


def test_tune_fusion_and_batch(qs_lib):
    from paper_2304_14969_amd import autotune
    qs = qs_lib
    keys = ("fused.mfma", "tile.mfma", "tile.low_bits")
    saved = {k: qs.tune_get(k) for k in keys}
    try:
        n = 14
        gates = workloads.random_circuit(n, 4, 5)
        r = autotune.tune_fusion(n, gates, kmaxes=(3, 4), tile_bits=(5, 6), reps=2)
        assert len(r["tried"]) == 4 + 4
        st = qs.State(n, qs.C64)
        c = qs.Circuit(n).add_gates(gates)
        c = c.use_tiles() if r["tiles"] else c.plan(r["kmax"])
        st.run(c)
        want = dense.run_circuit(dense.basis_state(n, 0), n, gates)
        assert_parity(st.amplitudes(), want, qs.C64, "tuned fusion")
        st.free()
        c.free()
        widths = workloads.batch_widths(16, 4, low=6, high=10)
        circs = [qs.Circuit(w).add_gates(workloads.random_circuit(w, 3, 40 + i))
                 for i, w in enumerate(widths)]
        rb = autotune.tune_batch(widths, circs, kmaxes=(2, 4), reps=2)
        assert rb["kmax"] in (2, 4)
        for c in circs:
            c.free()
    finally:
        for k, v in saved.items():
            qs.tune_set(k, v)
