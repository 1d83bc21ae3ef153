"""The descending-p protocol of Sec. III-C on a small case with a tight cap."""
import pytest

import workloads
from parity import C64

pytestmark = pytest.mark.gpu


def test_minimum_p_is_the_boundary(qs_lib):
    from paper_2304_14969_amd import protocol
    n = 12
    gates = workloads.grid_circuit(3, 4, 6, 3)
    cap = 2 ** 6
    res = protocol.minimum_p(n, gates, max_amps=cap, step=0.1)
    best = res["best"]
    assert best is not None and best["ok"]
    assert best["max_sub"] <= 6
    p = best["p"]
    # the next p down fails (unless p reached 0)
    if p > 1e-9:
        nxt = protocol.approx_run(n, gates, round(p - 0.1, 10), max_amps=cap)
        assert not nxt["ok"]
    # runs are deterministic: the same p completes again with the same F
    again = protocol.approx_run(n, gates, p, max_amps=cap)
    assert again["ok"] and again["F"] == best["F"]


def test_exact_run_never_rounds_with_big_cap(qs_lib):
    from paper_2304_14969_amd import protocol
    n = 10
    r = protocol.approx_run(n, workloads.grid_circuit(2, 5, 5, 1), 0.0, record=True)
    assert r["ok"] and abs(r["F"] - 1) < 1e-5
    assert all(a[2] <= 1e-5 for a in r["log"] if a[3])


def test_validation_grid_small(qs_lib):
    """The validation protocol on one small set: every p from 0 to 1 in steps
    of 0.25 gives one observation; the model tracks the exact fidelity."""
    from paper_2304_14969_amd import protocol
    r = protocol.validation_grid(workloads.grid_circuit, sets=((6, 6), (12, 6)), circuits=2,
                                 step=0.25)
    assert r["observations"] == 2 * 2 * 5
    assert set(r["rmse_per_set"]) == {"6x6", "12x6"}
    assert 0.0 <= r["rmse_overall"] < 0.15 and abs(r["mean_err"]) < 0.1
