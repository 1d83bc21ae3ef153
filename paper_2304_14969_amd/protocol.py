"""Approximate-mode run protocols (host orchestration over the C ABI).

`approx_run` applies a gate list to a factorized state with separation after
every multi-qubit gate at threshold p. `minimum_p` is the search of Sec. III-C:
starting from p = 1, lower p by 0.025 after every circuit that completes and
keep the fidelity estimate of the smallest p that completes before the
amplitude cap (the paper's out-of-memory condition) is hit.
"""
from __future__ import annotations

import time

from . import C64, SEP_AFTER_2Q, CapacityError, Circuit, State


def approx_run(n: int, gates, p: float, max_amps: int = 2 ** 30, dtype: int = C64,
               record: bool = False, keep: bool = False, features: bool = False,
               proposer=None, cutoff: float = 0.5) -> dict:
    """One run; returns completion, time, fidelity estimate and table stats.
    With keep=True the state is returned under "state" (caller frees it).
    features=True also returns the proposal features of every attempt;
    proposer= runs the learned schedule."""
    import torch

    st = State(n, dtype, factorized=True, max_amps=max_amps)
    st.set_policy(SEP_AFTER_2Q, p)
    if record or features:
        record = True
        st.record_attempts()
    if features:
        st.record_features()
    if proposer is not None:
        st.set_proposer(proposer, cutoff)
    circ = Circuit(n).add_gates(gates)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok = True
    try:
        st.run(circ)
    except CapacityError:
        ok = False
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    subs = st.subsystems()
    out = {"ok": ok, "p": p, "time_s": dt, "F": st.fidelity_estimate(),
           "max_sub": max(len(s) for s in subs), "n_sub": len(subs)}
    if record:
        att = st.attempts()
        out["attempts"] = len(att)
        out["roundings"] = sum(a[3] for a in att)
        out["log"] = att
    if features:
        out["features"] = st.features()
    if proposer is not None:
        out.update(st.proposer_stats())
    circ.free()
    if keep:
        out["state"] = st
    else:
        st.free()
    return out


def minimum_p(n: int, gates, max_amps: int = 2 ** 30, step: float = 0.025,
              dtype: int = C64) -> dict:
    """Smallest p on the grid 1, 1-step, ... that completes; its run record
    plus the number of runs and the total time spent in the search."""
    best = None
    runs = 0
    total = 0.0
    k = 0
    while True:
        p = round(1.0 - k * step, 10)
        if p < 0:
            break
        r = approx_run(n, gates, p, max_amps=max_amps, dtype=dtype)
        runs += 1
        total += r["time_s"]
        if not r["ok"]:
            break
        best = r
        k += 1
    return {"best": best, "runs": runs, "search_time_s": total}
