"""Approximate-mode run protocols (host orchestration over the C ABI).

`approx_run` applies a gate list to a factorized state with separation after
every multi-qubit gate at threshold p. `minimum_p` is the search of Sec. III-C:
starting from p = 1, lower p by 0.025 after every circuit that completes and
keep the fidelity estimate of the smallest p that completes before the
amplitude cap (the paper's out-of-memory condition) is hit.
"""
from __future__ import annotations

import time

import numpy as np

from . import C64, MLP, SEP_AFTER_2Q, CapacityError, Circuit, State, mlp_init


def approx_run(n: int, gates, p: float, max_amps: int = 2 ** 30, dtype: int = C64,
               record: bool = False, keep: bool = False, features: bool = False,
               proposer=None, cutoff: float = 0.5, retest_on_merge: bool = True,
               min_qubits: int = 2) -> dict:
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
        st.set_proposer(proposer, cutoff, retest_on_merge, min_qubits)
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


def collect_attempts(n: int, circuits, ps, max_amps: int = 2 ** 30, dtype: int = C64):
    """Training data for the proposal network: the features of every exact
    test the plain schedule makes on each circuit at each threshold in ps,
    labelled 1 where the test rounded."""
    X, y = [], []
    for gates in circuits:
        for p in ps:
            r = approx_run(n, gates, p, max_amps=max_amps, dtype=dtype, features=True)
            X.append(r["features"])
            y.append(np.array([a[3] for a in r["log"]], dtype=np.float32))
    return np.concatenate(X), np.concatenate(y)


def train_proposer(X, y, steps: int = 3000, batch: int = 256, lr: float = 3e-3,
                   seed: int = 0, recall: float = 0.95):
    """Train a network on shuffled (X, y) with the library's GPU kernels and
    pick the cutoff: the largest score that still proposes a fraction
    `recall` of the training roundings. Returns (net, cutoff, final loss)."""
    order = np.random.default_rng(seed).permutation(len(y))
    net = MLP(mlp_init(seed))
    loss = net.train(X[order], y[order], steps=steps, batch=min(batch, len(y)), lr=lr)
    pos = np.sort(net.forward(X[y > 0.5]))
    cutoff = float(pos[int(np.floor((1.0 - recall) * len(pos)))]) if len(pos) else 0.5
    return net, cutoff, loss


# width x depth sets of the fidelity-model validation (Appendix: Table of RMSE
# per subset), with the grid each width is laid out on (a line for 19)
VALIDATION_SETS = ((6, 6), (12, 6), (18, 6), (12, 12), (18, 12), (18, 18), (15, 15), (19, 10))
VALIDATION_GRIDS = {6: (2, 3), 12: (3, 4), 15: (3, 5), 18: (3, 6), 19: (1, 19)}


def validation_grid(make_circuit, sets=VALIDATION_SETS, circuits: int = 10, step: float = 0.025,
                    seed0: int = 20000, dtype: int = C64) -> dict:
    """The fidelity model against the gold standard (Appendix, Eq. rmse):
    for every width x depth set, `circuits` circuits from
    make_circuit(rows, cols, depth, seed) on that width's grid; each runs once
    exactly (dense) and once in the approximate mode for every p on 0, step,
    ..., 1, and each run is one observation (F, F_exact = |<approx|exact>|^2).
    Returns the RMSE per set and overall, the observation count and the mean
    signed error F - F_exact."""
    import math

    ps = [round(k * step, 10) for k in range(int(round(1.0 / step)) + 1)]
    per_set, all_err = {}, []
    for width, depth in sets:
        rows, cols = VALIDATION_GRIDS[width]
        errs = []
        for c in range(circuits):
            gates = make_circuit(rows, cols, depth, seed0 + 1000 * width + 100 * depth + c)
            circ = Circuit(width).add_gates(gates)
            exact = State(width, dtype)
            exact.run(circ)
            approx = State(width, dtype)
            for p in ps:
                st = State(width, dtype, factorized=True)
                st.set_policy(SEP_AFTER_2Q, p)
                st.run(circ)
                st.expand_into(approx)
                fx = abs(approx.inner(exact)) ** 2
                errs.append(st.fidelity_estimate() - fx)
                st.free()
            approx.free()
            exact.free()
            circ.free()
        per_set[f"{width}x{depth}"] = round(math.sqrt(sum(e * e for e in errs) / len(errs)), 5)
        all_err += errs
    return {"rmse_per_set": per_set,
            "rmse_overall": round(math.sqrt(sum(e * e for e in all_err) / len(all_err)), 5),
            "mean_err": round(sum(all_err) / len(all_err), 5),
            "observations": len(all_err), "circuits_per_set": circuits, "p_step": step}


def depth_sweep(make_circuit, rows: int, cols: int, depths, circuits: int = 10,
                max_amps: int = 2 ** 30, seed0: int = 30000, dtype: int = C64) -> dict:
    """Achievable fidelity against depth (the experiment of Fig. 3): for each
    depth, `circuits` circuits from make_circuit(rows, cols, depth, seed), the
    descending-p search of each, and the mean, median and spread of the
    fidelity estimate at the smallest completed p (0 where even p = 1 fails)."""
    out = {}
    for d in depths:
        Fs, pmin, secs = [], [], 0.0
        for c in range(circuits):
            r = minimum_p(rows * cols, make_circuit(rows, cols, d, seed0 + 100 * d + c),
                          max_amps=max_amps, dtype=dtype)
            b = r["best"]
            Fs.append(b["F"] if b else 0.0)
            pmin.append(b["p"] if b else None)
            secs += r["search_time_s"]
        ok = [p for p in pmin if p is not None]
        out[str(d)] = {"F_mean": float(np.mean(Fs)), "F_median": float(np.median(Fs)),
                       "F_max": float(np.max(Fs)),
                       "p_min_mean": float(np.mean(ok)) if ok else None,
                       "search_s": round(secs, 3)}
    return out


def heat_map(make_circuit, rows: int, cols: int, depths, ps, circuits: int = 5,
             max_amps: int = 2 ** 30, seed0: int = 40000, dtype: int = C64) -> dict:
    """Fidelity over threshold and depth (the heat maps of the appendix): the
    mean fidelity estimate of `circuits` circuits for every (p, depth), with
    runs that hit the amplitude cap counted as 0 and reported separately."""
    grid, fails = {}, {}
    for d in depths:
        gates = [make_circuit(rows, cols, d, seed0 + 100 * d + c) for c in range(circuits)]
        for p in ps:
            Fs, nf = [], 0
            for g in gates:
                r = approx_run(rows * cols, g, p, max_amps=max_amps, dtype=dtype)
                Fs.append(r["F"] if r["ok"] else 0.0)
                nf += 0 if r["ok"] else 1
            grid[f"{p:g},{d}"] = float(np.mean(Fs))
            fails[f"{p:g},{d}"] = nf
    return {"F_mean": grid, "capacity_failures": fails, "circuits": circuits}
