"""Benchmark: exact QFT on 27 qubits, complex64 (1 GiB), on one MI355X.

One step = one full QFT-27 (qs_qft over all 27 qubits, bit reversal included
as a relabelling) on a state resident in HBM. The input is an i.i.d. complex
Gaussian vector (seed 0), normalized, uploaded before the timed region.
Consecutive steps transform the state again; each step is a complete QFT.

Printed: one JSON line with the time per QFT-27, the dominant kernel's
achieved HBM bandwidth against the 8 TB/s peak (HIP events around every
launch inside the timed region, algorithmic bytes from the library), and the
FP64 oracle timed on the host cores on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 27] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the QFT pass kernels, from two rocprofv3 --pmc runs
# of `bench.py --quick` (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
# scaled by what the counter reads for a copy of a known 1 GiB
# (`bench.py --calibrate-copy`: FETCH_SIZE reads 0.50002 of the bytes copied,
# WRITE_SIZE 1.00000). Valid only for the kernel source they were taken on.
TRAFFIC_SOURCE = os.path.join(ROOT, "paper_2304_14969_amd", "csrc", "k_qft.hip")
TRAFFIC = {"sha256": "520832e791190b013b4035e0ae100f64b1a51a8c2b966522abec2112a7e844bb",
           "bytes_per_launch": {"qft_col8": 2147830219, "qft_lds": 2147588925}}


def measured_traffic(kernel: str):
    import hashlib
    if TRAFFIC["sha256"] is None:
        return None
    with open(TRAFFIC_SOURCE, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != TRAFFIC["sha256"]:
            return None
    return TRAFFIC["bytes_per_launch"].get(kernel)
METRIC = "exact QFT-27 seconds & HBM GB/s; 54q×7-layer approx time at equal fidelity"


def cpu_baseline(n: int, m: int = 20) -> dict:
    """The FP64 oracle as it is, timed on one host core (numpy/BLAS limited
    to one thread): the whole QFT circuit of an m-qubit complex Gaussian
    state (H and controlled phases gate by gate, the bit reversal as SWAPs
    that move amplitudes), one warm-up run, then the median of three. Scaled
    to n qubits by the gate count and the vector length (every oracle gate
    sweeps the whole vector). Beside it, the per-gate cost at n qubits: one H,
    one controlled phase and one SWAP on a 2^n vector (median of three
    each), weighted by the n-qubit gate counts."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import dense

    a = workloads.gaussian_state(m, 1)
    runs = []
    with threadpool_limits(1):
        dense.qft(a, m)
        for _ in range(3):
            t0 = time.perf_counter()
            dense.qft(a, m)
            runs.append(time.perf_counter() - t0)
    med = sorted(runs)[1]
    cm, cn = workloads.qft_gate_counts(m), workloads.qft_gate_counts(n)
    scale = sum(cn.values()) / sum(cm.values()) * 2.0 ** (n - m)
    g = np.random.default_rng(1)
    x = (g.standard_normal(2 ** n) + 1j * g.standard_normal(2 ** n)) / math.sqrt(2 ** (n + 1))
    per = {}
    with threadpool_limits(1):
        for kind, fn in (("h", lambda v: dense.apply_1q(v, n, n - 1, dense.H)),
                         ("cp", lambda v: dense.apply_cphase(v, n, 3, n - 2, 0.1)),
                         ("swap", lambda v: dense.apply_swap(v, n, 0, n - 1))):
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                fn(x)
                ts.append(time.perf_counter() - t0)
            per[kind] = sorted(ts)[1]
    del x
    per_gate = sum(cn[k] * per[k] for k in cn)
    return {"value": med * scale, "unit": f"s per QFT-{n}", "cores": 1, "kind": "oracle",
            "host_cpus": os.cpu_count(), "affinity_cpus": len(os.sched_getaffinity(0)),
            "sample": (f"oracle QFT circuit on a {m}-qubit complex128 Gaussian state, 1 thread: "
                       f"{med:.3f} s (median of 3 after a warm-up; runs "
                       f"{', '.join(f'{r:.3f}' for r in runs)}), scaled by the gate count "
                       f"({sum(cn.values())} / {sum(cm.values())}) and the length 2^{n - m}"),
            "per_gate_estimate": {"value": per_gate, "h_s": per["h"], "cp_s": per["cp"],
                                  "swap_s": per["swap"],
                                  "note": f"one gate of each kind on a 2^{n} vector, median of 3, "
                                          f"weighted by {cn['h']} H + {cn['cp']} CP + "
                                          f"{cn['swap']} SWAP"}}


def error_vs_oracle(qs, workloads, n: int, a, js=(0, 1, 12345, 2 ** 26 + 3, 2 ** 27 - 1)) -> dict:
    """One QFT of the benchmark's input on the GPU against single outputs of
    the oracle's direct sum of Eq. dft (float64)."""
    import numpy as np
    from oracle import dense

    js = [j % (2 ** n) for j in js]
    with qs.State(n, qs.C64) as st:
        st.set_amplitudes(a)
        st.qft()
        got = st.gather(np.array(js, dtype=np.uint64))
    want = dense.dft_entries(a, n, js)
    d = np.abs(got - want)
    return {"outputs": js, "max_abs": float(d.max()), "max_rel": float(d.max() / np.abs(want).max()),
            "reference": "oracle direct sum of Eq. dft, float64"}


def _kernel_rates(prof: dict, flops_of=None) -> dict:
    out = {}
    for k, v in prof.items():
        avg = v["total_ms"] / v["launches"]
        row = {"launches": v["launches"], "avg_ms": round(avg, 4),
               "GBps": round(v["bytes"] / v["launches"] / (avg * 1e-3) / 1e9, 1)}
        if flops_of is not None and flops_of(k):
            row["TFLOPs"] = round(flops_of(k) / (avg * 1e-3) / 1e12, 2)
        out[k] = row
    return out


def bench_circuit(qs, workloads, torch, n: int = 32, layers: int = 10, seed: int = 0,
                  kmaxes=(4, 5)) -> dict:
    """Exact random circuit (U3 on every qubit, then CZ/iSWAP on a random
    matching, per layer): tile passes (several gates per HBM sweep, rounds of
    dense 4-qubit blocks on the matrix cores), and for comparison one sweep
    per fused block of at most kmax qubits, for each kmax in kmaxes."""
    gates = workloads.random_circuit(n, layers, seed)
    st = qs.State(n, qs.C64)
    out = {"workload": f"random circuit n={n}, {layers} layers (U3 + CZ/iSWAP matching), "
                       f"seed {seed}, complex64", "gates": len(gates)}
    for mode in ("tiles",) + tuple(kmaxes):
        c = qs.Circuit(n).add_gates(gates)
        if mode == "tiles":
            c.use_tiles()
            ti = c.tile_info(qs.C64)
        else:
            kmax = mode
            c.plan(kmax)
        st.set_basis(0)
        st.run(c)
        torch.cuda.synchronize()
        st.set_basis(0)
        st.profile_start()
        t0 = time.perf_counter()
        st.run(c)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = st.profile_stop()
        norm = st.norm()
        if mode == "tiles":
            def flops(name, rounds=ti["rounds"], passes=ti["passes"]):
                # dense 16x16 complex blocks: 8 x 16 real flops per amplitude per round
                return 8.0 * 16 * 2 ** n * rounds / passes if name == "tile_mfma" else 0.0
            out["tiles"] = {"s": round(dt, 4), "sweeps": ti["passes"], "rounds": ti["rounds"],
                            "norm_after": norm, "kernels": _kernel_rates(prof, flops)}
        else:
            def flops(name):  # complex (2^k x 2^k) times 2^n amplitudes, 8 real flops per MAC
                for k in (4, 5):
                    if name.startswith(f"fused{k}_mfma"):
                        return 8.0 * 2 ** k * 2 ** n
                return 0.0
            out[f"blocks_k{kmax}"] = {"s": round(dt, 4), "sweeps": c.info()["blocks"],
                                      "norm_after": norm, "kernels": _kernel_rates(prof, flops)}
        c.free()
    st.free()
    out["s"] = out["tiles"]["s"]
    return out


FP32_MFMA_PEAK_TFLOPS = 157.3
FP64_MFMA_PEAK_TFLOPS = 78.6


def bench_sweeps(qs, np, torch, n: int = 30, reps: int = 6) -> dict:
    """Per-gate sweeps and fused blocks on an n-qubit complex64 state (8 GiB at
    30): average launch time, algorithmic bytes per second (every amplitude
    the gate changes read and written once) against the 8 TB/s peak, and for
    the matrix-core blocks flops against the FP32 matrix peak. One-qubit gates
    on bits 1-6 exchange partners by wavefront shuffles, from bit 7 on they
    read strided pairs. Gates with a control or phase bit below bit 3 change
    amplitudes in runs shorter than a 64-byte segment, so their sweeps move
    whole segments for part of them."""
    def haar(d, seed):
        g = np.random.default_rng(seed)
        z = (g.standard_normal((d, d)) + 1j * g.standard_normal((d, d))) / math.sqrt(2)
        q, r = np.linalg.qr(z)
        return q * (np.diag(r) / np.abs(np.diag(r)))

    H = np.array([[1, 1], [1, -1]]) / math.sqrt(2)
    X = np.array([[0, 1], [1, 0]])
    st = qs.State(n, qs.C64)
    st.set_basis(1)
    ops = [("1q bit 0", lambda: st.apply_1q(0, H)), ("1q bit 1", lambda: st.apply_1q(1, H)),
           ("1q bit 3", lambda: st.apply_1q(3, H)), ("1q bit 6", lambda: st.apply_1q(6, H)),
           ("1q bit 7", lambda: st.apply_1q(7, H)),
           ("1q bit 15", lambda: st.apply_1q(15, H)), (f"1q bit {n - 1}", lambda: st.apply_1q(n - 1, H)),
           ("cx 5 -> 22", lambda: st.apply_ctrl([5], 1, 22, X)),
           ("cx 1 -> 22", lambda: st.apply_ctrl([1], 1, 22, X)),
           ("cphase 5,17", lambda: st.apply_cphase(5, 17, 0.3)),
           ("cphase 2,17", lambda: st.apply_cphase(2, 17, 0.3)),
           ("fused 2 (4, 21)", lambda: st.apply_fused([4, 21], haar(4, 1))),
           ("fused 3 (6, 13, 25)", lambda: st.apply_fused([6, 13, 25], haar(8, 2))),
           ("fused 4 (2, 8, 19, 27)", lambda: st.apply_fused([2, 8, 19, 27], haar(16, 3))),
           ("fused 5 (0, 6, 13, 22, 28)", lambda: st.apply_fused([0, 6, 13, 22, 28], haar(32, 4)))]
    out = {"workload": f"one gate or fused block at a time on n={n} qubits, complex64 "
                       f"({2 ** n * 8 / 2 ** 30:g} GiB); the c128 rows on n={n - 1} qubits, "
                       f"complex128 (the same bytes)", "peak_GBps": HBM_PEAK_GBS, "gates": {}}

    def measure(st, nq, ops, prefix, mfma_peak):
        for name, fn in ops:
            fn()
            torch.cuda.synchronize()
            st.profile_start()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            prof = st.profile_stop()
            (kname, v), = prof.items()
            avg = v["total_ms"] / v["launches"]
            gbps = v["bytes"] / v["launches"] / (avg * 1e-3) / 1e9
            row = {"kernel": kname, "avg_ms": round(avg, 4), "GBps": round(gbps, 1),
                   "frac": round(gbps / HBM_PEAK_GBS, 3)}
            if kname.endswith("_mfma"):
                k = int(kname[5])
                tflops = 8.0 * 2 ** k * 2 ** nq / (avg * 1e-3) / 1e12
                row["TFLOPs"] = round(tflops, 2)
                row["mfma_frac"] = round(tflops / mfma_peak, 3)
            out["gates"][prefix + name] = row

    measure(st, n, ops, "", FP32_MFMA_PEAK_TFLOPS)
    st.free()
    # complex128 blocks run on the FP64 matrix cores
    st = qs.State(n - 1, qs.C128)
    st.set_basis(1)
    ops = [("1q bit 5", lambda: st.apply_1q(5, H)),
           ("fused 3 (6, 13, 25)", lambda: st.apply_fused([6, 13, 25], haar(8, 2))),
           ("fused 4 (2, 8, 19, 27)", lambda: st.apply_fused([2, 8, 19, 27], haar(16, 3))),
           ("fused 5 (0, 6, 13, 22, 28)", lambda: st.apply_fused([0, 6, 13, 22, 28], haar(32, 4)))]
    measure(st, n - 1, ops, "c128 ", FP64_MFMA_PEAK_TFLOPS)
    st.free()
    return out


def bench_qft_sizes(qs, workloads, torch, sizes=range(28, 33), steps: int = 5) -> dict:
    """Exact QFT at 28 to 32 qubits (complex64, 2 to 32 GiB): time per
    transform, passes, and each pass kernel's average time and GB/s. The
    state is made dense by transforming a basis state first (pass times do
    not depend on the values)."""
    out = {"workload": "exact QFT on n = 28 ... 32 qubits, complex64 (2 - 32 GiB), dense state "
                       "(QFT of a basis state, x from seed n), resident in HBM"}
    for n in sizes:
        st = qs.State(n, qs.C64)
        st.set_basis(workloads.basis_index(n, n))
        st.qft()
        st.qft()
        stream = torch.cuda.current_stream()
        torch.cuda.synchronize()
        st.profile_start()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            st.qft()
        e1.record(stream)
        torch.cuda.synchronize()
        prof = st.profile_stop()
        ms = e0.elapsed_time(e1) / steps
        passes = sum(v["launches"] for v in prof.values()) / steps
        total = sum(v["bytes"] for v in prof.values()) / steps
        out[f"n{n}"] = {"ms_per_qft": round(ms, 4), "passes": passes,
                        "hbm_GBps_effective": round(total / (ms * 1e-3) / 1e9, 1),
                        "kernels": _kernel_rates(prof), "norm_after": st.norm()}
        st.free()
        print(f"qft sizes: n={n} done ({ms:.3f} ms per transform)", file=sys.stderr, flush=True)
    return out


def bench_approx(qs, workloads, protocol, np, family: str, p_cmp: float = 0.6,
                 test_seeds=range(10), train_seeds=range(10000, 10060),
                 train_ps=(0.7, 0.6, 0.5), min_qubits: int = 12) -> dict:
    """54-qubit, 7-layer approximate runs: the paper's descending-p search,
    then plain vs learned schedule at one threshold on held-out circuits."""
    if family == "grid":
        gen = lambda s: workloads.grid_circuit(6, 9, 7, s)  # noqa: E731
        desc = "6x9 grid, U3 + nearest-neighbour couplers in the ABCDCDAB pattern, 7 layers"
    else:
        gen = lambda s: workloads.random_circuit(54, 7, s)  # noqa: E731
        desc = "54 qubits, U3 + CZ/iSWAP on a random matching, 7 layers"
    out = {"workload": desc + ", complex64, cap 2^30 amplitudes"}
    search = []
    for s in list(test_seeds)[:3]:
        r = protocol.minimum_p(54, gen(s))
        b = r["best"]
        search.append({"seed": s, "p_min": b and b["p"], "F": b and b["F"],
                       "run_s": b and round(b["time_s"], 4), "max_sub": b and b["max_sub"],
                       "runs": r["runs"], "search_s": round(r["search_time_s"], 3)})
    out["minimum_p"] = search
    t0 = time.perf_counter()
    X, y = protocol.collect_attempts(54, [gen(s) for s in train_seeds], train_ps)
    net, cutoff, loss = protocol.train_proposer(X, y, recall=0.97)
    out["training"] = {"rows": int(len(y)), "positive": round(float(y.mean()), 4),
                       "loss": round(loss, 4), "cutoff": round(cutoff, 4),
                       "collect_and_train_s": round(time.perf_counter() - t0, 2)}
    # "plain_per_gate": the paper's form, every gate and every test launched
    # and synchronized on its own; "plain": the same decisions with tests
    # deferred and batched; "learned": batched, with the proposal network
    per_gate = {"factor.defer": 0, "factor.batch_1q": 0, "factor.tile_1q": 0}
    rows = {"plain_per_gate": [], "plain": [], "learned": []}
    for s in test_seeds:
        g = gen(s)
        saved = {k: qs.tune_get(k) for k in per_gate}
        for k, v in per_gate.items():
            qs.tune_set(k, v)
        try:
            rows["plain_per_gate"].append(protocol.approx_run(54, g, p_cmp, record=True))
        finally:
            for k, v in saved.items():
                qs.tune_set(k, v)
        rows["plain"].append(protocol.approx_run(54, g, p_cmp, record=True))
        rows["learned"].append(protocol.approx_run(54, g, p_cmp, record=True, proposer=net,
                                                   cutoff=cutoff, min_qubits=min_qubits))
    net.free()
    cmp = {}
    for k, rs in rows.items():
        ok = [r for r in rs if r["ok"]]
        cmp[k] = {"completed": len(ok), "of": len(rs),
                  "time_s_mean": round(sum(r["time_s"] for r in rs) / len(rs), 5),
                  "time_s_median": round(float(np.median([r["time_s"] for r in rs])), 5),
                  "logF_mean": round(float(np.mean([np.log(r["F"]) for r in ok])), 3) if ok else None,
                  "exact_tests": sum(r["attempts"] for r in rs),
                  "roundings": sum(r["roundings"] for r in rs)}
    cmp["p"] = p_cmp
    cmp["learned_rule_violations"] = sum(1 for r in rows["learned"] for a in r["log"]
                                         if a[3] and a[2] > p_cmp / 2 + 1e-6)
    out["plain_vs_learned"] = cmp
    return out


def test_costs(qs, workloads, np, torch, sizes=(8, 12, 16, 20, 24, 27), reps: int = 5) -> dict:
    """What one exact separability test and one proposal cost: a factorized
    state whose qubits all share one entangled subsystem of n_S qubits, every
    qubit marked dirty, tested at p = 0 (nothing rounds); and one scoring call
    of the network on 54 rows of features."""
    out = {}
    for ns in sizes:
        # U3 on every qubit, a chain of CZ, U3 again: one entangled subsystem
        ang = np.random.default_rng(500 + ns).uniform(0.0, 2 * math.pi, (2, ns, 3))
        gates = ([("u3", q, *map(float, ang[0, q])) for q in range(ns)]
                 + [("cz", q, q + 1) for q in range(ns - 1)]
                 + [("u3", q, *map(float, ang[1, q])) for q in range(ns)])
        ts = []
        for _ in range(reps):
            st = qs.State(ns, qs.C64, factorized=True, max_amps=2 ** 30)
            c = qs.Circuit(ns).add_gates(gates)
            st.run(c)
            assert len(st.subsystems()) == 1
            st.mark_dirty((1 << ns) - 1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st.try_separate(0.0)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) / ns)
            st.free()
            c.free()
        out[f"exact_test_n{ns}_us"] = round(float(np.median(ts)) * 1e6, 2)
    net = qs.MLP(qs.mlp_init(1))
    X = np.random.default_rng(2).standard_normal((54, 32)).astype(np.float32)
    net.forward(X)
    ts = []
    for _ in range(20):
        t0 = time.perf_counter()
        net.forward(X)
        ts.append(time.perf_counter() - t0)
    net.free()
    out["proposal_54_rows_us"] = round(float(np.median(ts)) * 1e6, 2)
    return out


def bench_learned(qs, workloads, protocol, np, torch, widths=(36, 45, 54), depths=(7, 10),
                  test_seeds=range(8), rows_target: int = 100000, reps: int = 3) -> dict:
    """The learned proposal where exact tests are many and large: random
    circuits (U3 + CZ/iSWAP on a random matching) of 36, 45 and 54 qubits with
    7 and 10 layers, each held-out circuit at its own smallest completing p
    (the descending search, cap 2^30). One network is trained on about 1e5
    attempts of the plain schedule on seeds from 10,000, at thresholds around
    each configuration's p_min. Both schedules run every test circuit at the
    same p (median of `reps` runs); reported: completions, mean time, mean
    log F, exact tests and skipped tests."""
    out = {"workload": "random circuits (U3 + CZ/iSWAP matching), 36/45/54 qubits, 7 and 10 "
                       "layers, each at its smallest completing p, cap 2^30, complex64"}
    gen = {(n, d): (lambda s, n=n, d=d: workloads.random_circuit(n, d, s))
           for n in widths for d in depths}
    pmins = {}
    for key, g in gen.items():
        pm = []
        for s in test_seeds:
            r = protocol.minimum_p(key[0], g(s))
            pm.append(r["best"]["p"] if r["best"] else None)
        pmins[key] = pm
    t0 = time.perf_counter()
    Xs, ys, rows, seed = [], [], 0, 10000
    while rows < rows_target:
        for (n, d), g in gen.items():
            ok = [p for p in pmins[(n, d)] if p is not None]
            base = float(np.median(ok)) if ok else 1.0
            ps = [q for q in (base - 0.05, base, base + 0.05, base + 0.1) if 0.0 < q <= 1.0]
            X, y = protocol.collect_attempts(n, [g(seed)], ps)
            Xs.append(X)
            ys.append(y)
            rows += len(y)
        seed += 1
    X, y = np.concatenate(Xs), np.concatenate(ys)
    net, cutoff, loss = protocol.train_proposer(X, y, steps=6000, recall=0.97)
    out["training"] = {"rows": int(len(y)), "positive": round(float(y.mean()), 4),
                       "seeds": f"10000-{seed - 1}", "loss": round(loss, 4),
                       "cutoff": round(cutoff, 4),
                       "collect_and_train_s": round(time.perf_counter() - t0, 1)}
    for (n, d), g in gen.items():
        res = {"plain": [], "learned": []}
        for s, p in zip(test_seeds, pmins[(n, d)]):
            if p is None:
                continue
            gates = g(s)
            for form in ("plain", "learned"):
                kw = {} if form == "plain" else {"proposer": net, "cutoff": cutoff}
                runs = [protocol.approx_run(n, gates, p, record=True, **kw) for _ in range(reps)]
                r = runs[-1]
                res[form].append({"ok": all(x["ok"] for x in runs),
                                  "t": float(np.median([x["time_s"] for x in runs])),
                                  "F": r["F"], "tests": r["attempts"],
                                  "skipped": r.get("skipped", 0), "max_sub": r["max_sub"]})
        row = {"p_min": pmins[(n, d)]}
        for form, rs in res.items():
            ok = [x for x in rs if x["ok"]]
            row[form] = {"completed": len(ok), "of": len(rs),
                         "time_ms_mean": round(1e3 * float(np.mean([x["t"] for x in rs])), 3)
                         if rs else None,
                         "logF_mean": round(float(np.mean([np.log(x["F"]) for x in ok])), 3)
                         if ok else None,
                         "exact_tests": sum(x["tests"] for x in rs),
                         "skipped": sum(x["skipped"] for x in rs),
                         "max_sub": max((x["max_sub"] for x in rs), default=None)}
        out[f"n{n}_d{d}"] = row
        print(f"learned: n={n} d={d} {json.dumps(row)}", file=sys.stderr, flush=True)
    net.free()
    out["costs"] = test_costs(qs, workloads, np, torch)
    return out


def bench_pairs(qs, workloads, np, torch, n: int = 54, layers: int = 7, seeds=range(5)) -> dict:
    """Entangled pairs weakly coupled along a chain (the workload of the
    two-qubit rounding): the one-qubit schedule against the pair policy at
    several thresholds, amplitude cap 2^30."""
    out = {"workload": f"{n}-qubit chain of entangled pairs, {layers} layers (U3, weak controlled "
                       "RY between neighbouring pairs, CNOT inside pairs), complex64, cap 2^30"}
    for name, policy, p in (("single_p0.05", qs.SEP_AFTER_2Q, 0.05),
                            ("single_p0.1", qs.SEP_AFTER_2Q, 0.1),
                            ("single_p0.2", qs.SEP_AFTER_2Q, 0.2),
                            ("pairs_p0.05", qs.SEP_AFTER_2Q_PAIRS, 0.05),
                            ("pairs_p0.1", qs.SEP_AFTER_2Q_PAIRS, 0.1)):
        rows = []
        for s in seeds:
            st = qs.State(n, qs.C64, factorized=True, max_amps=2 ** 30)
            st.set_policy(policy, p)
            c = qs.Circuit(n).add_gates(workloads.pair_chain_circuit(n, layers, s))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ok = True
            try:
                st.run(c)
            except qs.CapacityError:
                ok = False
            torch.cuda.synchronize()
            rows.append({"ok": ok, "t": time.perf_counter() - t0, "F": st.fidelity_estimate(),
                         "max_sub": max(len(x) for x in st.subsystems())})
            st.free()
            c.free()
        ok = [r for r in rows if r["ok"]]
        out[name] = {"completed": len(ok), "of": len(rows),
                     "time_s_median": round(float(np.median([r["t"] for r in rows])), 5),
                     "F_mean": round(float(np.mean([r["F"] for r in ok])), 4) if ok else None,
                     "max_sub_max": max(r["max_sub"] for r in rows)}
    return out


def bench_qft_factorized(qs, workloads, np, torch) -> dict:
    """QFT on factorized states (the inputs of Fig. 1): |0...0> and basis
    states, which the Z-eigenstate shortcut keeps a product of one-qubit
    subsystems, and a GHZ state, whose single subsystem runs the dense passes."""
    out = {"workload": "QFT on factorized complex64 states: |0...0>, |x> (x from the seed), GHZ"}
    for n in (27, 63):
        for kind in ("zero", "basis"):
            ts = []
            for rep in range(5):
                st = qs.State(n, qs.C64, factorized=True)
                if kind == "basis":
                    st.set_basis(workloads.basis_index(n, rep))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st.qft()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                nsub = len(st.subsystems())
                st.free()
            out[f"{kind}_n{n}"] = {"ms_median": round(float(np.median(ts[1:])) * 1e3, 3),
                                   "subsystems_after": nsub}
    n = 27
    ts = []
    for rep in range(3):
        st = qs.State(n, qs.C64, factorized=True)
        c = qs.Circuit(n).add_gates([("h", 0)] + [("cx", q, q + 1) for q in range(n - 1)])
        st.run(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.qft()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        st.free()
        c.free()
    out[f"ghz_n{n}"] = {"ms_median": round(float(np.median(ts)) * 1e3, 3)}
    return out


def bench_held(qs, workloads, np, torch) -> dict:
    """Held controlled phases and inversions (factor.hold) in exact factorized
    runs, on and off, and holding with the kickback shortcut off
    (factor.kickback): Bernstein-Vazirani circuits (every CX lands on an
    ancilla in |->) and a mix of controlled phases, inversions and the
    one-qubit gates that move them; cap 2^30 amplitudes, complex64."""
    out = {"workload": "exact factorized runs, complex64, cap 2^30: Bernstein-Vazirani "
                       "(n - 1 data qubits, ancilla in |->); held_gate_mix (2000 gates)"}
    saved = qs.tune_get("factor.hold")
    saved_kick = qs.tune_get("factor.kickback")

    def run(n, gates, hold, reps, kick=1):
        qs.tune_set("factor.hold", hold)
        qs.tune_set("factor.kickback", kick)
        ts, info = [], {}
        for _ in range(reps):
            st = qs.State(n, qs.C64, factorized=True, max_amps=2 ** 30)
            c = qs.Circuit(n).add_gates(gates)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            try:
                st.run(c)
                torch.cuda.synchronize()
            except qs.CapacityError as e:
                info = {"completed": False, "error": str(e)[:80]}
                st.free()
                c.free()
                break
            ts.append(time.perf_counter() - t0)
            subs = st.subsystems()
            held, removed = st.held_count()
            info = {"completed": True, "largest_subsystem": max(len(x) for x in subs),
                    "subsystems": len(subs), "held": held, "removed": removed,
                    "shortcuts": st.shortcut_count()}
            st.free()
            c.free()
        if ts:
            info["ms_median"] = round(float(np.median(ts)) * 1e3, 3)
        return info

    try:
        for n in (24, 40, 55):
            gates, secret = workloads.phase_kickback_circuit(n, n)
            for hold in (1, 0):
                out[f"bv_n{n}_hold{hold}"] = dict(run(n, gates, hold, 5), ones=sum(secret))
            out[f"bv_n{n}_hold1_kickback0"] = dict(run(n, gates, 1, 5, kick=0), ones=sum(secret))
        gates = workloads.held_gate_mix(24, 2000, 7)
        for hold in (1, 0):
            out[f"mix_n24_hold{hold}"] = run(24, gates, hold, 3)
    finally:
        qs.tune_set("factor.hold", saved)
        qs.tune_set("factor.kickback", saved_kick)
    return out


def bench_batch(qs, workloads, torch, count: int = 1024, seed: int = 300, depth: int = 8) -> dict:
    """Many small random circuits (12-20 qubits) in one arena: batched tile
    passes (one launch per pass index over all kets), batched fused blocks
    (one launch per block width per pass), each eager and as a replayed HIP
    graph, and one state at a time."""
    widths = workloads.batch_widths(count, seed)
    circs = [qs.Circuit(n).add_gates(workloads.random_circuit(n, depth, seed * 1000 + i))
             for i, n in enumerate(widths)]
    out = {"workload": f"{count} random circuits of 12-20 qubits, depth {depth}, complex64"}
    for mode in ("tiles", "blocks"):
        b = qs.Batch(widths, qs.C64, stream=torch.cuda.Stream())  # capture needs its own stream
        b.use_tiles(mode == "tiles")
        b.run(circs, 4)
        b.synchronize()
        t0 = time.perf_counter()
        b.reset()
        b.run(circs, 4)
        b.synchronize()
        t_run = time.perf_counter() - t0
        b.capture(circs, 4)
        b.reset()
        b.replay()
        b.synchronize()
        t0 = time.perf_counter()
        b.reset()
        b.replay()
        b.synchronize()
        t_graph = time.perf_counter() - t0
        info = b.info()
        b.free()
        out[mode] = {"launches": info["launches"], "batched_s": round(t_run, 4),
                     "graph_replay_s": round(t_graph, 4)}
        out["total_amps"] = info["total_amps"]
    for c in circs:
        c.plan(4)
    t0 = time.perf_counter()
    for n, c in zip(widths, circs):
        st = qs.State(n, qs.C64)
        st.run(c)
        st.free()
    torch.cuda.synchronize()
    out["one_by_one_s"] = round(time.perf_counter() - t0, 4)
    for c in circs:
        c.free()
    return out


def bench_depth_sweep(workloads, protocol, circuits: int = 10) -> dict:
    """Fig. 3's experiment: 54 qubits on the 6x9 grid, depths 1 to 10, the
    mean fidelity estimate at the smallest p that completes (cap 2^30)."""
    t0 = time.perf_counter()
    depths = {}
    for d in range(1, 11):
        depths.update(protocol.depth_sweep(workloads.grid_circuit, 6, 9, [d], circuits))
        print(f"depth sweep: depth {d} done, {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
    return {"workload": f"54-qubit 6x9 grid, paper's family, {circuits} circuits per depth, "
                        "descending-p search, cap 2^30 amplitudes, complex64",
            "depths": depths, "wall_s": round(time.perf_counter() - t0, 1)}


def bench_heat_maps(workloads, protocol, circuits: int = 5) -> dict:
    """The appendix heat maps: mean fidelity estimate over p and depth at
    widths 25 (5x5), 36 (6x6) and 49 (7x7)."""
    t0 = time.perf_counter()
    ps = [round(0.1 * k, 3) for k in range(0, 11)]
    out = {"workload": f"paper's family on 5x5, 6x6, 7x7 grids, depths 1-14, p 0 ... 1 step 0.1, "
                       f"{circuits} circuits per cell, cap 2^30, complex64"}
    for rows in (5, 6, 7):
        F, fails = {}, {}
        for d in range(1, 15):
            r = protocol.heat_map(workloads.grid_circuit, rows, rows, [d], ps, circuits)
            F.update(r["F_mean"])
            fails.update(r["capacity_failures"])
            print(f"heat map: width {rows * rows} depth {d} done, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
        out[f"width{rows * rows}"] = {"F_mean": F, "capacity_failures": fails}
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    return out


def bench_validation(qs, workloads, protocol, circuits: int = 25) -> dict:
    """The fidelity model against the gold standard over the paper's
    validation sets (Appendix: widths x depths 6x6 ... 19x10, p from 0 to 1
    in steps of 0.025; 100 circuits per set there, `circuits` here)."""
    t0 = time.perf_counter()
    out = protocol.validation_grid(workloads.grid_circuit, circuits=circuits)
    out["workload"] = ("paper's circuit family on 2x3 ... 3x6 grids and a 19-qubit line, "
                       f"{circuits} circuits per width x depth set, 41 values of p, complex64")
    out["wall_s"] = round(time.perf_counter() - t0, 2)
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=27)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline leg")
    ap.add_argument("--quick", action="store_true",
                    help="only the QFT (skip the circuit, approximate, batch and validation runs)")
    ap.add_argument("--section", action="append", default=[],
                    choices=["qft_sizes", "sweeps", "circuit", "approx", "learned", "pairs", "qft_factorized",
                             "held", "batch",
                             "validation",
                             "depth_sweep", "heat_maps"],
                    help="run only these secondary sections (repeatable; default: all)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy one 1-GiB device buffer into another three times (the known-size "
                         "reference for the HBM byte counters) and exit")
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="library tuning knob (qs_tune_set), repeatable")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.calibrate_copy:
        src = torch.ones(2 ** 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": src.numel() * 4,
                          "bytes_written": dst.numel() * 4, "launches": 3}), flush=True)
        return 0

    import paper_2304_14969_amd as qs
    import workloads

    qs.load()
    tuning = {}
    for kv in args.tune:
        k, v = kv.split("=", 1)
        qs.tune_set(k, int(v))
        tuning[k] = int(v)
    n = args.n
    st = qs.State(n, qs.C64)
    a = workloads.gaussian_state(n, 0)
    st.set_amplitudes(a)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        st.qft()
    torch.cuda.synchronize()

    st.profile_start()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        st.qft()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = st.profile_stop()
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps

    # dominant kernel = largest total time
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    bytes_per_launch = dom["bytes"] / dom["launches"]
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    passes = sum(v["launches"] for v in prof.values()) / args.steps
    total_bytes = sum(v["bytes"] for v in prof.values()) / args.steps
    kernels = {k: {"launches_per_step": v["launches"] / args.steps,
                   "avg_ms": v["total_ms"] / v["launches"],
                   "GBps": v["bytes"] / v["launches"] / (v["total_ms"] / v["launches"] * 1e-3) / 1e9}
               for k, v in prof.items()}

    # sanity: norm preserved after all the transforms
    norm = st.norm()

    # a device-to-device copy of 1 GiB: the bandwidth a plain streaming kernel
    # reaches on this card (context for the roofline fraction)
    src = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(5):
        dst.copy_(src)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * src.numel() * 4 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst

    # gate-by-gate QFT for comparison (27 H, 351 CP, 13 relabels)
    st.set_amplitudes(a)
    gates = [g for g in _qft_gates(n)]
    for g in gates:
        qs.apply_gate(st, g)
    torch.cuda.synchronize()
    gb0 = time.perf_counter()
    for g in gates:
        qs.apply_gate(st, g)
    torch.cuda.synchronize()
    gate_by_gate_ms = (time.perf_counter() - gb0) * 1e3
    st.free()

    out = {
        "metric": METRIC,
        "value": ms_per_step / 1e3,
        "unit": "s per QFT-27",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"exact QFT on n={n} qubits, complex64 ({2 ** n * 8 / 2 ** 30:g} GiB), "
                               "i.i.d. complex Gaussian input (seed 0), state resident in HBM",
                   "n": n, "passes_per_qft": passes, "tuning": tuning},
        "hbm_GBps_effective": total_bytes / (ms_per_step * 1e-3) / 1e9,
        "hbm_copy_GBps": copy_gbps,
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "gate_by_gate_ms": gate_by_gate_ms,
        "norm_after": norm,
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": dom_name, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
                     "traffic": measured_traffic(dom_name)},
        "cpu_baseline": None,
    }
    if not args.quick:
        from paper_2304_14969_amd import protocol
        sec = {}
        want = set(args.section) or {"qft_sizes", "sweeps", "circuit", "approx", "learned", "pairs",
                                     "qft_factorized", "held", "batch", "validation"}
        if "qft_sizes" in want:
            sec["qft_sizes"] = bench_qft_sizes(qs, workloads, torch)
        if "sweeps" in want:
            sec["sweeps_n30"] = bench_sweeps(qs, np, torch)
        if "circuit" in want:
            sec["circuit_n32"] = bench_circuit(qs, workloads, torch)
        if "approx" in want:
            for fam in ("grid", "matching"):
                sec[f"approx54_{fam}"] = bench_approx(qs, workloads, protocol, np, fam)
        if "learned" in want:
            sec["learned"] = bench_learned(qs, workloads, protocol, np, torch)
        if "pairs" in want:
            sec["pair_chain54"] = bench_pairs(qs, workloads, np, torch)
        if "qft_factorized" in want:
            sec["qft_factorized"] = bench_qft_factorized(qs, workloads, np, torch)
        if "held" in want:
            sec["held"] = bench_held(qs, workloads, np, torch)
        if "batch" in want:
            sec["batch1024"] = bench_batch(qs, workloads, torch)
        if "validation" in want:
            sec["validation"] = bench_validation(qs, workloads, protocol)
        # long sweeps (minutes), only when asked for by name
        if "depth_sweep" in args.section:
            sec["depth_sweep54"] = bench_depth_sweep(workloads, protocol)
        if "heat_maps" in args.section:
            sec["heat_maps"] = bench_heat_maps(workloads, protocol)
        out["secondary"] = sec
    if not args.no_cpu:
        out["error_vs_oracle"] = error_vs_oracle(qs, workloads, n, a)
        out["cpu_baseline"] = cpu_baseline(n)
    print(json.dumps(out), flush=True)
    return 0


def _qft_gates(n):
    """QFT circuit as a gate list (H, controlled phases, SWAP relabels)."""
    out = []
    for j in range(n - 1, -1, -1):
        out.append(("h", j))
        for m in range(j - 1, -1, -1):
            out.append(("cp", m, j, math.pi / 2 ** (j - m)))
    for i in range(n // 2):
        out.append(("swap", i, n - 1 - i))
    return out


if __name__ == "__main__":
    sys.exit(main())
