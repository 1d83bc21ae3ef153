"""Autotuner: times the library's launch-shape choices on the device at hand
and keeps the fastest.

Three searches, each over the documented range of its knobs:

- `tune_qft(n)`: the QFT pass shapes (`qft.lds_bits`, `qft.high_pass`,
  `qft.threads`, `qft.round_bits`, `qft.col_max`) on an n-qubit complex64
  state; the winner is left set in the library (`qs_tune_set`).
- `tune_fusion(n, gates)`: how to run one circuit: fused blocks (block width
  kmax, matrix-core switch `fused.mfma`) or tile passes (`tile.low_bits`,
  `tile.mfma`); leaves the winning knobs set and returns the choice.
- `tune_batch(widths, circuits)`: kmax of the batched launches.

Every candidate is warmed up once and then timed `reps` times with HIP events
on the state's stream; the median decides. Nothing here changes results
beyond float32 rounding order: every knob selects between kernels that compute
the same transform.
"""
from __future__ import annotations

import itertools
import statistics

from . import C64, Batch, Circuit, State, tune_get, tune_set

QFT_KEYS = ("qft.lds_bits", "qft.high_pass", "qft.threads", "qft.round_bits", "qft.col_max")


def _time(fn, stream, reps: int) -> float:
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        b.synchronize()
        out.append(a.elapsed_time(b))
    return statistics.median(out)


def qft_candidates(n: int):
    """The pass-shape grid: contiguous tile bits (0 = the largest), strided-LDS
    or register passes above it, thread cap, in-register round width, and the
    widest strided pass (7 bits with 512-byte rows, 8 with 256-byte rows)."""
    lds = [0] + [b for b in (11, 12) if b <= n]
    return list(itertools.product(lds, (0, 1), (0, 256, 512), (4, 5), (7, 8)))


def tune_qft(n: int = 27, reps: int = 5, candidates=None) -> dict:
    """Fastest QFT pass shapes for n qubits (complex64); leaves them set."""
    before = {k: tune_get(k) for k in QFT_KEYS}
    st = State(n, C64)
    st.set_basis(1)
    results = []
    try:
        for cand in candidates or qft_candidates(n):
            for k, v in zip(QFT_KEYS, cand):
                tune_set(k, v)
            results.append((_time(st.qft, st.stream, reps), cand))
    finally:
        st.free()
    best_ms, best = min(results)
    for k, v in zip(QFT_KEYS, best):
        tune_set(k, v)
    return {"best": dict(zip(QFT_KEYS, best)), "ms": best_ms, "before": before,
            "tried": [{"ms": round(t, 4), **dict(zip(QFT_KEYS, c))} for t, c in results]}


def tune_fusion(n: int, gates, kmaxes=(3, 4, 5), tile_bits=(4, 5, 6), reps: int = 3) -> dict:
    """Fastest way to run one circuit on complex64: fused blocks (width kmax,
    with or without matrix cores) or tile passes (row bits, matrix-core or
    register rounds). Leaves the winning knobs set; returns the choice
    (`tiles` True/False, kmax) for Circuit.use_tiles / Circuit.plan."""
    st = State(n, C64)
    keys = ("fused.mfma", "tile.mfma", "tile.low_bits")
    before = {k: tune_get(k) for k in keys}
    results = []
    try:
        for mfma in (1, 0):
            tune_set("fused.mfma", mfma)
            for kmax in kmaxes:
                c = Circuit(n).add_gates(gates).plan(kmax)
                results.append((_time(lambda: st.run(c), st.stream, reps),
                                {"tiles": False, "kmax": kmax, "fused.mfma": mfma,
                                 "sweeps": c.info()["blocks"]}))
                c.free()
        tune_set("fused.mfma", before["fused.mfma"])
        if n >= 4 + 7:
            for tm in (1, 0):
                for lb in tile_bits:
                    if n < lb + 7:
                        continue
                    tune_set("tile.mfma", tm)
                    tune_set("tile.low_bits", lb)
                    c = Circuit(n).add_gates(gates).use_tiles()
                    results.append((_time(lambda: st.run(c), st.stream, reps),
                                    {"tiles": True, "tile.mfma": tm, "tile.low_bits": lb,
                                     "sweeps": c.tile_info(C64)["passes"]}))
                    c.free()
    finally:
        st.free()
        for k, v in before.items():
            tune_set(k, v)
    best_ms, best = min(results, key=lambda r: r[0])
    for k in keys:
        if k in best:
            tune_set(k, best[k])
    return {**best, "ms": best_ms, "before": before,
            "tried": [{"ms": round(t, 4), **cfg} for t, cfg in results]}


def tune_batch(widths, circuits, kmaxes=(2, 3, 4, 5), reps: int = 3) -> dict:
    """Fastest block width for batched runs of these circuits (every ket on
    blocks: tile passes off)."""
    import torch
    b = Batch(widths, C64, stream=torch.cuda.Stream())
    b.use_tiles(False)
    results = []
    try:
        for kmax in kmaxes:
            def step(k=kmax):
                b.reset()
                b.run(circuits, k)
            results.append((_time(step, b.stream, reps), kmax))
    finally:
        b.free()
    best_ms, kmax = min(results)
    return {"kmax": kmax, "ms": best_ms,
            "tried": [{"ms": round(t, 4), "kmax": k} for t, k in results]}
