"""Parity bars between the HIP path and the FP64 oracle.

complex64 runs: max |a_gpu - a_oracle| <= 1e-5 and 1 - |<gpu|oracle>|^2 <= 1e-6
(the tolerance stated for FP32 exact runs). complex128 runs: 1e-12 on both.
The relative error max|d| / max|a| is also reported, because at n = 27 a
typical amplitude is ~8.6e-5 and the absolute bound alone is loose.
"""
import numpy as np

C64, C128 = 1, 2
TOL = {C64: (1e-5, 1e-6), C128: (1e-12, 1e-12)}


def compare(got, want, dtype):
    got = np.asarray(got, dtype=np.complex128)
    want = np.asarray(want, dtype=np.complex128)
    d = np.abs(got - want)
    max_abs = float(d.max()) if d.size else 0.0
    infid = 1.0 - abs(np.vdot(got, want)) ** 2 / (np.vdot(got, got).real * np.vdot(want, want).real)
    rel = max_abs / float(np.abs(want).max()) if d.size else 0.0
    return {"max_abs": max_abs, "infidelity": float(infid), "max_rel": rel}


def assert_parity(got, want, dtype, what=""):
    r = compare(got, want, dtype)
    amax, fmax = TOL[dtype]
    assert r["max_abs"] <= amax, f"{what}: max |d| = {r['max_abs']:.3e} > {amax} ({r})"
    assert r["infidelity"] <= fmax, f"{what}: 1-F = {r['infidelity']:.3e} > {fmax} ({r})"
    return r
