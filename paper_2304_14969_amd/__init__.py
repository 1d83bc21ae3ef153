"""Python binding of libqs.so, the MI355X state-vector simulator.

Argument marshalling only: every operation runs in the HIP kernels behind the
C ABI declared in include/qs.h. PyTorch supplies device memory (its caching
allocator, through the library's allocator hooks) and the stream on which the
library launches its work. There is no CPU fallback: if the library is not
built or no GPU is visible, `load()` raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# QS_LIB names another build of the library (the sanitized host-code build of
# the CPU tests); the default is the one next to this file.
LIB_PATH = os.environ.get("QS_LIB") or os.path.join(HERE, "libqs.so")

C64, C128 = 1, 2
GATHER_NOALLOC_MAX = 65536  # QS_GATHER_NOALLOC_MAX of qs.h
OK, E_INVAL, E_NOMEM, E_CAPACITY, E_DEVICE, E_NUMERIC, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MAX_FUSED = 6
MAX_QUBITS = 34

_ERRNAMES = {E_INVAL: "QS_E_INVAL", E_NOMEM: "QS_E_NOMEM", E_CAPACITY: "QS_E_CAPACITY",
             E_DEVICE: "QS_E_DEVICE", E_NUMERIC: "QS_E_NUMERIC", E_UNSUPPORTED: "QS_E_UNSUPPORTED"}


class QSError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class CapacityError(QSError):
    pass


_lib = None
_alloc_cb = None
_free_cb = None
_live = weakref.WeakSet()   # states and circuits to release before interpreter teardown
_closing = False


def _release_all():
    """Free every live handle while torch (the allocator behind the library's
    hooks) is still alive; later finalizers then do nothing."""
    global _closing
    for obj in list(_live):
        try:
            obj.free()
        except Exception:
            pass
    _closing = True

_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)


class Attempt(C.Structure):
    _fields_ = [("qubit", C.c_int32), ("n_sub", C.c_int32), ("eps", C.c_double),
                ("rounded", C.c_int32), ("pair", C.c_int32), ("gates", C.c_uint64)]


class TrainCfg(C.Structure):
    _fields_ = [("steps", C.c_uint32), ("batch", C.c_uint32), ("lr", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 48), ("launches", C.c_uint64), ("total_ms", C.c_double),
                ("bytes", C.c_double)]

_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)

# (name, restype, argtypes) of every exported entry point
_SIGS = [
    ("qs_last_error", C.c_char_p, []),
    ("qs_version", C.c_int, []),
    ("qs_set_allocator", C.c_int, [_ALLOC_FN, _FREE_FN, C.c_void_p]),
    ("qs_alloc", C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_void_p)]),
    ("qs_free", C.c_int, [C.c_void_p]),
    ("qs_set_stream", C.c_int, [C.c_void_p, C.c_void_p]),
    ("qs_synchronize", C.c_int, [C.c_void_p]),
    ("qs_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("qs_set_basis", C.c_int, [C.c_void_p, C.c_uint64]),
    ("qs_set_amplitudes", C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int]),
    ("qs_apply_1q", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double)]),
    ("qs_apply_ctrl", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_int, C.c_uint64, C.c_int,
                                C.POINTER(C.c_double)]),
    ("qs_apply_cphase", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double]),
    ("qs_apply_swap", C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    ("qs_apply_fused", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_double)]),
    ("qs_apply_gate", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.c_int,
                                C.POINTER(C.c_double)]),
    ("qs_qft", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int]),
    ("qs_amplitudes", C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_int]),
    ("qs_amplitudes_gather", C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.c_uint64,
                                       C.POINTER(C.c_double)]),
    ("qs_amplitudes_gather_noalloc", C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.c_uint64,
                                               C.POINTER(C.c_double)]),
    ("qs_probs", C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_uint64]),
    ("qs_norm", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("qs_check", C.c_int, [C.c_void_p, C.c_double]),
    ("qs_circuit_create", C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    ("qs_circuit_free", C.c_int, [C.c_void_p]),
    ("qs_circuit_add_gate", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
    ("qs_circuit_add_matrix", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_double)]),
    ("qs_circuit_use_tiles", C.c_int, [C.c_void_p, C.c_int]),
    ("qs_circuit_tile_info", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("qs_circuit_plan", C.c_int, [C.c_void_p, C.c_int]),
    ("qs_circuit_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("qs_circuit_block", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.POINTER(C.c_double)]),
    ("qs_run", C.c_int, [C.c_void_p, C.c_void_p]),
    ("qs_alloc_factorized", C.c_int, [C.c_int, C.c_int, C.c_uint64, C.POINTER(C.c_void_p)]),
    ("qs_set_separation_policy", C.c_int, [C.c_void_p, C.c_int, C.c_double]),
    ("qs_try_separate", C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_int)]),
    ("qs_try_separate_pair", C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double,
                                       C.POINTER(C.c_int)]),
    ("qs_shortcut_count", C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    ("qs_held_count", C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    ("qs_hermitian4_top", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("qs_mark_dirty", C.c_int, [C.c_void_p, C.c_uint64]),
    ("qs_fidelity_estimate", C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    ("qs_subsystems", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("qs_subsystem_qubits", C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("qs_set_attempt_log", C.c_int, [C.c_void_p, C.POINTER(Attempt), C.c_uint64, C.POINTER(C.c_uint64)]),
    ("qs_expand", C.c_int, [C.c_void_p, C.c_void_p]),
    ("qs_inner_product", C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("qs_batch_create", C.c_int, [C.c_int, C.POINTER(C.c_int), C.c_int, C.POINTER(C.c_void_p)]),
    ("qs_batch_free", C.c_int, [C.c_void_p]),
    ("qs_batch_set_stream", C.c_int, [C.c_void_p, C.c_void_p]),
    ("qs_batch_reset", C.c_int, [C.c_void_p]),
    ("qs_batch_run", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_int]),
    ("qs_batch_capture", C.c_int, [C.c_void_p, C.POINTER(C.c_void_p), C.c_int]),
    ("qs_batch_replay", C.c_int, [C.c_void_p]),
    ("qs_batch_use_tiles", C.c_int, [C.c_void_p, C.c_int]),
    ("qs_batch_info", C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_uint64)]),
    ("qs_batch_amplitudes", C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_uint64, C.c_int]),
    ("qs_batch_synchronize", C.c_int, [C.c_void_p]),
    ("qs_mlp_create", C.c_int, [C.POINTER(C.c_void_p)]),
    ("qs_mlp_free", C.c_int, [C.c_void_p]),
    ("qs_mlp_set_stream", C.c_int, [C.c_void_p, C.c_void_p]),
    ("qs_mlp_set_params", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_uint64]),
    ("qs_mlp_get_params", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_uint64]),
    ("qs_mlp_forward", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_uint64, C.POINTER(C.c_float)]),
    ("qs_mlp_grad", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_uint64,
                              C.POINTER(C.c_float), C.POINTER(C.c_double)]),
    ("qs_mlp_train", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_uint64,
                               C.POINTER(TrainCfg), C.POINTER(C.c_double)]),
    ("qs_set_proposer", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("qs_set_feature_log", C.c_int, [C.c_void_p, C.POINTER(C.c_float), C.c_uint64]),
    ("qs_proposer_stats", C.c_int, [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)]),
    ("qs_tune_set", C.c_int, [C.c_char_p, C.c_int64]),
    ("qs_tune_get", C.c_int, [C.c_char_p, C.POINTER(C.c_int64)]),
    ("qs_profile_start", C.c_int, [C.c_void_p]),
    ("qs_profile_stop", C.c_int, [C.c_void_p, C.POINTER(KernelStat), C.c_int, C.POINTER(C.c_int)]),
]


def exported_names() -> list:
    return [s[0] for s in _SIGS]


def open_library(path: str = LIB_PATH) -> C.CDLL:
    """dlopen libqs.so and attach prototypes (no GPU needed)."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2304_14969_amd.build.build()")
    lib = C.CDLL(path)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def hermitian4_top(h) -> tuple:
    """The pair rounding's host step (qs_hermitian4_top): the largest
    eigenvalue of the Hermitian part of a 4x4 complex matrix and its
    phase-fixed unit eigenvector. Host code only; needs the library, not a GPU."""
    lib = _lib if _lib is not None else open_library()
    hm = np.ascontiguousarray(np.asarray(h, dtype=np.complex128).reshape(4, 4))
    lam = C.c_double()
    phi = np.zeros(4, dtype=np.complex128)
    _check(lib, lib.qs_hermitian4_top(_dptr(hm.view(np.float64)), C.byref(lam),
                                      _dptr(phi.view(np.float64))))
    return lam.value, phi


def load(use_torch_allocator: bool = True) -> C.CDLL:
    """Open the library for GPU use. Raises if it is missing or no GPU is visible."""
    global _lib, _alloc_cb, _free_cb
    if _lib is not None:
        return _lib
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the simulator has no CPU path")
    # registered after torch's own exit handlers, so it runs before them
    atexit.register(_release_all)
    lib = open_library()
    if use_torch_allocator:
        def _alloc(nbytes, _user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes))
            except RuntimeError:
                return None

        def _free(ptr, _user):
            torch.cuda.caching_allocator_delete(ptr)
        _alloc_cb, _free_cb = _ALLOC_FN(_alloc), _FREE_FN(_free)
        _check(lib, lib.qs_set_allocator(_alloc_cb, _free_cb, None))
    _lib = lib
    return lib


def _check(lib, rc: int):
    if rc != OK:
        msg = lib.qs_last_error().decode(errors="replace")
        if rc == E_CAPACITY:
            raise CapacityError(rc, msg)
        raise QSError(rc, msg)


def _dptr(arr: np.ndarray):
    return arr.ctypes.data_as(C.POINTER(C.c_double))


def mat_arg(m, k: int) -> np.ndarray:
    """2^k x 2^k complex matrix -> contiguous float64 (re, im) interleaved,
    row-major; the shape is checked because the library reads 2*4^k doubles."""
    m = np.ascontiguousarray(np.asarray(m, dtype=np.complex128))
    if m.shape != (2 ** k, 2 ** k):
        raise ValueError(f"matrix of shape {m.shape} for a {k}-qubit gate")
    return np.ascontiguousarray(m.view(np.float64).reshape(-1))


GATE = {"h": 1, "x": 2, "y": 3, "z": 4, "u3": 5, "cz": 6, "iswap": 7, "cp": 8, "swap": 9,
        "cx": 10, "cy": 11, "ax": 12, "ay": 13, "az": 14, "cu3": 15}


class Circuit:
    """Host-side gate list, fused into blocks by the library's planner.
    Needs only the library, not a GPU (planning is host code)."""

    def __init__(self, n: int, lib=None):
        self.lib = lib or (_lib if _lib is not None else open_library())
        h = C.c_void_p()
        _check(self.lib, self.lib.qs_circuit_create(n, C.byref(h)))
        self.h = h
        self.n = n
        _live.add(self)

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.qs_circuit_free(self.h)
            self.h = None

    def __del__(self):
        if _closing:
            return
        try:
            self.free()
        except Exception:
            pass

    def add(self, kind: str, qubits, params=()):
        q = (C.c_int * len(qubits))(*qubits)
        p = (C.c_double * max(1, len(params)))(*params)
        _check(self.lib, self.lib.qs_circuit_add_gate(self.h, GATE[kind], q, p))

    def add_matrix(self, qubits, m):
        q = (C.c_int * len(qubits))(*qubits)
        _check(self.lib, self.lib.qs_circuit_add_matrix(self.h, q, len(qubits),
                                                        _dptr(mat_arg(m, len(qubits)))))

    def add_gates(self, gates):
        """workloads gate tuples: h, u3, cp, cz, iswap, swap, cx-type, mat, and
        ctrl with one control (a controlled U3)."""
        for g in gates:
            k = g[0]
            if k == "h":
                self.add("h", [g[1]])
            elif k == "u3":
                self.add("u3", [g[1]], g[2:5])
            elif k == "cp":
                self.add("cp", [g[1], g[2]], [g[3]])
            elif k in ("cz", "iswap", "swap", "cx", "cy", "ax", "ay", "az"):
                self.add(k, [g[1], g[2]])
            elif k == "mat":
                self.add_matrix(list(g[1]), g[2])
            elif k == "ctrl" and len(g[1]) == 1:
                # ("ctrl", [c], cval, t, theta, phi, lam): controlled U3
                self.add("cu3", [g[1][0], g[3]], [g[4], g[5], g[6], float(g[2] & 1)])
            else:
                raise ValueError(f"gate {k!r} has no circuit form")
        return self

    def plan(self, kmax: int = 0):
        _check(self.lib, self.lib.qs_circuit_plan(self.h, kmax))
        return self

    def info(self) -> dict:
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(self.lib, self.lib.qs_circuit_info(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return {"gates": a.value, "blocks": b.value, "max_k": c.value}

    def use_tiles(self, on: bool = True):
        _check(self.lib, self.lib.qs_circuit_use_tiles(self.h, int(bool(on))))
        return self

    def tile_info(self, dtype: int = C64) -> dict:
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(self.lib, self.lib.qs_circuit_tile_info(self.h, dtype, C.byref(a), C.byref(b),
                                                       C.byref(c)))
        return {"passes": a.value, "blocks": b.value, "rounds": c.value}

    def block(self, i: int):
        k = C.c_int()
        q = (C.c_int * MAX_FUSED)()
        _check(self.lib, self.lib.qs_circuit_block(self.h, i, C.byref(k), q, None))
        d = 2 ** k.value
        m = np.empty(2 * d * d, dtype=np.float64)
        _check(self.lib, self.lib.qs_circuit_block(self.h, i, C.byref(k), q, _dptr(m)))
        return list(q[:k.value]), m.view(np.complex128).reshape(d, d)


class Batch:
    """Many small kets in one device arena, run pass by pass (one launch per
    block width per pass for the whole batch)."""

    def __init__(self, widths, dtype: int = C64, stream=None):
        import torch
        self.lib = load()
        self.widths = list(widths)
        self.dtype = dtype
        arr = (C.c_int * len(self.widths))(*self.widths)
        h = C.c_void_p()
        _check(self.lib, self.lib.qs_batch_create(len(self.widths), arr, dtype, C.byref(h)))
        self.h = h
        _live.add(self)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        _check(self.lib, self.lib.qs_batch_set_stream(self.h, C.c_void_p(self.stream.cuda_stream)))

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.qs_batch_free(self.h)
            self.h = None

    def __del__(self):
        if _closing:
            return
        try:
            self.free()
        except Exception:
            pass

    def _circ_array(self, circuits):
        if len(circuits) != len(self.widths):
            raise ValueError("one circuit per ket")
        self._keep = list(circuits)
        return (C.c_void_p * len(circuits))(*[c.h.value for c in circuits])

    def reset(self):
        _check(self.lib, self.lib.qs_batch_reset(self.h))

    def run(self, circuits, kmax: int = 0):
        _check(self.lib, self.lib.qs_batch_run(self.h, self._circ_array(circuits), kmax))

    def capture(self, circuits, kmax: int = 0):
        _check(self.lib, self.lib.qs_batch_capture(self.h, self._circ_array(circuits), kmax))

    def replay(self):
        _check(self.lib, self.lib.qs_batch_replay(self.h))

    def synchronize(self):
        _check(self.lib, self.lib.qs_batch_synchronize(self.h))

    def use_tiles(self, on: bool = True):
        _check(self.lib, self.lib.qs_batch_use_tiles(self.h, int(bool(on))))
        return self

    def info(self) -> dict:
        n, t = C.c_int(), C.c_uint64()
        _check(self.lib, self.lib.qs_batch_info(self.h, C.byref(n), C.byref(t)))
        return {"launches": n.value, "total_amps": t.value}

    def amplitudes(self, i: int) -> np.ndarray:
        out = np.empty(2 ** self.widths[i], dtype=np.complex64 if self.dtype == C64 else np.complex128)
        _check(self.lib, self.lib.qs_batch_amplitudes(self.h, i, out.ctypes.data, out.size, self.dtype))
        return out


MLP_INPUTS, MLP_PARAMS = 32, 6337


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class ProposeCfg(C.Structure):
    _fields_ = [("cutoff", C.c_double), ("flags", C.c_int32), ("min_qubits", C.c_int32)]


def mlp_init(seed: int) -> np.ndarray:
    """Initial network parameters, packed W1 (32x64), b1, W2 (64x64), b2,
    W3 (64), b3: every layer's weights and biases uniform in
    +-1/sqrt(fan_in), drawn from a seeded PCG64 stream."""
    g = np.random.default_rng(seed)
    parts = []
    for fan_in, shape in ((32, (32, 64)), (32, (64,)), (64, (64, 64)), (64, (64,)),
                          (64, (64,)), (64, (1,))):
        lim = 1.0 / np.sqrt(fan_in)
        parts.append(g.uniform(-lim, lim, shape).reshape(-1))
    return np.concatenate(parts).astype(np.float32)


class MLP:
    """The separability-proposal network (parameters on the GPU)."""

    def __init__(self, params=None, stream=None):
        import torch
        self.lib = load()
        h = C.c_void_p()
        _check(self.lib, self.lib.qs_mlp_create(C.byref(h)))
        self.h = h
        _live.add(self)
        s = stream if stream is not None else torch.cuda.current_stream()
        _check(self.lib, self.lib.qs_mlp_set_stream(self.h, C.c_void_p(s.cuda_stream)))
        if params is not None:
            self.set_params(params)

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.qs_mlp_free(self.h)
            self.h = None

    def __del__(self):
        if _closing:
            return
        try:
            self.free()
        except Exception:
            pass

    def set_params(self, vec):
        v = np.ascontiguousarray(np.asarray(vec, dtype=np.float32).reshape(-1))
        if v.size != MLP_PARAMS:
            raise ValueError("wrong parameter count")
        _check(self.lib, self.lib.qs_mlp_set_params(self.h, _fptr(v), v.size))

    def get_params(self) -> np.ndarray:
        v = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(self.lib, self.lib.qs_mlp_get_params(self.h, _fptr(v), v.size))
        return v

    @staticmethod
    def _rows(X):
        X = np.ascontiguousarray(np.asarray(X, dtype=np.float32))
        if X.ndim != 2 or X.shape[1] != MLP_INPUTS:
            raise ValueError("rows of 32 features expected")
        return X

    def forward(self, X) -> np.ndarray:
        X = self._rows(X)
        out = np.empty(X.shape[0], dtype=np.float32)
        _check(self.lib, self.lib.qs_mlp_forward(self.h, _fptr(X), X.shape[0], _fptr(out)))
        return out

    def grad(self, X, y):
        X = self._rows(X)
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float32).reshape(-1))
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = C.c_double()
        _check(self.lib, self.lib.qs_mlp_grad(self.h, _fptr(X), _fptr(y), X.shape[0], _fptr(g),
                                              C.byref(loss)))
        return g, loss.value

    def train(self, X, y, steps: int, batch: int = 256, lr: float = 1e-3, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8) -> float:
        X = self._rows(X)
        y = np.ascontiguousarray(np.asarray(y, dtype=np.float32).reshape(-1))
        cfg = TrainCfg(steps, batch, lr, beta1, beta2, eps)
        loss = C.c_double()
        _check(self.lib, self.lib.qs_mlp_train(self.h, _fptr(X), _fptr(y), X.shape[0], C.byref(cfg),
                                               C.byref(loss)))
        return loss.value


def tune_set(key: str, value: int):
    lib = load()
    _check(lib, lib.qs_tune_set(key.encode(), int(value)))


def tune_get(key: str) -> int:
    lib = load()
    v = C.c_int64()
    _check(lib, lib.qs_tune_get(key.encode(), C.byref(v)))
    return v.value


SEP_NONE, SEP_AFTER_2Q, SEP_AFTER_2Q_PAIRS = 0, 1, 2
PROPOSE_RETEST_ON_MERGE = 1


class State:
    """An n-qubit ket on the GPU (owned by the library): dense by default,
    factorized (approximate mode) when max_amps is given."""

    def __init__(self, n: int, dtype: int = C64, stream=None, factorized: bool = False,
                 max_amps: int = 2 ** 30):
        self.lib = load()
        h = C.c_void_p()
        if factorized:
            _check(self.lib, self.lib.qs_alloc_factorized(n, dtype, int(max_amps), C.byref(h)))
        else:
            _check(self.lib, self.lib.qs_alloc(n, dtype, C.byref(h)))
        self.factorized = factorized
        self._log = None
        self.h = h
        self.n = n
        self.dtype = dtype
        _live.add(self)
        self.set_stream(stream)

    # -- lifecycle
    def set_stream(self, stream=None):
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        _check(self.lib, self.lib.qs_set_stream(self.h, C.c_void_p(s.cuda_stream)))

    def free(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _check(self.lib, self.lib.qs_free(self.h))
            self.h = None

    def __del__(self):
        if _closing:
            return
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.free()

    def synchronize(self):
        _check(self.lib, self.lib.qs_synchronize(self.h))

    # -- initial states
    def set_basis(self, x: int):
        _check(self.lib, self.lib.qs_set_basis(self.h, int(x)))

    def set_amplitudes(self, a: np.ndarray):
        a = np.ascontiguousarray(a)
        if a.dtype == np.complex128:
            dt = C128
        elif a.dtype == np.complex64:
            dt = C64
        else:
            raise TypeError("amplitudes must be complex64 or complex128")
        _check(self.lib, self.lib.qs_set_amplitudes(self.h, a.ctypes.data, a.size, dt))

    # -- gates
    def apply_1q(self, q: int, m):
        _check(self.lib, self.lib.qs_apply_1q(self.h, q, _dptr(mat_arg(m, 1))))

    def apply_ctrl(self, ctrls, cvals: int, target: int, m):
        c = (C.c_int * len(ctrls))(*ctrls)
        _check(self.lib, self.lib.qs_apply_ctrl(self.h, c, len(ctrls), int(cvals), target,
                                                _dptr(mat_arg(m, 1))))

    def apply_cphase(self, a: int, b: int, theta: float):
        _check(self.lib, self.lib.qs_apply_cphase(self.h, a, b, float(theta)))

    def apply_swap(self, a: int, b: int):
        _check(self.lib, self.lib.qs_apply_swap(self.h, a, b))

    def apply_fused(self, qubits, m):
        qs = (C.c_int * len(qubits))(*qubits)
        _check(self.lib, self.lib.qs_apply_fused(self.h, qs, len(qubits),
                                                 _dptr(mat_arg(m, len(qubits)))))

    def run(self, circ: "Circuit"):
        _check(self.lib, self.lib.qs_run(self.h, circ.h))

    def qft(self, start: int = 0, length: int | None = None, inverse: bool = False):
        length = self.n - start if length is None else length
        _check(self.lib, self.lib.qs_qft(self.h, start, length, int(bool(inverse))))

    # -- readout
    def amplitudes(self, dtype=np.complex128) -> np.ndarray:
        out = np.empty(2 ** self.n, dtype=dtype)
        dt = C128 if out.dtype == np.complex128 else C64
        _check(self.lib, self.lib.qs_amplitudes(self.h, out.ctypes.data, out.size, dt))
        return out

    def gather(self, idx) -> np.ndarray:
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
        out = np.empty(idx.size, dtype=np.complex128)
        _check(self.lib, self.lib.qs_amplitudes_gather(
            self.h, idx.ctypes.data_as(C.POINTER(C.c_uint64)), idx.size,
            out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def gather_noalloc(self, idx) -> np.ndarray:
        """qs_amplitudes_gather_noalloc: at most GATHER_NOALLOC_MAX indices,
        dense states, no device allocation."""
        idx = np.ascontiguousarray(np.asarray(idx, dtype=np.uint64))
        out = np.empty(idx.size, dtype=np.complex128)
        _check(self.lib, self.lib.qs_amplitudes_gather_noalloc(
            self.h, idx.ctypes.data_as(C.POINTER(C.c_uint64)), idx.size,
            out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def probs(self) -> np.ndarray:
        out = np.empty(2 ** self.n, dtype=np.float64)
        _check(self.lib, self.lib.qs_probs(self.h, _dptr(out), out.size))
        return out

    def norm(self) -> float:
        v = C.c_double()
        _check(self.lib, self.lib.qs_norm(self.h, C.byref(v)))
        return v.value

    def check(self, tol: float):
        _check(self.lib, self.lib.qs_check(self.h, float(tol)))

    # -- approximate mode
    def set_policy(self, policy: int, p: float):
        _check(self.lib, self.lib.qs_set_separation_policy(self.h, policy, float(p)))

    def try_separate(self, p: float) -> int:
        k = C.c_int()
        _check(self.lib, self.lib.qs_try_separate(self.h, float(p), C.byref(k)))
        return k.value

    def try_separate_pair(self, qa: int, qb: int, p: float) -> bool:
        """The two-qubit rounding of (qa, qb); True if the pair was split off."""
        r = C.c_int()
        _check(self.lib, self.lib.qs_try_separate_pair(self.h, int(qa), int(qb), float(p),
                                                       C.byref(r)))
        return bool(r.value)

    def shortcut_count(self) -> int:
        """Operands dropped by the Z-eigenstate shortcut so far."""
        v = C.c_uint64()
        _check(self.lib, self.lib.qs_shortcut_count(self.h, C.byref(v)))
        return v.value

    def held_count(self):
        """(gates held back between subsystems, those of them that never
        caused a merge of their own) so far."""
        a, b = C.c_uint64(), C.c_uint64()
        _check(self.lib, self.lib.qs_held_count(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def mark_dirty(self, mask: int):
        _check(self.lib, self.lib.qs_mark_dirty(self.h, int(mask)))

    def fidelity_estimate(self) -> float:
        v = C.c_double()
        _check(self.lib, self.lib.qs_fidelity_estimate(self.h, C.byref(v)))
        return v.value

    def subsystems(self) -> list:
        """Qubit lists of the subsystems, in bit order."""
        ns = C.c_int()
        _check(self.lib, self.lib.qs_subsystems(self.h, None, None, C.byref(ns)))
        out = []
        for s in range(ns.value):
            q = (C.c_int * 64)()
            nq = C.c_int()
            _check(self.lib, self.lib.qs_subsystem_qubits(self.h, s, q, C.byref(nq)))
            out.append(list(q[:nq.value]))
        return out

    def record_attempts(self, cap: int = 1 << 20):
        """Start recording separability attempts into a buffer owned here."""
        self._log = (Attempt * cap)()
        self._log_count = C.c_uint64()
        _check(self.lib, self.lib.qs_set_attempt_log(self.h, self._log, cap, C.byref(self._log_count)))

    def attempts(self) -> list:
        n = min(self._log_count.value, len(self._log)) if self._log is not None else 0
        # one-qubit attempts: (qubit, n_sub, eps, rounded); two-qubit ones
        # (the pair rounding) carry the second qubit as a fifth entry
        return [(a.qubit, a.n_sub, a.eps, bool(a.rounded)) if a.pair == 0 else
                (a.qubit, a.n_sub, a.eps, bool(a.rounded), a.pair - 1) for a in self._log[:n]]

    def attempt_gates(self) -> list:
        """For each attempt of attempts(): the number of multi-qubit gates
        applied before it (where in the circuit the test looked at the state)."""
        n = min(self._log_count.value, len(self._log)) if self._log is not None else 0
        return [int(a.gates) for a in self._log[:n]]

    def record_features(self, cap: int = 1 << 20):
        """Record the 32 proposal features of every attempt (call after
        record_attempts; rows align with attempts())."""
        self._feat = np.zeros((cap, MLP_INPUTS), dtype=np.float32)
        _check(self.lib, self.lib.qs_set_feature_log(self.h, _fptr(self._feat), cap))

    def features(self) -> np.ndarray:
        n = min(self._log_count.value, len(self._feat))
        return self._feat[:n].copy()

    def set_proposer(self, net: "MLP | None", cutoff: float = 0.5, retest_on_merge: bool = True,
                     min_qubits: int = 2):
        self._proposer = net
        cfg = ProposeCfg(float(cutoff), PROPOSE_RETEST_ON_MERGE if retest_on_merge else 0,
                         int(min_qubits))
        _check(self.lib, self.lib.qs_set_proposer(self.h, net.h if net is not None else None,
                                                  C.byref(cfg)))

    def proposer_stats(self) -> dict:
        a, b = C.c_uint64(), C.c_uint64()
        _check(self.lib, self.lib.qs_proposer_stats(self.h, C.byref(a), C.byref(b)))
        return {"skipped": a.value, "fallback_tests": b.value}

    def expand_into(self, dense: "State"):
        _check(self.lib, self.lib.qs_expand(self.h, dense.h))

    def inner(self, other: "State") -> complex:
        re, im = C.c_double(), C.c_double()
        _check(self.lib, self.lib.qs_inner_product(self.h, other.h, C.byref(re), C.byref(im)))
        return complex(re.value, im.value)

    # -- timing
    def profile_start(self):
        _check(self.lib, self.lib.qs_profile_start(self.h))

    def profile_stop(self) -> dict:
        """{kernel: {"launches", "total_ms", "bytes"}} since profile_start."""
        buf = (KernelStat * 64)()
        cnt = C.c_int()
        _check(self.lib, self.lib.qs_profile_stop(self.h, buf, 64, C.byref(cnt)))
        return {buf[i].name.decode(): {"launches": int(buf[i].launches),
                                       "total_ms": float(buf[i].total_ms),
                                       "bytes": float(buf[i].bytes)} for i in range(cnt.value)}


# ------------------------------------------------------------------ gate lists


def apply_gate(st: State, g):
    """Dispatch one gate tuple (the workloads gate-list format) to the
    library; every matrix is built in the library (qs_apply_gate), except the
    explicit ones of "mat" tuples."""
    k = g[0]
    if k == "mat":
        st.apply_fused(list(g[1]), g[2])
        return
    if k == "ctrl":
        qubits = list(g[1]) + [g[3]]
        params = [g[4], g[5], g[6], float(g[2] & ((1 << len(g[1])) - 1))]
        kind = GATE["cu3"]
    elif k in ("h", "x", "y", "z"):
        qubits, params, kind = [g[1]], [], GATE[k]
    elif k == "u3":
        qubits, params, kind = [g[1]], list(g[2:5]), GATE[k]
    elif k == "cp":
        qubits, params, kind = [g[1], g[2]], [g[3]], GATE[k]
    elif k in GATE:
        qubits, params, kind = [g[1], g[2]], [], GATE[k]
    else:
        raise ValueError(f"unknown gate {k!r}")
    q = (C.c_int * len(qubits))(*qubits)
    p = (C.c_double * max(1, len(params)))(*params)
    _check(st.lib, st.lib.qs_apply_gate(st.h, kind, q, len(qubits), p))


def run_gates(st: State, gates):
    for g in gates:
        apply_gate(st, g)
