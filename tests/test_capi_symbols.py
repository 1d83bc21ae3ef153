"""The C-ABI library loads without a GPU and exports every entry point that
include/qs.h declares (no compute calls here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def declared_functions():
    names = []
    for fn in sorted(os.listdir(HEADER_DIR)):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(qs_\w+)\s*\(", text, flags=re.M):
            if "typedef" in text[text.rfind("\n", 0, m.start()) + 1:m.start() + 1]:
                continue
            names.append(m.group(1))
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    import paper_2304_14969_amd as qs
    if not os.path.exists(qs.LIB_PATH):
        pytest.fail("libqs.so is not built (run __graft_entry__.build())")
    return qs.open_library()


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("qs_alloc", "qs_free", "qs_apply_1q", "qs_apply_ctrl", "qs_apply_fused",
                 "qs_qft", "qs_amplitudes", "qs_probs", "qs_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header(lib):
    import paper_2304_14969_amd as qs
    assert set(declared_functions()) <= set(qs.exported_names())


def test_error_paths_without_gpu(lib):
    """Argument checks happen before any device work."""
    h = ctypes.c_void_p()
    assert lib.qs_alloc(0, 1, ctypes.byref(h)) == -1
    assert b"outside" in lib.qs_last_error()
    assert lib.qs_alloc(5, 7, ctypes.byref(h)) == -1
    assert lib.qs_alloc(5, 1, None) == -1
    assert lib.qs_apply_swap(None, 0, 1) == -1
    assert lib.qs_free(None) == 0
    assert lib.qs_version() >= 100
