"""The host-side C++ of the library (the C ABI's argument checks, the
circuit planner and its tile plans, the factorized-state host steps, the
batch and network drivers) built with AddressSanitizer and
UndefinedBehaviorSanitizer, and the CPU tests that reach it run against that
build in a child process with the sanitizer runtime preloaded: any invalid
memory access or undefined behaviour aborts the child. Needs no GPU."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

HOST_TESTS = ["tests/test_planner_cpu.py", "tests/test_pair_eigen_cpu.py",
              "tests/test_capi_symbols.py", "tests/test_host_calls_cpu.py"]


@pytest.fixture(scope="module")
def san_lib():
    sys.path.insert(0, ROOT)
    from paper_2304_14969_amd import build
    try:
        runtime = build.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    return build.build_sanitized(), runtime


def test_host_code_under_asan_and_ubsan(san_lib):
    lib, runtime = san_lib
    env = dict(os.environ)
    env.update(QS_LIB=lib, LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *HOST_TESTS], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-3000:] + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
