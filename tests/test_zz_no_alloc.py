"""qs_amplitudes_gather_noalloc (the gather that allocates nothing, staging in
the library's fixed device array) through the C ABI, against
qs_amplitudes_gather on the same state: two calls in a row, the second with
fewer indices, on states whose qubit labels are permuted (a QFT leaves its
range bit-reversed, a SWAP relabels two more), so the index map is
exercised. Both read the same amplitudes and widen them to float64, so the
outputs must agree exactly. Sizes beyond the limit and factorized states are
refused before any device work."""
import numpy as np
import pytest

import workloads
from parity import C64, C128

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [C64, C128])
def test_gather_noalloc_matches_gather(qs_lib, dtype):
    qs = qs_lib
    n = 18
    a = workloads.gaussian_state(n, 5)
    g = np.random.default_rng(7)
    with qs.State(n, dtype) as st:
        st.set_amplitudes(a)
        st.qft()
        st.apply_swap(0, 5)
        for m in (qs.GATHER_NOALLOC_MAX, 1000):
            idx = g.integers(0, 2 ** n, m).astype(np.uint64)
            want = st.gather(idx)
            got = st.gather_noalloc(idx)
            assert got.shape == (m,)
            assert np.array_equal(got, want), m
        # an unrelabelled state: the uploaded amplitudes come back as they were
        st.set_amplitudes(a)
        idx = np.array([0, 1, 2 ** n - 1, 12345], dtype=np.uint64)
        got = st.gather_noalloc(idx)
        tol = 1e-7 if dtype == C64 else 0.0
        assert np.abs(got - a[idx.astype(np.int64)]).max() <= tol


def test_gather_noalloc_refusals(qs_lib):
    qs = qs_lib
    with qs.State(10, C64) as st:
        too_many = np.zeros(qs.GATHER_NOALLOC_MAX + 1, dtype=np.uint64)
        with pytest.raises(qs.QSError) as e:
            st.gather_noalloc(too_many)
        assert e.value.code == -1
        with pytest.raises(qs.QSError) as e:
            st.gather_noalloc(np.array([2 ** 10], dtype=np.uint64))
        assert e.value.code == -1
        assert st.gather_noalloc(np.zeros(0, dtype=np.uint64)).shape == (0,)
    st = qs.State(6, C64, factorized=True)
    try:
        with pytest.raises(qs.QSError) as e:
            st.gather_noalloc(np.array([0], dtype=np.uint64))
        assert e.value.code == -6
    finally:
        st.free()
