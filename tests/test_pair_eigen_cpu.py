"""The host step of the pair rounding (cyclic Jacobi on the real embedding of
a 4x4 Hermitian matrix, in the library) against numpy's Hermitian
eigensolver, without a GPU: the largest eigenvalue, its eigenvector up to the
documented phase, degenerate and diagonal cases, and reduced density matrices
of random states (the matrices the rounding sees)."""
import numpy as np
import pytest

from oracle import factor


@pytest.fixture(scope="module")
def qs():
    import paper_2304_14969_amd as m
    m.open_library()
    return m


def _check_top(qs, h, tol=1e-12):
    lam, phi = qs.hermitian4_top(h)
    hh = (h + h.conj().T) / 2
    w, v = np.linalg.eigh(hh)
    assert abs(lam - w[-1]) <= tol * max(1.0, abs(w[-1]))
    assert abs(np.linalg.norm(phi) - 1) < 1e-12
    np.testing.assert_allclose(hh @ phi, lam * phi, atol=1e-10 * max(1.0, np.abs(hh).max()))
    big = np.abs(phi) > 1e-9 * np.abs(phi).max()
    k = int(np.argmax(big))
    assert abs(phi[k].imag) < 1e-12 and phi[k].real > 0
    if w[-1] - w[-2] > 1e-6:  # a simple top eigenvalue: the same vector as eigh, up to phase
        assert abs(abs(np.vdot(v[:, -1], phi)) - 1) < 1e-9
    return lam, phi


@pytest.mark.parametrize("seed", range(20))
def test_random_hermitian(qs, seed):
    g = np.random.default_rng(seed)
    a = g.normal(size=(4, 4)) + 1j * g.normal(size=(4, 4))
    _check_top(qs, a + a.conj().T)


@pytest.mark.parametrize("seed", range(10))
def test_reduced_density_matrices(qs, seed):
    """The oracle's pair density of random states: the library's top
    eigenpair gives the oracle's eps_B = 1 - lambda and the same projector."""
    g = np.random.default_rng(100 + seed)
    n = 6
    a = g.normal(size=2 ** n) + 1j * g.normal(size=2 ** n)
    a /= np.linalg.norm(a)
    rho = factor.pair_density(a, n, seed % n, (seed + 2) % n)
    lam, phi = _check_top(qs, rho)
    eps, ophi = factor.pair_dominant(rho)
    assert abs((1 - lam) - eps) < 1e-12
    np.testing.assert_allclose(np.outer(phi, phi.conj()), np.outer(ophi, ophi.conj()), atol=1e-9)


def test_diagonal_degenerate_and_pure(qs):
    lam, phi = _check_top(qs, np.diag([0.1, 0.6, 0.2, 0.1]).astype(complex))
    assert abs(lam - 0.6) < 1e-15 and abs(abs(phi[1]) - 1) < 1e-12
    _check_top(qs, np.eye(4, dtype=complex) / 4)                  # fully degenerate
    v = np.array([0.5, 0.5j, -0.5, 0.5], dtype=complex)
    lam, phi = _check_top(qs, np.outer(v, v.conj()))               # pure: lambda = 1
    assert abs(lam - 1) < 1e-14


def test_bad_input(qs):
    h = np.eye(4, dtype=complex)
    h[1, 2] = np.nan
    with pytest.raises(qs.QSError):
        qs.hermitian4_top(h)
