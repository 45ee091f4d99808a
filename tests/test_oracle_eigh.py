"""Pins for the oracle's dense Hermitian eigensolver.

Expected values come from prescribed spectra (A = Q diag(lam) Q^H), the
closed form of tridiag(-1, 2, -1), the 2x2 closed form, an independent
cyclic Jacobi solver written in this file, and numpy's LAPACK eigvalsh
(tests only; the oracle never calls it)."""
import math

import numpy as np
import pytest

from oracle import eigh
from workloads import gen

EPS = np.finfo(float).eps


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 33, 90])
def test_prescribed_spectrum(n):
    lam = np.sort(np.random.default_rng(n).uniform(-10, 10, n))
    a = gen.prescribed_problem(n, lam, 100 + n)
    w, v = eigh.eigh(a)
    nrm = np.abs(lam).max()
    assert np.abs(w - lam).max() <= 50 * n * EPS * nrm
    assert np.abs(a @ v - v * w).max() <= 50 * n * EPS * nrm
    assert np.abs(v.conj().T @ v - np.eye(n)).max() <= 50 * n * EPS


def test_tridiagonal_closed_form_real_and_complex_phases():
    n = 60
    exact = 2.0 - 2.0 * np.cos(np.arange(1, n + 1) * math.pi / (n + 1))
    w, _ = eigh.tridiagonal_qr(np.full(n, 2.0), np.full(n - 1, 1.0))   # same spectrum as -1
    assert np.abs(np.sort(w) - exact).max() < 1e-13
    ph = np.exp(1j * np.random.default_rng(0).uniform(0, 2 * math.pi, n - 1))
    a = np.diag(np.full(n, 2.0 + 0j)) - np.diag(ph, -1) - np.diag(ph.conj(), 1)
    w2, v2 = eigh.eigh(a)
    assert np.abs(w2 - exact).max() < 1e-13
    assert np.abs(a @ v2 - v2 * w2).max() < 1e-13


def test_two_by_two_closed_form():
    a, d, b = 1.3, -0.4, 0.7 - 0.2j
    m = np.array([[a, b], [np.conj(b), d]])
    r = math.sqrt(((a - d) / 2) ** 2 + abs(b) ** 2)
    w, _ = eigh.eigh(m)
    assert np.allclose(w, [(a + d) / 2 - r, (a + d) / 2 + r], rtol=0, atol=1e-15)


def _jacobi_real_symmetric(s, sweeps=30):
    """Cyclic Jacobi eigenvalue iteration (Golub & Van Loan Sec. 8.5)."""
    s = s.copy()
    n = s.shape[0]
    for _ in range(sweeps):
        off = np.sqrt((s ** 2).sum() - (np.diag(s) ** 2).sum())
        if off < 1e-15 * np.abs(s).max():
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                if s[p, q] == 0.0:
                    continue
                tau = (s[q, q] - s[p, p]) / (2 * s[p, q])
                t = math.copysign(1.0, tau) / (abs(tau) + math.sqrt(1 + tau * tau))
                c = 1 / math.sqrt(1 + t * t)
                sn = t * c
                j = np.eye(n)
                j[p, p] = j[q, q] = c
                j[p, q], j[q, p] = sn, -sn
                s = j.T @ s @ j
    return np.sort(np.diag(s))


def test_jacobi_cross_check_via_real_embedding():
    n = 12
    g = gen.random_block(n, n, 4)
    a = 0.5 * (g + g.conj().T)
    emb = np.block([[a.real, -a.imag], [a.imag, a.real]])   # eigenvalues of a, each twice
    ref = _jacobi_real_symmetric(emb)[::2]
    w = eigh.eigvalsh(a)
    assert np.abs(w - ref).max() < 1e-12


def test_against_lapack_random_hermitian():
    for n in [7, 40, 120]:
        g = gen.random_block(n, n, n)
        a = 0.5 * (g + g.conj().T)
        w, v = eigh.eigh(a)
        ref = np.linalg.eigvalsh(a)
        assert np.abs(w - ref).max() <= 20 * n * EPS * np.abs(ref).max()
        assert np.abs(v.conj().T @ v - np.eye(n)).max() <= 20 * n * EPS


def test_repeated_eigenvalues_and_diagonal_input():
    lam = np.array([1.0, 1.0, 1.0, 2.0, 2.0, 5.0])
    a = gen.prescribed_problem(6, lam, 3)
    w, v = eigh.eigh(a)
    assert np.abs(w - lam).max() < 1e-13
    assert np.abs(v.conj().T @ v - np.eye(6)).max() < 1e-13
    d = np.array([3.0, -1.0, 2.0, 0.0])
    w, v = eigh.eigh(np.diag(d).astype(complex))
    assert np.array_equal(w, np.sort(d))
    assert np.abs(np.diag(d) @ v - v * w).max() < 1e-15
