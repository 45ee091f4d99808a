"""Pins for the oracle's Chebyshev machinery (Sec. 3.1.1, Alg. 2).

Every expected value here comes from somewhere other than the oracle:
numpy's Chebyshev-series evaluator, the growth formula printed in
Sec. 3.1.1, the spectral closed form of a polynomial of a Hermitian
matrix, or an identity derived from the recurrence."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

from oracle import chebyshev
from workloads import gen


def _cheb_np(m, t):
    coef = np.zeros(m + 1)
    coef[m] = 1.0
    return npcheb.chebval(t, coef)


@pytest.mark.parametrize("m", [0, 1, 2, 3, 7, 10, 25, 40])
def test_closed_form_matches_series(m):
    t = np.linspace(-2.5, 2.5, 101)
    ref = _cheb_np(m, t)
    got = chebyshev.cheb(m, t)
    assert np.allclose(got, ref, rtol=1e-11, atol=1e-11)


def test_growth_formula_outside_interval():
    # Sec. 3.1.1: C_m(t) = (|rho|^m + |rho|^-m)/2 for t > 1 (and |C_m| for t < -1)
    for t in [1.01, 1.3, 2.0, 5.0, -1.2, -3.0]:
        r = chebyshev.rho(np.array([t]))[0]
        for m in [1, 4, 9, 20]:
            assert abs(abs(_cheb_np(m, t)) - 0.5 * (r ** m + r ** -m)) <= 1e-10 * abs(_cheb_np(m, t))


def test_rho_is_one_inside_and_limit_outside():
    assert np.all(chebyshev.rho(np.linspace(-1, 1, 11)) == 1.0)
    t = 1.7
    r = chebyshev.rho(np.array([t]))[0]
    assert abs((2 * abs(_cheb_np(200, t))) ** (1 / 200) - r) < 1e-12 * r


def test_sigma_recursion_is_ratio_of_chebyshev_values():
    c, e, gamma = 3.0, 4.0, -2.5
    tg = (gamma - c) / e
    s = chebyshev.sigmas(30, c, e, gamma)
    for i in range(1, 31):
        assert abs(s[i - 1] - _cheb_np(i - 1, tg) / _cheb_np(i, tg)) < 1e-13 * abs(s[i - 1])


def _herm(n, seed, lo=-3.0, hi=4.0):
    g = np.random.default_rng(seed)
    lam = np.sort(g.uniform(lo, hi, n))
    q = gen._NumpyBackend().qr_unitary(gen.random_block(n, n, seed + 1))
    return lam, q, (q * lam) @ q.conj().T


@pytest.mark.parametrize("degrees", [[1], [4, 4, 4], [1, 2, 2, 5, 9, 9, 13], [3, 7, 7, 8]])
def test_filter_matches_spectral_closed_form(degrees):
    lam, q, h = _herm(48, 11)
    y0 = gen.random_block(48, len(degrees), 5)
    c, e, gamma = 2.0, 2.0, -3.2
    got = chebyshev.chebyshev_filter(h, y0, degrees, c, e, gamma)
    t = (lam - c) / e
    tg = (gamma - c) / e
    for j, m in enumerate(degrees):
        col = q @ ((_cheb_np(m, t) / _cheb_np(m, tg)) * (q.conj().T @ y0[:, j]))
        assert np.linalg.norm(got[:, j] - col) <= 1e-12 * np.linalg.norm(col)


def test_variable_degree_equals_per_column_uniform_filter():
    lam, q, h = _herm(40, 3)
    y0 = gen.random_block(40, 5, 9)
    deg = [2, 3, 3, 6, 8]
    c, e, gamma = 1.0, 3.0, -3.5
    got = chebyshev.chebyshev_filter(h, y0, deg, c, e, gamma)
    for j, m in enumerate(deg):
        one = chebyshev.chebyshev_filter(h, y0[:, j:j + 1], [m], c, e, gamma)
        assert np.allclose(got[:, j], one[:, 0], rtol=1e-13, atol=1e-13 * np.abs(one).max())


def test_filter_on_diagonal_matrix():
    d = np.linspace(-5, 5, 30)
    h = np.diag(d).astype(complex)
    y0 = np.eye(30, 3, dtype=complex) + 0.5
    c, e, gamma = 1.0, 4.0, -5.0
    got = chebyshev.chebyshev_filter(h, y0, [6, 6, 6], c, e, gamma)
    scale = _cheb_np(6, (d - c) / e) / _cheb_np(6, (gamma - c) / e)
    assert np.allclose(got, scale[:, None] * y0, rtol=1e-12, atol=1e-12)


def test_gamma_only_rescales_columns():
    lam, q, h = _herm(32, 8)
    y0 = gen.random_block(32, 3, 1)
    deg = [3, 5, 9]
    c, e = 2.0, 2.5
    y1 = chebyshev.chebyshev_filter(h, y0, deg, c, e, -3.0)
    y2 = chebyshev.chebyshev_filter(h, y0, deg, c, e, -4.0)
    for j, m in enumerate(deg):
        f = _cheb_np(m, (-3.0 - c) / e) / _cheb_np(m, (-4.0 - c) / e)
        assert np.allclose(y2[:, j], y1[:, j] * f, rtol=1e-12, atol=1e-14)


def test_filter_rejects_zero_degrees():
    h = np.eye(4, dtype=complex)
    y = np.ones((4, 2), dtype=complex)
    with pytest.raises(ValueError):
        chebyshev.chebyshev_filter(h, y, [0, 2], 0.0, 1.0, -2.0)


def test_filter_is_independent_of_column_order():
    # the definition is per column: any order of the degrees gives the same
    # columns (Alg. 2 sorts them only to keep the active ones contiguous)
    lam, q, h = _herm(36, 4)
    deg = [7, 1, 4, 4, 2, 9]
    y0 = gen.random_block(36, len(deg), 13)
    c, e, gamma = 1.5, 2.5, -3.4
    got = chebyshev.chebyshev_filter(h, y0, deg, c, e, gamma)
    perm = np.argsort(deg, kind="stable")
    srt = chebyshev.chebyshev_filter(h, y0[:, perm], [deg[p] for p in perm], c, e, gamma)
    assert np.allclose(got[:, perm], srt, rtol=1e-13, atol=1e-13 * np.abs(srt).max())
    t, tg = (lam - c) / e, (gamma - c) / e
    for j, m in enumerate(deg):
        col = q @ ((_cheb_np(m, t) / _cheb_np(m, tg)) * (q.conj().T @ y0[:, j]))
        assert np.linalg.norm(got[:, j] - col) <= 1e-12 * np.linalg.norm(col)


def test_filter_of_an_empty_block():
    h = np.eye(5, dtype=complex)
    assert chebyshev.chebyshev_filter(h, np.zeros((5, 0), complex), [], 0.0, 1.0, -2.0).shape \
        == (5, 0)


def test_filter_damps_interval_and_amplifies_below():
    lam, q, h = _herm(60, 21, lo=-6.0, hi=6.0)
    alpha, beta = 0.0, 6.0
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    y0 = q[:, [0, 59]]           # lowest and highest eigenvector
    y = chebyshev.chebyshev_filter(h, y0, [12, 12], c, e, lam[0])
    # the lowest eigenvector keeps unit size (p_m(gamma) = 1), the top one shrinks
    assert abs(np.linalg.norm(y[:, 0]) - 1.0) < 1e-10
    assert np.linalg.norm(y[:, 1]) < 1e-3
