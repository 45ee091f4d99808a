"""The oracle's pins have teeth: plausible mistakes, planted in copies of
oracle functions on the CPU, must make the corresponding pin fail."""
import numpy as np
import scipy.linalg
from numpy.polynomial import chebyshev as npcheb

from oracle import chebyshev, eigh
from workloads import gen


def _cheb_np(m, t):
    coef = np.zeros(m + 1)
    coef[m] = 1.0
    return npcheb.chebval(t, coef)


def _filter_pin_holds(filt):
    n = 40
    lam = np.sort(np.random.default_rng(11).uniform(-3, 4, n))
    q = gen._NumpyBackend().qr_unitary(gen.random_block(n, n, 12))
    h = (q * lam) @ q.conj().T
    deg = [2, 5, 5, 9]
    y0 = gen.random_block(n, 4, 5)
    c, e, gamma = 2.0, 2.0, -3.2
    got = filt(h, y0, deg, c, e, gamma)
    for j, m in enumerate(deg):
        col = q @ ((_cheb_np(m, (lam - c) / e) / _cheb_np(m, (gamma - c) / e))
                   * (q.conj().T @ y0[:, j]))
        if np.linalg.norm(got[:, j] - col) > 1e-12 * np.linalg.norm(col):
            return False
    return True


def _filter_variant(y_old_is_current=False, shift_sign=1.0, sigma_index_shift=0):
    """A copy of the oracle's per-column recurrence with one planted
    mistake: the subtracted term taken from Y_i instead of Y_{i-1}, the
    shift added instead of subtracted, or the sigmas used one step late."""
    def filt(h, y0, m, c, e, gamma):
        sig = chebyshev.sigmas(max(m) + 1, c, e, gamma)
        out = np.empty_like(y0)
        for j, mj in enumerate(m):
            prev = y0[:, j].copy()
            cur = (sig[0] / e) * (h @ prev - shift_sign * c * prev)
            for i in range(1, mj):
                s_new = sig[i + sigma_index_shift]
                s_old = sig[i - 1 + sigma_index_shift]
                old = cur if y_old_is_current else prev
                nxt = (2 * s_new / e) * (h @ cur - shift_sign * c * cur) - s_new * s_old * old
                prev, cur = cur, nxt
            out[:, j] = cur
        return out
    return filt


def test_filter_pin_accepts_oracle_and_a_faithful_copy():
    assert _filter_pin_holds(chebyshev.chebyshev_filter)
    assert _filter_pin_holds(_filter_variant())


def test_filter_pin_catches_wrong_term_sign_and_sigma_index():
    assert not _filter_pin_holds(_filter_variant(y_old_is_current=True))
    assert not _filter_pin_holds(_filter_variant(shift_sign=-1.0))
    assert not _filter_pin_holds(_filter_variant(sigma_index_shift=1))


def test_reduction_pin_catches_plain_transpose():
    n = 24
    lam = np.linspace(-2, 5, n)
    m = gen.prescribed_problem(n, lam, 2)
    b = gen.random_hpd(n, 4, weight=0.5)
    l = np.linalg.cholesky(b)
    a = l @ m @ l.conj().T
    w = scipy.linalg.solve_triangular(l, a, lower=True)
    wrong = scipy.linalg.solve_triangular(l, w.T, lower=True).T     # L^-1 A L^-T
    wrong = 0.5 * (wrong + wrong.conj().T)
    assert np.abs(eigh.eigvalsh(wrong) - lam).max() > 1e-3


def test_eigh_pin_catches_dropped_phase_correction():
    n = 30
    lam = np.sort(np.random.default_rng(1).uniform(-5, 5, n))
    a = gen.prescribed_problem(n, lam, 8)
    d, e, _, _ = eigh.householder_tridiagonal(a)
    w_bad, _ = eigh.tridiagonal_qr(d, e.real)      # phases ignored
    w_ok, _ = eigh.tridiagonal_qr(d, np.abs(e))
    assert np.abs(np.sort(w_ok) - lam).max() < 1e-12
    assert np.abs(np.sort(w_bad) - lam).max() > 1e-6
