"""Pins for the oracle's ChFSI loop (Alg. 1) and its steps.

Expected values: prescribed spectra, generalized pencils with known
eigenvalues, textbook theorems (Rayleigh-Ritz exactness when the subspace
is the whole space, Cauchy interlacing, Lanczos Ritz values inside the
spectrum), the published SplitMix64 output sequence, the defining
inequality of the degree rule, and the paper's directional claims (warm
start beats random start; per-vector degrees beat a fixed degree)."""
import math

import numpy as np
import pytest

from oracle import chebyshev, chfsi, counter_rng, eigh
from workloads import gen


def test_splitmix64_reference_outputs():
    # first outputs of SplitMix64 seeded with 0 (published reference values)
    got = [int(x) for x in counter_rng.raw(0, 0, 4)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


def test_counter_block_layout_and_range():
    z = counter_rng.complex_block(7, 1, 5, 3)
    u = counter_rng.uniform(7, 1, 30) - 0.5
    assert z.shape == (5, 3)
    assert z[2, 1] == complex(u[2 * (2 + 5)], u[2 * (2 + 5) + 1])
    assert np.all(np.abs(z.real) <= 0.5) and np.all(np.abs(z.imag) <= 0.5)


def test_lanczos_bounds_bracket_the_spectrum():
    lam = np.sort(np.random.default_rng(2).normal(0, 10, 300))
    a = gen.prescribed_problem(300, lam, 5)
    v0 = counter_rng.complex_block(0, 0, 300, 1)
    upper, tmin, tmax = chfsi.lanczos_bounds(a, 20, v0)
    assert upper >= lam[-1]
    assert lam[0] <= tmin and tmax <= lam[-1]
    assert upper - lam[-1] < 0.5 * (lam[-1] - lam[0])


def test_lanczos_exact_on_small_invariant_space():
    lam = np.array([-2.0, 0.5, 3.0, 7.0])
    a = gen.prescribed_problem(4, lam, 1)
    upper, tmin, tmax = chfsi.lanczos_bounds(a, 20, counter_rng.complex_block(1, 0, 4, 1))
    assert abs(tmin - lam[0]) < 1e-12 and abs(tmax - lam[-1]) < 1e-12
    assert upper >= lam[-1] - 1e-12


def test_rayleigh_ritz_exact_when_subspace_is_whole_space():
    lam = np.sort(np.random.default_rng(3).uniform(-4, 4, 25))
    a = gen.prescribed_problem(25, lam, 9)
    q = chfsi.orthonormalize(gen.random_block(25, 25, 1), np.zeros((25, 0), complex))
    mu, qw, zw = chfsi.rayleigh_ritz(a, q)
    assert np.abs(mu - lam).max() < 1e-12
    assert chfsi.residual_norms(qw, zw, mu).max() < 1e-12


def test_rayleigh_ritz_interlacing():
    lam = np.sort(np.random.default_rng(4).uniform(-4, 4, 80))
    a = gen.prescribed_problem(80, lam, 10)
    q = chfsi.orthonormalize(gen.random_block(80, 12, 2), np.zeros((80, 0), complex))
    mu, qw, zw = chfsi.rayleigh_ritz(a, q)
    k = 12
    assert np.all(mu >= lam[:k] - 1e-12)
    assert np.all(mu <= lam[80 - k:] + 1e-12)
    # residuals agree with the definition ||A q - mu q||
    direct = np.linalg.norm(a @ qw - qw * mu, axis=0)
    assert np.allclose(chfsi.residual_norms(qw, zw, mu), direct, rtol=1e-10, atol=1e-13)


def test_orthonormalize_against_locked_vectors():
    n = 50
    ql = chfsi.orthonormalize(gen.random_block(n, 4, 3), np.zeros((n, 0), complex))
    y = gen.random_block(n, 6, 4)
    q = chfsi.orthonormalize(y, ql)
    assert np.abs(q.conj().T @ q - np.eye(6)).max() < 1e-14
    assert np.abs(ql.conj().T @ q).max() < 1e-14
    yp = y - ql @ (ql.conj().T @ y)
    assert np.abs(q @ (q.conj().T @ yp) - yp).max() < 1e-13


def test_degree_rule_is_minimal_degree_meeting_tolerance():
    mu = np.array([-20.0, -18.5, -17.0, -16.0, -15.2])
    res = np.array([1e-2, 3e-5, 4e-4, 1e-1, 2e-3])
    alpha, beta, tol = -15.0, 40.0, 1e-9
    deg = chfsi.degree_rule(mu, res, 4, alpha, beta, tol, 40)
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    for j in range(4):
        t = (mu[j] - c) / e
        r = abs(t) + math.sqrt(t * t - 1)
        m = int(deg[j])
        if m < 40:
            assert res[j] / r ** m <= tol * (1 + 1e-12)
            assert m == 1 or res[j] / r ** (m - 1) > tol
    assert deg[4] == deg[:4].max()       # the guard takes the largest wanted degree


def test_degree_rule_clamps():
    deg = chfsi.degree_rule(np.array([-15.01, -15.005]), np.array([1.0, 1.0]), 2, -15.0, 40.0,
                            1e-12, 40)
    assert list(deg) == [40, 40]
    deg = chfsi.degree_rule(np.array([-100.0]), np.array([2e-9]), 1, -15.0, 40.0, 1e-9, 40)
    assert list(deg) == [1]


def test_reduce_to_standard_identity_and_diagonal():
    n = 20
    a = gen.random_hermitian_unit(n, 3)
    h, _ = chfsi.reduce_to_standard(a, np.eye(n, dtype=complex))
    assert np.abs(h - a).max() < 1e-15
    da = np.linspace(-3, 3, n)
    db = np.linspace(1, 2, n)
    h, _ = chfsi.reduce_to_standard(np.diag(da).astype(complex), np.diag(db).astype(complex))
    assert np.allclose(np.sort(np.diag(h).real), np.sort(da / db), rtol=1e-15)
    assert np.abs(h - np.diag(np.diag(h))).max() == 0.0


def test_reduction_uses_conjugate_transpose():
    # A = L M L^H with B = L L^H has pencil eigenvalues eig(M); a plain
    # transpose in the reduction would break this.
    n = 30
    lam = np.linspace(-2, 5, n)
    m = gen.prescribed_problem(n, lam, 2)
    b = gen.random_hpd(n, 4, weight=0.5)
    l = np.linalg.cholesky(b)
    a = l @ m @ l.conj().T
    h, _ = chfsi.reduce_to_standard(a, b)
    assert np.abs(eigh.eigvalsh(h) - lam).max() < 1e-12


def _solve(a, nev, nex, **kw):
    b = kw.pop("b", None)
    return chfsi.chfsi(a, nev, nex, b=b, opts=chfsi.Options(**kw))


def test_chfsi_standard_matches_prescribed_spectrum():
    conf = gen.small_config("s", 240, 12, 4, False)
    seq = gen.Sequence(conf)
    a = next(seq.problems())[1]
    r = _solve(a, 12, 4)
    assert r.status == chfsi.STATUS_OK
    assert np.abs(r.lam[:12] - seq.lam[:12]).max() <= 1e-10 * np.abs(seq.lam[:12]).min()
    res = np.linalg.norm(a @ r.x[:, :12] - r.x[:, :12] * r.lam[:12], axis=0)
    assert res.max() <= 1e-10 * r.norm_h
    assert np.abs(r.x.conj().T @ r.x - np.eye(16)).max() < 1e-12


def test_chfsi_generalized_known_pencil_eigenvalues():
    n, nev, nex = 160, 8, 3
    lam = gen.spectrum(n, np.random.Generator(np.random.PCG64(5)))
    m = gen.prescribed_problem(n, lam, 6)
    b = gen.random_hpd(n, 7)
    l = np.linalg.cholesky(b)
    a = l @ m @ l.conj().T
    a = 0.5 * (a + a.conj().T)
    r = _solve(a, nev, nex, b=b)
    assert r.status == chfsi.STATUS_OK
    assert np.abs(r.lam[:nev] - lam[:nev]).max() <= 1e-10 * np.abs(lam[:nev]).min()
    x = r.x
    assert np.abs(x.conj().T @ b @ x - np.eye(nev + nex)).max() < 1e-12
    gres = np.linalg.norm(a @ x[:, :nev] - (b @ x[:, :nev]) * r.lam[:nev], axis=0)
    assert gres.max() < 1e-9 * np.abs(lam).max()


def test_generalized_with_identity_b_equals_standard():
    conf = gen.small_config("s", 120, 6, 2, False)
    a = next(gen.Sequence(conf).problems())[1]
    r1 = _solve(a, 6, 2)
    r2 = _solve(a, 6, 2, b=np.eye(120, dtype=complex))
    assert np.abs(r1.lam[:6] - r2.lam[:6]).max() < 1e-12


def test_chfsi_vs_own_dense_solver_along_a_sequence():
    conf = gen.small_config("s", 200, 10, 4, True, length=3)
    seq = gen.Sequence(conf)
    probs = [a.copy() for _, a in seq.problems()]
    rs = chfsi.solve_sequence(probs, 10, 4, b=seq.B)
    for a, r in zip(probs, rs):
        h, _ = chfsi.reduce_to_standard(a, seq.B)
        ref = eigh.eigvalsh(h)[:10]
        assert r.status == chfsi.STATUS_OK
        assert np.abs(r.lam[:10] - ref).max() <= 1e-10 * np.abs(ref).min()


def test_warm_start_needs_fewer_matvecs_than_random_start():
    # Sec. 4.2: approximate eigenvectors of the previous problem beat random vectors
    conf = gen.small_config("s", 300, 15, 5, False, length=3)
    probs = [a.copy() for _, a in gen.Sequence(conf).problems()]
    warm = chfsi.solve_sequence(probs, 15, 5, warm=True)
    cold = chfsi.solve_sequence(probs, 15, 5, warm=False)
    for w, c in zip(warm[1:], cold[1:]):
        assert w.matvecs < 0.7 * c.matvecs
        assert np.abs(w.lam[:15] - c.lam[:15]).max() < 1e-11 * np.abs(c.lam[:15]).max()


def test_analytic_degrees_need_fewer_matvecs_than_fixed_degree():
    # Sec. 3.1.1 / 4.2: Single Optimization lowers the number of mat-vecs
    conf = gen.small_config("s", 300, 15, 5, False, length=2)
    probs = [a.copy() for _, a in gen.Sequence(conf).problems()]
    opt = chfsi.solve_sequence(probs, 15, 5, opts=chfsi.Options(degree_mode=0))
    fix = chfsi.solve_sequence(probs, 15, 5, opts=chfsi.Options(degree_mode=1, deg0=20))
    assert sum(r.matvecs for r in opt) < sum(r.matvecs for r in fix)
    for a, b in zip(opt, fix):
        assert np.abs(a.lam[:15] - b.lam[:15]).max() < 1e-11 * np.abs(b.lam[:15]).max()


def test_literal_alpha_rule_converges_to_same_eigenvalues():
    conf = gen.small_config("s", 150, 8, 3, False)
    a = next(gen.Sequence(conf).problems())[1]
    r0 = _solve(a, 8, 3)
    r1 = _solve(a, 8, 3, alpha_rule=1)
    assert r1.status == chfsi.STATUS_OK
    assert np.abs(r0.lam[:8] - r1.lam[:8]).max() < 1e-11 * np.abs(r0.lam[:8]).max()


def test_status_codes():
    conf = gen.small_config("s", 100, 5, 2, False)
    a = next(gen.Sequence(conf).problems())[1]
    assert _solve(a, 5, 2, max_iter=1).status == chfsi.STATUS_NO_CONVERGENCE
    bad = a.copy()
    bad[3, 4] = np.nan
    assert _solve(bad, 5, 2).status == chfsi.STATUS_NONFINITE
    b = np.eye(100, dtype=complex)
    b[7, 7] = -1.0
    assert _solve(a, 5, 2, b=b).status == chfsi.STATUS_NOT_HPD
    with pytest.raises(ValueError):
        _solve(a, 5, 0)


def test_filter_is_the_dominant_cost():
    # Sec. 3.1: filter work O(m n^2 k) dominates (m >> 1)
    conf = gen.small_config("s", 200, 10, 4, False)
    a = next(gen.Sequence(conf).problems())[1]
    r = _solve(a, 10, 4)
    assert r.filter_matvecs > 0.8 * r.matvecs


def test_std_n1000_sequence_matches_prescribed_and_dense_spectra():
    """The full n = 1000 standard workload: problem 1 has the prescribed
    spectrum; problem 2 is checked against the oracle's own dense solver."""
    conf = gen.CONFIGS["std-n1000"]
    seq = gen.Sequence(conf)
    probs = [a.copy() for _, a in seq.problems()]
    rs = chfsi.solve_sequence(probs, conf.nev, conf.nex)
    assert all(r.status == chfsi.STATUS_OK for r in rs)
    lam = seq.lam[:conf.nev]
    assert np.abs(rs[0].lam[:conf.nev] - lam).max() <= 1e-10 * np.abs(lam).min()
    ref = eigh.eigvalsh(probs[1])[:conf.nev]
    assert np.abs(rs[1].lam[:conf.nev] - ref).max() <= 1e-10 * np.abs(ref).min()
    # warm-started problems need far fewer mat-vecs than the cold first one
    assert max(r.matvecs for r in rs[1:]) < 0.5 * rs[0].matvecs


def test_previous_eigenvalues_as_filter_bounds():
    """Alg. 1 takes the previous problem's eigenvalues as inputs; using them
    instead of a start Rayleigh-Ritz saves mat-vecs and gives the same
    eigenvalues."""
    conf = gen.small_config("s", 300, 15, 5, False, length=3)
    probs = [a.copy() for _, a in gen.Sequence(conf).problems()]
    plain = chfsi.solve_sequence(probs, 15, 5)
    lam = chfsi.solve_sequence(probs, 15, 5, with_lambda=True)
    for p, q in zip(plain[1:], lam[1:]):
        assert q.status == chfsi.STATUS_OK
        assert q.matvecs < p.matvecs
        assert np.abs(p.lam[:15] - q.lam[:15]).max() < 1e-11 * np.abs(p.lam[:15]).max()
