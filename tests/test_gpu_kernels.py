"""GPU parity of the library's steps (called through the C ABI) against the
CPU oracle, on the same seeded inputs: complex GEMM, the Chebyshev filter
(Alg. 2), orthonormalisation, Rayleigh-Ritz + residuals, Lanczos bounds
and the reduction to standard form.  Sizes span several 64-wide tiles and
ragged tails."""
import numpy as np
import pytest

import paper_1404_4161_amd as ch
from oracle import chebyshev, chfsi as ochfsi, counter_rng, eigh
from workloads import gen

from .gpu_util import dev, host, rel_col_err

pytestmark = pytest.mark.gpu


def _rand(m, n, seed):
    return gen.random_block(m, n, seed)


@pytest.mark.parametrize("opa,opb", [("N", "N"), ("N", "C"), ("C", "N"), ("C", "C")])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 5, 9), (64, 64, 64), (130, 67, 71),
                                   (200, 129, 300), (40, 36, 5000), (8, 3, 0), (130, 67, 1001),
                                   (2048, 1030, 777)])
def test_zgemm_matches_numpy(opa, opb, M, N, K):
    """K >= 512 runs the 3M split (for N, N the direct-to-LDS tile, whose K
    tail reads a zero page: 1001 and 777 leave 1 of 8); (130, 67, 1001)
    splits K, (2048, 1030, 777) is a launch of 544 tiles without split-K
    and with ragged edges."""
    a = _rand(M, K, 1) if opa == "N" else _rand(K, M, 1)
    b = _rand(K, N, 2) if opb == "N" else _rand(N, K, 2)
    c = _rand(M, N, 3)
    alpha, beta = 0.7 - 0.3j, -0.4 + 1.1j
    opA = a if opa == "N" else a.conj().T
    opB = b if opb == "N" else b.conj().T
    ref = alpha * (opA @ opB) + beta * c
    cd = dev(c)
    ch.chfsi_zgemm(opa, opb, alpha, dev(a), dev(b), beta, cd)
    got = host(cd)
    scale = (np.abs(opA) @ np.abs(opB)).max() + np.abs(c).max()
    assert np.abs(got - ref).max() <= 1e-14 * max(K, 1) * scale


def _herm_problem(n, seed):
    lam = np.sort(np.random.default_rng(seed).uniform(-20, 40, n))
    return lam, gen.prescribed_problem(n, lam, seed + 1)


@pytest.mark.parametrize("n,k,degrees", [
    (200, 5, [1, 1, 2, 3, 3]),
    (333, 37, None),
    (1000, 70, "cfg"),
])
def test_filter_matches_oracle(n, k, degrees):
    lam, h = _herm_problem(n, 7)
    g = np.random.default_rng(n)
    if degrees is None:
        degrees = np.sort(g.integers(1, 16, k)).tolist()
    elif degrees == "cfg":
        degrees = [10] * k
    y0 = _rand(n, k, 11)
    alpha, beta = -15.0, 41.0
    c, e, gamma = 0.5 * (alpha + beta), 0.5 * (beta - alpha), -20.5
    ref = chebyshev.chebyshev_filter(h, y0, degrees, c, e, gamma)
    yd = dev(y0)
    flops, launches = ch.chfsi_filter(dev(h), yd, degrees, c, e, gamma)
    got = host(yd)
    assert rel_col_err(got, ref).max() < 1e-11
    assert launches == max(degrees)
    assert flops == pytest.approx(8.0 * n * n * sum(degrees))


def test_filter_single_column_and_all_degree_one():
    n = 97
    lam, h = _herm_problem(n, 3)
    y0 = _rand(n, 1, 4)
    ref = chebyshev.chebyshev_filter(h, y0, [6], 10.0, 30.0, -19.0)
    yd = dev(y0)
    ch.chfsi_filter(dev(h), yd, [6], 10.0, 30.0, -19.0)
    assert rel_col_err(host(yd), ref).max() < 1e-12
    y1 = _rand(n, 3, 5)
    ref1 = chebyshev.chebyshev_filter(h, y1, [1, 1, 1], 10.0, 30.0, -19.0)
    yd1 = dev(y1)
    ch.chfsi_filter(dev(h), yd1, [1, 1, 1], 10.0, 30.0, -19.0)
    assert rel_col_err(host(yd1), ref1).max() < 1e-13


def test_filter_rejects_unsorted_degrees():
    h = dev(np.eye(8))
    y = dev(np.ones((8, 2)))
    with pytest.raises(ch.ChfsiError):
        ch.chfsi_filter(h, y, [3, 1], 0.0, 1.0, -2.0)


@pytest.mark.parametrize("n,k,nl", [(150, 20, 0), (300, 45, 30), (1000, 70, 0)])
def test_orthonormalize_matches_oracle_span(n, k, nl):
    y = _rand(n, k, 21)
    ql = ochfsi.orthonormalize(_rand(n, nl, 22), np.zeros((n, 0), complex)) if nl else None
    ref = ochfsi.orthonormalize(y, ql if nl else np.zeros((n, 0), complex))
    yd = dev(y)
    ch.chfsi_orthonormalize(yd, dev(ql) if nl else None)
    q = host(yd)
    assert np.abs(q.conj().T @ q - np.eye(k)).max() < 1e-13
    if nl:
        assert np.abs(ql.conj().T @ q).max() < 1e-13
    # same span as the oracle's QR basis
    assert np.abs(ref @ (ref.conj().T @ q) - q).max() < 1e-12


def test_orthonormalize_ill_conditioned_block_uses_shift():
    n, k = 400, 24
    lam, h = _herm_problem(n, 5)
    y0 = _rand(n, k, 6)
    # filtering a random block with a high degree makes it nearly rank deficient
    y = chebyshev.chebyshev_filter(h, y0, [40] * k, 25.0, 16.0, -20.0)
    yd = dev(y)
    shifted = ch.chfsi_orthonormalize(yd)
    q = host(yd)
    assert np.abs(q.conj().T @ q - np.eye(k)).max() < 1e-12
    assert shifted in (0, 1)


@pytest.mark.parametrize("n,k", [(130, 17), (1000, 70)])
def test_rayleigh_ritz_and_residuals_match_oracle(n, k):
    lam, h = _herm_problem(n, 9)
    q = ochfsi.orthonormalize(_rand(n, k, 3), np.zeros((n, 0), complex))
    mu_ref, q_ref, z_ref = ochfsi.rayleigh_ritz(h, q)
    res_ref = ochfsi.residual_norms(q_ref, z_ref, mu_ref)
    qd = dev(q)
    zd = dev(np.zeros((n, k), complex))
    mu, res = ch.chfsi_rayleigh_ritz(dev(h), qd, zd)
    assert np.abs(mu - mu_ref).max() <= 1e-12 * np.abs(lam).max()
    assert np.abs(res - res_ref).max() <= 1e-11 * np.abs(lam).max()
    qg, zg = host(qd), host(zd)
    assert np.abs(zg - h @ qg).max() < 1e-11 * np.abs(lam).max()
    assert np.abs(qg.conj().T @ qg - np.eye(k)).max() < 1e-12


def _projected(k, kind, seed):
    """k x k Hermitian test matrices for the projected eigenproblem:
    'dense' random, 'near' a separated diagonal plus a 1e-6 coupling,
    'clustered' a spectrum with close (gaps 1e-5, 1e-7, 1e-10) and exactly
    degenerate pairs and a triple, mixed by rotations inside those groups,
    plus a 1e-8 coupling (what Rayleigh-Ritz sees in the loops of a
    warm-started sequence)."""
    g = np.random.default_rng(seed)

    def herm(scale):
        a = g.standard_normal((k, k)) + 1j * g.standard_normal((k, k))
        return scale * 0.5 * (a + a.conj().T)

    if kind == "dense":
        return herm(1.0)
    d = np.sort(np.concatenate([g.uniform(-20, -15, k - k // 6), g.uniform(-15, -14, k // 6)]))
    if kind == "near":
        m = np.diag(d).astype(complex) + herm(1e-6)
        return 0.5 * (m + m.conj().T)
    d[10] = d[9] + 1e-5
    d[21] = d[20] + 1e-7
    d[31] = d[30] + 1e-10
    d[41] = d[40]
    d[51], d[52] = d[50] + 1e-9, d[50] + 2e-9
    q = np.eye(k, dtype=complex)
    for i, j in [(9, 10), (20, 21), (30, 31), (40, 41), (50, 51), (51, 52)]:
        th, ph = g.uniform(0.2, 1.3), np.exp(1j * g.uniform(0, 6.2))
        r = np.eye(k, dtype=complex)
        r[i, i], r[i, j], r[j, i], r[j, j] = (np.cos(th), np.sin(th) * ph,
                                              -np.sin(th) * np.conj(ph), np.cos(th))
        q = q @ r
    m = q @ np.diag(d) @ q.conj().T + herm(1e-8)
    return 0.5 * (m + m.conj().T)


@pytest.mark.parametrize("kind,k", [("dense", 100), ("near", 1), ("near", 70), ("near", 480),
                                    ("clustered", 130), ("clustered", 480)])
@pytest.mark.parametrize("mode", [0, 1])
def test_projected_eigenproblem_matches_oracle(kind, k, mode):
    """Rayleigh-Ritz's k x k eigenproblem: the dense solver (mode 0) and the
    refinement from the identity with its fallback (mode 1) both give the
    oracle's eigenvalues to 1e-13 of ||G||, a unitary W to 1e-13 and
    residuals ||G W - W diag(mu)|| to 1e-13 ||G||; the refinement is the one
    that answers on the nearly diagonal matrices (with their clusters), the
    fallback on the dense one."""
    gm = _projected(k, kind, 5 + k)
    ref = eigh.eigvalsh(gm)
    mu, wd, refined = ch.chfsi_eigh_projected(dev(gm), mode=mode)
    w = host(wd)
    scale = np.abs(ref).max()
    assert np.all(np.diff(mu) >= 0)
    assert np.abs(mu - ref).max() <= 1e-13 * scale
    assert np.abs(w.conj().T @ w - np.eye(k)).max() <= 1e-13
    assert np.abs(gm @ w - w * mu).max() <= 1e-13 * scale
    assert refined == (mode == 1 and kind != "dense")


def test_projected_eigenproblem_refinement_only_reports_failure():
    gm = _projected(64, "dense", 3)
    with pytest.raises(ch.ChfsiError) as ei:
        ch.chfsi_eigh_projected(dev(gm), mode=2)
    assert ei.value.status == ch.binding.CHFSI_NO_CONVERGENCE
    mu, _, refined = ch.chfsi_eigh_projected(dev(_projected(64, "near", 3)), mode=2)
    assert refined == 1


@pytest.mark.parametrize("n", [5, 300, 1000])
def test_lanczos_bounds_match_oracle(n):
    lam, h = _herm_problem(n, 13)
    v0 = counter_rng.complex_block(3, counter_rng.STREAM_LANCZOS, n, 1)
    ref = ochfsi.lanczos_bounds(h, 20, v0)
    got = ch.chfsi_lanczos_bounds(dev(h), 20, 3)
    assert abs(got[0] - ref[0]) <= 1e-9 * abs(ref[0])
    assert abs(got[1] - ref[1]) <= 1e-9 * max(abs(ref[1]), 1.0)
    assert abs(got[2] - ref[2]) <= 1e-9 * abs(ref[2])
    assert got[0] >= lam[-1] - 1e-9


@pytest.mark.parametrize("n", [64, 300, 700, 1100])
def test_reduce_standard_matches_oracle(n):
    a = gen.prescribed_problem(n, np.linspace(-20, 40, n), 2)
    b = gen.random_hpd(n, 3)
    h_ref, l_ref = ochfsi.reduce_to_standard(a, b)
    hd, ld = ch.chfsi_reduce_standard(dev(a), dev(b))
    h, l = host(hd), host(ld)
    assert np.abs(l - l_ref).max() < 1e-13
    assert np.abs(h - h_ref).max() < 1e-12 * np.abs(h_ref).max()
    assert np.abs(h - h.conj().T).max() == 0.0


def test_reduce_standard_detects_non_hpd():
    n = 70
    a = gen.random_hermitian_unit(n, 1)
    b = np.eye(n, dtype=complex)
    b[66, 66] = -1.0
    with pytest.raises(ch.ChfsiError) as ei:
        ch.chfsi_reduce_standard(dev(a), dev(b))
    assert ei.value.status == ch.binding.CHFSI_NOT_HPD


@pytest.mark.parametrize("delta,n,k", [(1e-3, 700, 40), (1e-6, 700, 40), (1e-3, 1000, 400)])
def test_defect_filter_matches_oracle_with_error_scaling_like_the_residual(delta, n, k):
    """The FP32 defect filter reproduces the oracle's FP64 filter on Ritz
    vectors; its error is about eps_fp32 * ||R|| / ||H|| (times the filter's
    growth), i.e. it shrinks with the residuals.  k = 400 runs the wide
    (128 x 128 tile) form while the window is at least 384 columns wide."""
    lam, h = _herm_problem(n, 23)
    q0 = np.linalg.eigh(h)[1][:, :k]
    noisy = q0 + delta * _rand(n, k, 24)
    q = ochfsi.orthonormalize(noisy, np.zeros((n, 0), complex))
    mu, q, z = ochfsi.rayleigh_ritz(h, q)
    res = ochfsi.residual_norms(q, z, mu)
    deg = np.sort(np.random.default_rng(3).integers(2, 20 if k < 100 else 9, k)).tolist()
    alpha, beta = float(mu[-1]) + 1.0, 41.0
    c, e, gamma = 0.5 * (alpha + beta), 0.5 * (beta - alpha), float(mu[0])
    ref = chebyshev.chebyshev_filter(h, q, deg, c, e, gamma)
    yd, f32 = ch.chfsi_filter_defect(dev(h), dev(q), dev(z), mu, deg, c, e, gamma)
    got = host(yd)
    err = rel_col_err(got, ref)
    norm_h = np.abs(lam).max()
    # eq. (resl): rounding grows like (|rho_1| / |rho_j|)^m relative to column j
    growth = (chebyshev.rho(np.array([(gamma - c) / e]))[0]
              / chebyshev.rho((mu - c) / e)) ** np.array(deg)
    bound = _defect_bound(err, deg, n, 2.0 ** -24, res, norm_h, growth, "FP32 defect filter")
    assert np.all(err <= bound), (err / bound).max()
    assert f32 == pytest.approx(8.0 * n * n * sum(m - 1 for m in deg))


def _defect_bound(err, deg, n, eps, res, norm_h, growth, label):
    """Error bound of a defect filter run column by column: each of the m_j
    steps adds at most about eps times |H| |E_i| to the defect, i.e. about
    sqrt(n) eps (r_j / ||H||) relative to the column (eq. resl: E_i scales
    with the residual r_j; the sqrt(n) takes |H| |E_i| to ||H|| ||E_i||
    for rounding errors of random sign over the n-term sums), and the
    later steps grow an error by at most the filter's growth factor; so
    err_j <= m_j sqrt(n) eps (r_j / ||H||) growth_j (plus 1e-13 for the
    FP64 parts).  Prints the largest ratio to the model without the
    m_j sqrt(n) factor."""
    model = eps * (res / norm_h) * growth
    print(f"{label}: max err / (eps r/||H|| growth) = {np.max(err / (model + 1e-300)):.1f} "
          f"(bound factor m sqrt(n) up to {np.max(deg) * np.sqrt(n):.0f})")
    return np.array(deg) * np.sqrt(n) * model + 1e-13


def _split_word_check(err, eps, res, norm_h, growth):
    """A split form that kept both words of every operand stays within a
    few times eps (r / ||H||) growth of the oracle (measured on these inputs:
    at most 0.2 times for BF16 words, 1.2 times for FP16 words); one that
    dropped an operand's second word errs by about 2^-8 (BF16) or 2^-11
    (FP16) per product, 85 or 680 times eps.  8 times the model separates
    the two."""
    assert np.all(err <= 8.0 * eps * (res / norm_h) * growth + 1e-13), \
        np.max(err / (eps * (res / norm_h) * growth + 1e-300))


def _ritz_block(n, k, delta, seed):
    lam, h = _herm_problem(n, seed)
    q0 = np.linalg.eigh(h)[1][:, :k]
    q = ochfsi.orthonormalize(q0 + delta * _rand(n, k, seed + 1), np.zeros((n, 0), complex))
    mu, q, z = ochfsi.rayleigh_ritz(h, q)
    return lam, h, mu, q, z


@pytest.mark.parametrize("n,k", [(333, 70), (1000, 130), (1000, 400)])
def test_bf16_split_step_error_is_within_the_split_precision(n, k):
    """One BF16-split defect step (every degree 2): E_2 = sa (H E_1 - c E_1)
    + cr R with H E_1 formed from two-word BF16 splits of H and E_1 (three
    products; 400 columns run the 128 x 128 tile).  Each product's dropped
    split terms are at most 3 * 2^-16
    |H_ik| |E_kj| (the FP32 accumulation adds far less), so the error of
    element (i, j) is below 3 * 2^-16 |sa| (|H| |E_1|)_ij; with rounding
    errors of random sign it is a few 2^-16 |sa| times the root sum of
    squares of those terms: 2e-4 of it is a 5x margin, which one BF16 word
    per operand or a dropped cross term (errors about 2^-9 per product)
    would exceed some 25 times."""
    lam, h, mu, q, z = _ritz_block(n, k, 1e-3, 41)
    deg = [2] * k
    alpha, beta = float(mu[-1]) + 1.0, 41.0
    c, e, gamma = 0.5 * (alpha + beta), 0.5 * (beta - alpha), float(mu[0])
    ref = chebyshev.chebyshev_filter(h, q, deg, c, e, gamma)
    yd, f16, f32 = ch.chfsi_filter_defect_split(dev(h), dev(q), dev(z), mu, deg, c, e, gamma, 1)
    got = host(yd)
    sig1 = e / (gamma - c)
    sig2 = 1.0 / (2.0 / sig1 - sig1)
    e1 = (sig1 / e) * (z - q * mu)
    sa = abs(2.0 * sig2 / e)
    tiny = 1e-12 * np.abs(ref).max()
    err = np.abs(got - ref)
    worst = 3.0 * 2.0 ** -16 * sa * (np.abs(h) @ np.abs(e1)) + tiny
    assert np.all(err <= worst), (err / worst).max()
    rss = sa * np.sqrt(np.abs(h) ** 2 @ np.abs(e1) ** 2)
    assert np.all(err <= 2e-4 * rss + tiny), (err / (2e-4 * rss)).max()
    # the split precision is really coarser than FP32's (the BF16 path ran)
    assert (err / rss).max() > 2.0 ** -20
    assert f16 == pytest.approx(8.0 * n * n * k) and f32 == 0.0


@pytest.mark.parametrize("delta,n,k,steps", [(1e-3, 700, 40, 99), (1e-6, 700, 40, 99),
                                             (1e-3, 1000, 200, 4), (1e-3, 1000, 400, 5)])
def test_bf16_split_filter_matches_oracle_with_error_scaling_like_the_residual(delta, n, k,
                                                                              steps):
    """The defect filter with its first `steps` steps in BF16-split form
    (the rest FP32) reproduces the oracle's FP64 filter with the error bound
    of the FP32 form scaled by the split's precision, 3 * 2^-16 instead of
    2^-24: it shrinks with the residuals."""
    lam, h, mu, q, z = _ritz_block(n, k, delta, 23)
    res = ochfsi.residual_norms(q, z, mu)
    deg = np.sort(np.random.default_rng(3).integers(2, 20 if k < 100 else 9, k)).tolist()
    alpha, beta = float(mu[-1]) + 1.0, 41.0
    c, e, gamma = 0.5 * (alpha + beta), 0.5 * (beta - alpha), float(mu[0])
    ref = chebyshev.chebyshev_filter(h, q, deg, c, e, gamma)
    yd, f16, f32 = ch.chfsi_filter_defect_split(dev(h), dev(q), dev(z), mu, deg, c, e, gamma,
                                                steps)
    err = rel_col_err(host(yd), ref)
    norm_h = np.abs(lam).max()
    growth = (chebyshev.rho(np.array([(gamma - c) / e]))[0]
              / chebyshev.rho((mu - c) / e)) ** np.array(deg)
    bound = _defect_bound(err, deg, n, 3.0 * 2.0 ** -16, res, norm_h, growth,
                          "BF16-split defect filter")
    assert np.all(err <= bound), (err / bound).max()
    _split_word_check(err, 3.0 * 2.0 ** -16, res, norm_h, growth)
    d = np.array(deg)
    want16 = sum(int(np.sum(d > i)) for i in range(1, min(steps, d.max() - 1) + 1))
    assert f16 == pytest.approx(8.0 * n * n * want16)
    assert f16 + f32 == pytest.approx(8.0 * n * n * sum(m - 1 for m in deg))


def _ritz_block_spread(n, k, seed, hscale):
    """Ritz block of (hscale * H) whose columns' perturbations span seven
    orders of magnitude (1e-9 .. 1e-2), so that the defect columns differ in
    scale by as much (each FP16 column scale is then exercised)."""
    lam, h = _herm_problem(n, seed)
    lam, h = lam * hscale, h * hscale
    q0 = np.linalg.eigh(h)[1][:, :k]
    d = 10.0 ** np.random.default_rng(seed + 2).uniform(-9, -2, k)
    q = ochfsi.orthonormalize(q0 + _rand(n, k, seed + 1) * d, np.zeros((n, 0), complex))
    mu, q, z = ochfsi.rayleigh_ritz(h, q)
    return lam, h, mu, q, z


@pytest.mark.parametrize("n,k,hscale", [(333, 70, 1.0), (1000, 130, 1e6), (1000, 400, 1e-5),
                                        (100, 3, 1.0), (2100, 70, 1.0)])
def test_fp16_split_step_error_is_within_the_split_precision(n, k, hscale):
    """One FP16-split defect step (every degree 2): H E_1 formed from
    two-word FP16 splits of 2^s H and of 2^s_j E_1[:, j] (three products,
    FP32 accumulation; 400 columns run the 128 x 128 tile).  The dropped
    split terms are at most 3 * 2^-22 |H_ik| |E_kj|; with FP32 accumulation
    over 1500 partial sums (about 2^-20 of the root sum of squares of the
    terms, at most a few times that over all elements) the error stays below
    2^-16 of that root sum of squares, which the BF16 words (errors of a few
    2^-16 typical) exceed.  The spectra are scaled by 1e6 and 1e-5 and the
    defect columns span seven orders of magnitude, so both the scale of H
    and the per-column scales of E_1 are exercised (unscaled FP16 would
    overflow or flush them).  n = 2100 with 70 columns splits K four ways
    (partial sums reduced by a second kernel)."""
    lam, h, mu, q, z = _ritz_block_spread(n, k, 41, hscale)
    deg = [2] * k
    alpha, beta = float(mu[-1]) + 1.0 * hscale, 41.0 * hscale
    c, e, gamma = 0.5 * (alpha + beta), 0.5 * (beta - alpha), float(mu[0])
    ref = chebyshev.chebyshev_filter(h, q, deg, c, e, gamma)
    yd, fh, f32 = ch.chfsi_filter_defect_split(dev(h), dev(q), dev(z), mu, deg, c, e, gamma, 1,
                                               fp16=True)
    got = host(yd)
    sig1 = e / (gamma - c)
    sig2 = 1.0 / (2.0 / sig1 - sig1)
    e1 = (sig1 / e) * (z - q * mu)
    sa = abs(2.0 * sig2 / e)
    rss = sa * np.sqrt(np.abs(h) ** 2 @ np.abs(e1) ** 2)
    # FP32 rounding of the epilogue's other terms (sa c E_1, cr R) and of the
    # stored E_2 = Y_2 - Q p_2(mu), with p_1 = sig1 t, p_2 = 2 sig2 t p_1 -
    # sig2 sig1 (t = (mu - c) / e, the scalar recurrence)
    t = (mu - c) / e
    p1 = sig1 * t
    p2 = 2.0 * sig2 * t * p1 - sig2 * sig1
    cr = 2.0 * sig2 * p1 / e
    e2 = ref - q * p2
    floor = (2.0 ** -21 * (sa * abs(c) * np.abs(e1) + np.abs(cr * (z - q * mu)) + np.abs(e2))
             + 1e-15 * np.abs(ref).max())
    err = np.abs(got - ref)
    print(f"max err / rss {np.max(err / (rss + 1e-300)):.3e} (2^{np.log2(np.max(err / (rss + 1e-300))):.1f})")
    assert np.all(err <= 2.0 ** -16 * rss + floor), (err / (2.0 ** -16 * rss + floor)).max()
    assert fh == pytest.approx(8.0 * n * n * k) and f32 == 0.0


@pytest.mark.parametrize("fp16", [True, False])
def test_split_filter_with_exact_eigenvectors_has_zero_defect_columns(fp16):
    """Columns that are exact eigenvectors (of a diagonal H, unit vectors)
    have residual, and so defect, exactly zero: the split forms must give
    exactly Q p(mu) there (an all-zero column takes scale 1 in the FP16
    form), while the perturbed columns beside them follow the oracle."""
    n, k = 300, 24
    lam = np.sort(np.random.default_rng(5).uniform(-20, 40, n))
    h = np.diag(lam).astype(complex)
    q = np.zeros((n, k), complex)
    q[np.arange(k), np.arange(k)] = 1.0
    # columns 12 .. 23 perturbed (a Ritz block of their own span)
    q[:, 12:] = ochfsi.orthonormalize(q[:, 12:] + 1e-4 * _rand(n, 12, 6), q[:, :12])
    mu = np.real(np.einsum("ij,ij->j", q.conj(), h @ q))
    z = h @ q
    deg = [6] * k
    alpha, beta = float(lam[k]) + 0.5, 41.0
    c, e, gamma = 0.5 * (alpha + beta), 0.5 * (beta - alpha), float(lam[0])
    ref = chebyshev.chebyshev_filter(h, q, deg, c, e, gamma)
    yd, fs, f32 = ch.chfsi_filter_defect_split(dev(h), dev(q), dev(z), mu, deg, c, e, gamma, 99,
                                               fp16=fp16)
    got = host(yd)
    # exact columns: Y = p(mu) q with p(mu) from the FP64 scalar recurrence
    assert np.array_equal(got[:, :12] == 0, ref[:, :12] == 0)
    err = rel_col_err(got, ref)
    assert err[:12].max() <= 1e-14, err[:12].max()
    assert err[12:].max() <= 1e-6, err[12:].max()
    assert f32 == 0.0 and fs == pytest.approx(8.0 * n * n * k * 5)


@pytest.mark.parametrize("delta,n,k,steps", [(1e-3, 700, 40, 99), (1e-6, 700, 40, 99),
                                             (1e-3, 1000, 200, 4), (1e-3, 1000, 400, 99),
                                             (1e-3, 1500, 40, 99)])
def test_fp16_split_filter_matches_oracle_with_error_scaling_like_the_residual(delta, n, k,
                                                                              steps):
    """The defect filter with its first `steps` steps in FP16-split form
    (the rest FP32) reproduces the oracle's FP64 filter with the error bound
    of the FP32 form scaled by the split's precision, 3 * 2^-22 instead of
    2^-24: it shrinks with the residuals."""
    lam, h, mu, q, z = _ritz_block(n, k, delta, 23)
    res = ochfsi.residual_norms(q, z, mu)
    deg = np.sort(np.random.default_rng(3).integers(2, 20 if k < 100 else 9, k)).tolist()
    alpha, beta = float(mu[-1]) + 1.0, 41.0
    c, e, gamma = 0.5 * (alpha + beta), 0.5 * (beta - alpha), float(mu[0])
    ref = chebyshev.chebyshev_filter(h, q, deg, c, e, gamma)
    yd, fh, f32 = ch.chfsi_filter_defect_split(dev(h), dev(q), dev(z), mu, deg, c, e, gamma,
                                               steps, fp16=True)
    err = rel_col_err(host(yd), ref)
    norm_h = np.abs(lam).max()
    growth = (chebyshev.rho(np.array([(gamma - c) / e]))[0]
              / chebyshev.rho((mu - c) / e)) ** np.array(deg)
    bound = _defect_bound(err, deg, n, 3.0 * 2.0 ** -22, res, norm_h, growth,
                          "FP16-split defect filter")
    assert np.all(err <= bound), (err / bound).max()
    _split_word_check(err, 3.0 * 2.0 ** -22, res, norm_h, growth)
    d = np.array(deg)
    wanth = sum(int(np.sum(d > i)) for i in range(1, min(steps, d.max() - 1) + 1))
    assert fh == pytest.approx(8.0 * n * n * wanth)
    assert fh + f32 == pytest.approx(8.0 * n * n * sum(m - 1 for m in deg))


@pytest.mark.parametrize("variant,k", [(0, 70), (1, 70), (2, 300), (3, 70), (4, 70), (3, 300),
                                       (5, 70), (5, 300), (6, 70), (6, 300)])
def test_filter_tile_variants_match_oracle(variant, k):
    """Every tile variant of the filter step gives the oracle's filter (the
    autotuner only chooses between them); the wide variant runs while the
    window is at least 256 columns wide, then the default takes over;
    variants 3 and 4 are the 3M complex split, 5 and 6 the direct-to-LDS
    tiles (3M, 4M) whose K tail reads a zero page."""
    n = 333
    lam, h = _herm_problem(n, 31)
    degrees = np.sort(np.random.default_rng(5).integers(1, 12, k)).tolist()
    y0 = _rand(n, k, 32)
    ref = chebyshev.chebyshev_filter(h, y0, degrees, 10.0, 31.0, -21.0)
    try:
        ch.chfsi_autotune_set(n, k, variant)
        yd = dev(y0)
        ch.chfsi_filter(dev(h), yd, degrees, 10.0, 31.0, -21.0)
    finally:
        ch.chfsi_autotune_reset()
    assert rel_col_err(host(yd), ref).max() < 1e-11


def test_autotuner_records_a_choice_per_shape():
    ch.chfsi_autotune_reset()
    try:
        v, tf = ch.chfsi_autotune_filter([700, 1300, 1300], [64, 130, 300])
        assert v.shape == (3,) and set(v.tolist()) <= set(range(ch.binding.FILTER_VARIANTS))
        assert tf.shape == (3, ch.binding.FILTER_VARIANTS)
        others = [v for v in range(ch.binding.FILTER_VARIANTS) if v != 2]
        assert np.all(tf[:, others] > 0) and np.all(tf[:2, 2] == 0) and tf[2, 2] > 0
        # another variant only when it is clearly (2 %) faster than the default
        d = ch.binding.DEFAULT_FILTER_VARIANT
        for q in range(3):
            if v[q] == d:
                assert np.all(tf[q] <= 1.02 * tf[q, d])
            else:
                assert tf[q, v[q]] > 1.02 * tf[q, d] and tf[q, v[q]] == tf[q].max()
    finally:
        ch.chfsi_autotune_reset()
