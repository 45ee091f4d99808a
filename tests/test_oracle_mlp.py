"""Pins for the oracle's degree network, its training step and the learned
degree rule.

Expected values come from outside the oracle's own formulas: central finite
differences of the loss, closed forms of a network with a single active
path, Adam's first step (which moves every weight by lr * sign(g) up to
eps), hand-derived features of inputs built so that |rho| and the residual
ratio are known exactly, and the paper's analytic rule (Sec. 3.1.1), which
the learned rule must reproduce when the network outputs 0."""
import math

import numpy as np
import pytest

from oracle import chebyshev, mlp
from oracle import chfsi as ochfsi


def _blob(seed, scale=0.3):
    g = np.random.default_rng(seed)
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.SL_MEAN] = g.normal(size=8) * 0.5
    p[mlp.SL_SCALE] = g.uniform(0.5, 2.0, 8)
    p[mlp.TRAINED] = g.normal(size=mlp.TRAINED.stop - mlp.TRAINED.start) * scale
    return p


def _data(n, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, 8))
    T = np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2]
    return X, T


def test_layout_sizes():
    assert mlp.N_PARAMS == 8 + 8 + 64 * 8 + 64 + 64 * 64 + 64 + 64 + 1 + 1 == 4818


def test_gradient_matches_central_differences():
    p = _blob(1)
    X, T = _data(37, 2)
    _, g = mlp.loss_and_grad(p, X, T)
    n = X.shape[0]

    def mse(q):
        y = mlp.forward(q, X)
        return float(np.mean((y - T) ** 2))

    rng = np.random.default_rng(3)
    idx = np.concatenate([
        rng.choice(np.arange(mlp.SL_W1.start, mlp.SL_W1.stop), 12, replace=False),
        rng.choice(np.arange(mlp.SL_B1.start, mlp.SL_B1.stop), 6, replace=False),
        rng.choice(np.arange(mlp.SL_W2.start, mlp.SL_W2.stop), 12, replace=False),
        rng.choice(np.arange(mlp.SL_B2.start, mlp.SL_B2.stop), 6, replace=False),
        rng.choice(np.arange(mlp.SL_W3.start, mlp.SL_W3.stop), 6, replace=False),
        [mlp.I_B3]])
    h = 1e-6
    for i in idx:
        q1, q2 = p.copy(), p.copy()
        q1[i] += h
        q2[i] -= h
        fd = (mse(q1) - mse(q2)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(fd), (i, fd, g[i])
    # statistics and margin are not trained
    assert np.all(g[mlp.SL_MEAN] == 0) and np.all(g[mlp.SL_SCALE] == 0) and g[mlp.I_MARGIN] == 0
    sse, _ = mlp.loss_and_grad(p, X, T)
    assert sse == pytest.approx(mse(p) * n, rel=1e-12)


def test_forward_single_path_closed_form():
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.SL_SCALE] = 1.0
    p[mlp.SL_MEAN.start + 2] = 0.5
    p[mlp.SL_SCALE.start + 2] = 2.0
    # hidden unit 5 of layer 1 reads feature 2; unit 7 of layer 2 reads it
    p[mlp.SL_W1.start + 5 * 8 + 2] = 1.3
    p[mlp.SL_B1.start + 5] = -0.2
    p[mlp.SL_W2.start + 7 * 64 + 5] = 0.9
    p[mlp.SL_B2.start + 7] = 0.1
    p[mlp.SL_W3.start + 7] = -1.7
    p[mlp.I_B3] = 0.25
    x = np.zeros((3, 8))
    x[:, 2] = [-1.0, 0.5, 3.0]
    z = (x[:, 2] - 0.5) / 2.0
    want = 0.25 - 1.7 * np.tanh(0.9 * np.tanh(1.3 * z - 0.2) + 0.1)
    # the other hidden units of layer 2 see tanh(b) = 0 through zero weights
    assert np.allclose(mlp.forward(p, x), want, rtol=0, atol=1e-15)


def test_zero_network_outputs_bias():
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.I_B3] = -0.75
    assert np.all(mlp.forward(p, np.random.default_rng(0).normal(size=(5, 8))) == -0.75)


def test_adam_first_step_is_sign_step():
    p = _blob(4)
    g = np.random.default_rng(5).normal(size=mlp.N_PARAMS)
    g[np.abs(g) < 1e-3] = 1e-3
    lr = 1e-2
    p1, m, v = mlp.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), lr, 1)
    d = p1 - p
    sl = mlp.TRAINED
    assert np.allclose(d[sl], -lr * np.sign(g[sl]), rtol=1e-4, atol=0)
    assert np.all(d[mlp.SL_MEAN] == 0) and np.all(d[mlp.SL_SCALE] == 0) and d[mlp.I_MARGIN] == 0
    assert np.allclose(m[sl], 0.1 * g[sl]) and np.allclose(v[sl], 0.001 * g[sl] ** 2)


def test_adam_two_steps_scalar_closed_form():
    # scalar b3 with gradients g1, g2: m2 = .09 g1 + .1 g2, v2 = .000999 g1^2 + .001 g2^2
    p = np.zeros(mlp.N_PARAMS)
    g1, g2, lr = 0.4, -1.1, 0.05
    G1 = np.zeros(mlp.N_PARAMS); G1[mlp.I_B3] = g1
    G2 = np.zeros(mlp.N_PARAMS); G2[mlp.I_B3] = g2
    p1, m, v = mlp.adam_step(p, G1, np.zeros_like(p), np.zeros_like(p), lr, 1)
    p2, m, v = mlp.adam_step(p1, G2, m, v, lr, 2)
    mhat = (0.09 * g1 + 0.1 * g2) / (1 - 0.81)
    vhat = (0.000999 * g1 ** 2 + 0.001 * g2 ** 2) / (1 - 0.999 ** 2)
    want = -lr * 1.0 - lr * mhat / (math.sqrt(vhat) + 1e-8)   # first step: -lr sign(g1)
    assert p2[mlp.I_B3] == pytest.approx(want, rel=1e-6)


def test_training_reduces_loss():
    p = _blob(6, scale=0.1)
    X, T = _data(200, 7)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    l0, _ = mlp.loss_and_grad(p, X, T)
    for t in range(1, 301):
        _, g = mlp.loss_and_grad(p, X, T)
        p, m, v = mlp.adam_step(p, g, m, v, 3e-3, t)
    l1, _ = mlp.loss_and_grad(p, X, T)
    assert l1 < 0.2 * l0


def _interval_for(ln_rho, alpha=-10.0, beta=30.0):
    """A Ritz value below alpha whose |rho| is exp(ln_rho): t = -cosh(ln_rho)."""
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    return c - e * math.cosh(ln_rho)


def test_features_closed_form():
    alpha, beta, gamma = -10.0, 30.0, -25.0
    s = 0.37
    mu = _interval_for(s, alpha, beta)
    tol_abs, norm_h = 1e-9, 40.0
    a = 9.5
    res = tol_abs * math.exp(a)
    e = 20.0
    f = mlp.features(mu, res, 0.5, alpha, beta, gamma, norm_h, tol_abs, 3)
    assert f[0] == pytest.approx(a, rel=1e-13)
    assert f[1] == pytest.approx(math.log(s), rel=1e-12)
    assert f[2] == pytest.approx(math.log(a / s), rel=1e-12)
    assert f[3] == pytest.approx(math.log(math.cosh(s)), rel=1e-12)
    assert f[4] == pytest.approx((mu - gamma) / (alpha - gamma), rel=1e-14)
    assert f[5] == pytest.approx(math.log(0.5 / e), rel=1e-14)
    assert f[6] == pytest.approx(math.log(res / norm_h), rel=1e-14)
    assert f[7] == 2.0
    # inside the damped interval there is no rate
    assert mlp.features(10.0, res, 0.5, alpha, beta, gamma, norm_h, tol_abs, 1) is None
    # converged residuals clamp to ratio 1; degree floor 1/2; loop clamp
    f = mlp.features(mu, 0.1 * tol_abs, 0.5, alpha, beta, gamma, norm_h, tol_abs, 9)
    assert f[0] == 0.0 and f[2] == pytest.approx(math.log(0.5)) and f[7] == 4.0


def _block(k, seed):
    g = np.random.default_rng(seed)
    mu = np.sort(np.concatenate([g.uniform(-24, -11, k - 4), g.uniform(-9, 20, 4)]))
    res = 10.0 ** g.uniform(-9, -1, k)
    return mu, res


def test_zero_output_network_reproduces_the_analytic_rule():
    k, nw = 40, 30
    mu, res = _block(k, 8)
    alpha, beta, gamma, norm_h, tol_abs = mu[-1], 60.0, mu[0] - 1.0, 60.0, 6e-9
    rule = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol_abs, 40)
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.SL_SCALE] = 1e3          # nothing is out of range
    deg, y, src, _ = mlp.learned_degrees(p, mu, res, nw, alpha, beta, gamma, norm_h, tol_abs, 2,
                                         40, rule=rule)
    assert np.all(y[src == 1] == 0.0)
    assert np.array_equal(deg, rule)


def test_slower_rate_scales_degrees_and_margin():
    k, nw = 30, 20
    mu, res = _block(k, 9)
    alpha, beta, gamma, norm_h, tol_abs = mu[-1], 60.0, mu[0] - 1.0, 60.0, 6e-9
    rule = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol_abs, 400)
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.SL_SCALE] = 1e3
    p[mlp.I_B3] = -math.log(2.0)   # vectors converge at half the analytic rate
    p[mlp.I_MARGIN] = math.log(1.5)
    deg, _, src, _ = mlp.learned_degrees(p, mu, res, nw, alpha, beta, gamma, norm_h, tol_abs, 1,
                                         400, rule=rule)
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    r = chebyshev.rho((mu - c) / e)
    for j in range(nw):
        if src[j] == 1:
            m_a = math.log(max(res[j] / tol_abs, 1.0)) / math.log(r[j])
            lo, hi = math.ceil(3.0 * m_a - 1e-9), math.ceil(3.0 * m_a + 1e-9)
            assert max(lo, 1) <= deg[j] <= max(hi, 1), (j, deg[j], 3.0 * m_a)
    fill = deg[src == 1].max()
    assert np.all(deg[src == 2] == fill)


def test_out_of_range_inputs_fall_back_to_the_rule():
    k, nw = 12, 10
    mu, res = _block(k, 10)
    alpha, beta, gamma, norm_h, tol_abs = mu[-1], 60.0, mu[0] - 1.0, 60.0, 6e-9
    rule = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol_abs, 40)
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.SL_SCALE] = 1e-3         # every standardised feature is huge
    p[mlp.I_B3] = -3.0
    deg, _, src, _ = mlp.learned_degrees(p, mu, res, nw, alpha, beta, gamma, norm_h, tol_abs, 1,
                                         40, rule=rule)
    assert np.all(src[:nw][src[:nw] != 2] == 0)
    assert np.array_equal(deg, rule)


def test_margin_only_in_loops_that_can_finish():
    k, nw = 30, 20
    mu, res = _block(k, 12)
    alpha, beta, gamma, norm_h, tol_abs = mu[-1], 60.0, mu[0] - 1.0, 60.0, 6e-9
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.SL_SCALE] = 1e3
    p[mlp.I_MARGIN] = math.log(2.0)
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    r = chebyshev.rho((mu - c) / e)
    m_a = np.array([math.log(max(res[j] / tol_abs, 1.0)) / math.log(r[j]) if r[j] > 1 else 0.0
                    for j in range(k)])
    big = int(np.ceil(m_a[:nw].max()))
    # every vector fits under the cap: the margin doubles the degrees
    rule = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol_abs, big)
    deg, _, src, _ = mlp.learned_degrees(p, mu, res, nw, alpha, beta, gamma, norm_h, tol_abs, 1,
                                         big, rule=rule)
    net = np.where(src == 1)[0]
    assert len(net) > 10
    for j in net:
        lo, hi = math.ceil(2 * m_a[j] - 1e-9), math.ceil(2 * m_a[j] + 1e-9)
        assert min(max(lo, 1), big) <= deg[j] <= min(max(hi, 1), big)
    # one vector needs more than the cap: no margin, the rule's degrees
    cap = big - 1
    rule = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol_abs, cap)
    deg, _, src, _ = mlp.learned_degrees(p, mu, res, nw, alpha, beta, gamma, norm_h, tol_abs, 1,
                                         cap, rule=rule)
    assert np.array_equal(deg, rule)


# ---------------------------------------------------------------------------
# the gap feature, the training target and the margin

def test_ritz_gap_closed_form():
    mu = [0.0, 1.0, 3.0, 7.0]
    assert [mlp.ritz_gap(mu, j, 5.0) for j in range(4)] == [1.0, 1.0, 2.0, 4.0]
    assert mlp.ritz_gap([2.5], 0, 0.75) == 0.75           # one value: the half-width e


def test_ritz_gap_pin_catches_one_sided_gap():
    def right_only(mu, j, e):
        return mu[j + 1] - mu[j] if j + 1 < len(mu) else e

    def left_only(mu, j, e):
        return mu[j] - mu[j - 1] if j > 0 else e

    mu = [0.0, 1.0, 3.0, 7.0]
    want = [1.0, 1.0, 2.0, 4.0]
    assert [right_only(mu, j, 5.0) for j in range(4)] != want
    assert [left_only(mu, j, 5.0) for j in range(4)] != want


@pytest.mark.parametrize("eff", [0.25, 0.5, 1.0, 2.0, 5.0])
def test_training_target_recovers_a_known_rate(eff):
    # a vector that converged eff times as fast as eq. (resl)'s model:
    # res_after = res_before |rho|^(-eff m)
    res, m, ln_rho, tol = 3e-4, 6, 0.35, 1e-9
    after = res * math.exp(-eff * m * ln_rho)
    y = mlp.training_target(res, after, m, ln_rho, tol)
    assert abs(y - math.log(eff)) < 1e-12


def test_training_target_floor_clip_and_exclusions():
    res, m, ln_rho, tol = 1e-3, 6, 0.25, 1e-9
    # below 1e-2 tol the residual is raised to it: eff = ln(1e-3/1e-11)/1.5 = 12.3, clipped to 8
    assert abs(mlp.training_target(res, 1e-30, m, ln_rho, tol) - math.log(8.0)) < 1e-15
    # just above the floor: not raised
    after = 2e-11
    want = math.log(math.log(res / after) / (m * ln_rho))
    assert abs(mlp.training_target(res, after, m, ln_rho, tol) - min(want, math.log(8.0))) < 1e-12
    # a residual that grew: eff < 0, clipped to 0.05
    assert abs(mlp.training_target(res, 2 * res, m, ln_rho, tol) - math.log(0.05)) < 1e-15
    # unusable records
    assert mlp.training_target(res, 1e-5, m, ln_rho, tol, fp32_loop=True) is None
    assert mlp.training_target(res, 1e-5, 0, ln_rho, tol) is None
    assert mlp.training_target(res, 0.0, m, ln_rho, tol) is None
    assert mlp.training_target(res, float("nan"), m, ln_rho, tol) is None
    assert mlp.training_target(res, 1e-5, m, 0.0, tol) is None


def test_holdout_margin_closed_forms():
    assert mlp.holdout_margin([1.0, -1.0, 1.0, -1.0], [0.0] * 4) == pytest.approx(3.0, abs=1e-15)
    assert mlp.holdout_margin([1.0, 2.0], [3.0, 4.0]) == 0.0          # all errors -2
    assert mlp.holdout_margin([0.5] * 4, [0.0] * 4) == pytest.approx(0.5, abs=1e-15)
    assert mlp.holdout_margin([2.0, 0.0], [0.0, 0.0], z=1.0) == pytest.approx(2.0, abs=1e-15)
    assert mlp.holdout_margin([], []) == 0.0
