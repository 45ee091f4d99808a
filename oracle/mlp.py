"""Degree network and its training step (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper picks each vector's filter degree from the residual model of
eq. (resl): m_j >= ln(Res_j / tol) / ln|rho_j| (Sec. 3.1.1, Single
Optimization), where 1/|rho_j| is the per-degree contraction of the
Chebyshev filter at the Ritz value.  The learned variant keeps that model
and corrects its rate with a small perceptron fitted to the solver's own
convergence logs:

  y_j  ~ ln( observed ln(Res_before / Res_after) / (m_j ln|rho_j|) )
  m_j  = max( ceil(m_a,j * exp(margin - y_j)), analytic m_j ),
  m_a,j = ln(Res_j / tol) / ln|rho_j|

so y = 0 (and margin = 0) gives back the analytic rule, and the network
can only raise a degree above the rule's.  The margin applies only in a loop
that can finish every wanted vector (all predicted degrees within the cap);
in the other loops some vectors continue anyway and margin 0 is used.  Everything here is
float64 numpy written from those definitions: the network (8 -> 64 -> 64 ->
1, tanh), the mean-squared-error gradient by backpropagation, Adam (Kingma
and Ba, ICLR 2015, with bias correction), the input features, the training
target y of one logged loop, the safety margin from held-out errors and the
learned degree rule.

Parameter blob layout (floats), the interface shared with the library:
  [0, 8) feature means, [8, 16) feature scales, [16, 528) W1 (64 x 8,
  row-major), [528, 592) b1, [592, 4688) W2 (64 x 64, row-major),
  [4688, 4752) b2, [4752, 4816) w3, [4816] b3, [4817] margin.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_H = 8, 64
SL_MEAN = slice(0, 8)
SL_SCALE = slice(8, 16)
SL_W1 = slice(16, 16 + N_H * N_IN)
SL_B1 = slice(SL_W1.stop, SL_W1.stop + N_H)
SL_W2 = slice(SL_B1.stop, SL_B1.stop + N_H * N_H)
SL_B2 = slice(SL_W2.stop, SL_W2.stop + N_H)
SL_W3 = slice(SL_B2.stop, SL_B2.stop + N_H)
I_B3 = SL_W3.stop
I_MARGIN = I_B3 + 1
N_PARAMS = I_MARGIN + 1
TRAINED = slice(SL_W1.start, I_B3 + 1)
OOD_LIMIT = 6.0


def unpack(blob):
    p = np.asarray(blob, dtype=np.float64)
    assert p.size == N_PARAMS
    scale = p[SL_SCALE].copy()
    scale[scale <= 0] = 1.0
    return dict(mean=p[SL_MEAN], scale=scale, W1=p[SL_W1].reshape(N_H, N_IN), b1=p[SL_B1],
                W2=p[SL_W2].reshape(N_H, N_H), b2=p[SL_B2], w3=p[SL_W3], b3=p[I_B3],
                margin=p[I_MARGIN])


def standardise(blob, X):
    q = unpack(blob)
    return (np.asarray(X, dtype=np.float64) - q["mean"]) / q["scale"]


def forward(blob, X):
    """Network output for each row of X (n x 8)."""
    q = unpack(blob)
    z = standardise(blob, X)
    h1 = np.tanh(z @ q["W1"].T + q["b1"])
    h2 = np.tanh(h1 @ q["W2"].T + q["b2"])
    return h2 @ q["w3"] + q["b3"]


def loss_and_grad(blob, X, T):
    """Sum of squared errors and the gradient of the MEAN squared error
    (1/n) sum (y_s - T_s)^2 with respect to every blob entry (zero for the
    statistics and the margin), by backpropagation."""
    q = unpack(blob)
    n = X.shape[0]
    z = standardise(blob, X)
    h1 = np.tanh(z @ q["W1"].T + q["b1"])
    h2 = np.tanh(h1 @ q["W2"].T + q["b2"])
    y = h2 @ q["w3"] + q["b3"]
    err = y - np.asarray(T, dtype=np.float64)
    dy = 2.0 * err / n                        # d loss / d y
    d2 = np.outer(dy, q["w3"]) * (1.0 - h2 ** 2)   # d loss / d (pre-activation 2)
    d1 = (d2 @ q["W2"]) * (1.0 - h1 ** 2)          # d loss / d (pre-activation 1)
    g = np.zeros(N_PARAMS)
    g[SL_W1] = (d1.T @ z).ravel()
    g[SL_B1] = d1.sum(axis=0)
    g[SL_W2] = (d2.T @ h1).ravel()
    g[SL_B2] = d2.sum(axis=0)
    g[SL_W3] = h2.T @ dy
    g[I_B3] = dy.sum()
    return float(err @ err), g


def adam_step(blob, grad, m, v, lr, t, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t >= 1) on the trained entries; returns new
    (blob, m, v) as float64 arrays."""
    p = np.asarray(blob, dtype=np.float64).copy()
    m = np.asarray(m, dtype=np.float64).copy()
    v = np.asarray(v, dtype=np.float64).copy()
    g = np.asarray(grad, dtype=np.float64)
    sl = TRAINED
    m[sl] = b1 * m[sl] + (1 - b1) * g[sl]
    v[sl] = b2 * v[sl] + (1 - b2) * g[sl] ** 2
    mhat = m[sl] / (1 - b1 ** t)
    vhat = v[sl] / (1 - b2 ** t)
    p[sl] -= lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


# ---------------------------------------------------------------------------
# training data: the target of one logged loop and the safety margin

# an observed residual below this fraction of the target is not trusted
# (it may sit on a rounding floor): it is raised to the fraction first
AFTER_FLOOR = 1e-2
# the observed speed relative to the model is clipped to [0.05, 8]
EFF_MIN, EFF_MAX = 0.05, 8.0


def training_target(res_before, res_after, degree, ln_rho, tol_abs, fp32_loop=False):
    """Target y of one vector in one loop, or None when the record is unusable.

    Eq. (resl) models the residual after a degree-m filter as
    res_before |rho|^-m, so the observed speed relative to the model is
        eff = ln(res_before / res_after') / (m ln|rho|),
    res_after' = max(res_after, AFTER_FLOOR tol_abs); y = ln(clip(eff,
    EFF_MIN, EFF_MAX)).  Loops filtered in FP32 are unusable (the residual
    can stop at FP32's rounding floor, which measures the precision, not the
    polynomial), and so are records without positive finite residuals, a
    degree of at least 1 and a positive ln|rho|.  A residual that grew gives
    a negative eff, which the clip raises to EFF_MIN."""
    if fp32_loop:
        return None
    vals = (res_before, res_after, ln_rho, tol_abs)
    if not all(math.isfinite(v) for v in vals) or degree < 1:
        return None
    if res_after <= 0.0 or res_before <= 0.0 or ln_rho <= 0.0:
        return None
    after = max(res_after, AFTER_FLOOR * tol_abs)
    eff = math.log(res_before / after) / (degree * ln_rho)
    if not math.isfinite(eff):
        return None
    return math.log(min(max(eff, EFF_MIN), EFF_MAX))


def holdout_margin(pred, target, z=3.0):
    """Safety margin of the learned degrees: mean + z * std (population) of
    the held-out prediction errors pred - target, floored at 0.  A larger
    prediction means a faster vector and a lower degree, so the margin
    lowers every prediction by an amount far into the tail of the errors."""
    d = np.asarray(pred, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    if d.size == 0:
        return 0.0
    return max(0.0, float(d.mean() + z * d.std()))


# ---------------------------------------------------------------------------
# features and the learned degree rule

def ritz_gap(mu, j, e):
    """Distance from mu[j] to its nearest neighbour in the ascending block
    (e when the block has one value)."""
    cands = []
    if j > 0:
        cands.append(mu[j] - mu[j - 1])
    if j + 1 < len(mu):
        cands.append(mu[j + 1] - mu[j])
    return min(cands) if cands else e


def features(mu, res, gap, alpha, beta, gamma, norm_h, tol_abs, loop):
    """The 8 inputs of one vector (None when |t| <= 1, no analytic rate):
    f0 = ln(max(res, tol)/tol), f1 = ln ln|rho|, f2 = ln max(f0/ln|rho|, 1/2),
    f3 = ln|t|, f4 = (mu - gamma)/(alpha - gamma), f5 = ln max(gap/e, 1e-12),
    f6 = ln(res/norm_h), f7 = min(loop - 1, 4); t = (mu - c)/e."""
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    t = (mu - c) / e
    if not abs(t) > 1.0:
        return None
    ln_rho = math.log(abs(t) + math.sqrt(t * t - 1.0))   # ln|rho|, |rho| = |t| + sqrt(t^2 - 1)
    f0 = math.log(max(res, tol_abs) / tol_abs)
    return np.array([
        f0,
        math.log(ln_rho),
        math.log(max(f0 / ln_rho, 0.5)),
        math.log(abs(t)),
        (mu - gamma) / (alpha - gamma) if alpha != gamma else 0.0,
        math.log(max(gap / e, 1e-12)),
        math.log(max(res, 1e-300) / norm_h),
        float(min(max(loop - 1, 0), 4)),
    ])


def learned_degrees(blob, mu, res, n_wanted, alpha, beta, gamma, norm_h, tol_abs, loop,
                    deg_max=40, rule=None, y_override=None):
    """Learned degrees of the active block.  `rule` gives the analytic
    degrees (fallback); y_override replaces the network output (to compare
    the decision with another implementation's outputs).  Returns
    (deg, y, src, continuous) with src 0 rule, 1 network, 2 guard fill and
    `continuous` the pre-ceil value m_a exp(margin - y)."""
    q = unpack(blob)
    k = len(mu)
    e = 0.5 * (beta - alpha)
    deg = np.zeros(k, dtype=np.int64)
    src = np.full(k, 2, dtype=np.int64)
    ys = np.full(k, np.nan)
    cont = np.full(k, np.nan)
    rows, feats = [], []
    for j in range(min(n_wanted, k)):
        f = features(mu[j], res[j], ritz_gap(mu, j, e), alpha, beta, gamma, norm_h, tol_abs, loop)
        if f is not None:
            rows.append(j)
            feats.append(f)
    if rows:
        X = np.array(feats)
        y = forward(blob, X) if y_override is None else np.asarray(y_override, float)[rows]
        zs = standardise(blob, X)
        m_a = X[:, 0] / np.exp(X[:, 1])
        use_net = np.all(np.abs(zs) <= OOD_LIMIT, axis=1) & np.isfinite(y)
        # the margin applies only when every wanted vector can finish in this
        # loop (all predicted degrees within deg_max)
        need = np.where(use_net, m_a * np.exp(-np.where(use_net, y, 0.0)), m_a)
        margin = q["margin"] if np.all(np.ceil(need) <= deg_max) else 0.0
        for r, j in enumerate(rows):
            ys[j] = y[r]
            if not use_net[r]:
                deg[j] = rule[j]
                src[j] = 0
                continue
            mc = m_a[r] * math.exp(margin - y[r])
            cont[j] = mc
            # never below the analytic degree
            deg[j] = min(max(int(math.ceil(mc)), 1, int(rule[j])), deg_max)
            src[j] = 1
    fill = int(deg[rows].max()) if rows else deg_max
    deg[src == 2] = fill
    return deg, ys, src, cont
