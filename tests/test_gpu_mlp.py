"""GPU parity of the degree network's kernels (through the C ABI) against
the float64 oracle (oracle/mlp.py): forward pass, mean-squared-error
gradient (several reduction chunks and a ragged tail), Adam, the training
loop, and the learned degree rule; plus the solver's convergence log and
its learned mode (the rule as floor and fallback)."""
import math

import numpy as np
import pytest

import paper_1404_4161_amd as ch
from paper_1404_4161_amd import learned
from oracle import chfsi as ochfsi, eigh, mlp
from workloads import gen

from .gpu_util import dev

pytestmark = pytest.mark.gpu


def _blob(seed, scale=0.3):
    g = np.random.default_rng(seed)
    p = np.zeros(mlp.N_PARAMS)
    p[mlp.SL_MEAN] = g.normal(size=8) * 0.5
    p[mlp.SL_SCALE] = g.uniform(0.5, 2.0, 8)
    p[mlp.TRAINED] = g.normal(size=mlp.TRAINED.stop - mlp.TRAINED.start) * scale
    return p.astype(np.float32)


def _data(n, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(n, 8)).astype(np.float32)
    T = (np.sin(X[:, 0]) + 0.3 * X[:, 1] * X[:, 2]).astype(np.float32)
    return X, T


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("n", [1, 255, 1000])
def test_forward_matches_oracle(n):
    p = _blob(1)
    X, _ = _data(n, 2)
    got = ch.chfsi_mlp_forward(_t(X), _t(p)).cpu().numpy()
    ref = mlp.forward(p.astype(np.float64), X.astype(np.float64))
    assert np.abs(got - ref).max() <= 2e-5 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n", [7, 2048, 4100])
def test_gradient_matches_oracle_and_is_deterministic(n):
    p = _blob(3)
    X, T = _data(n, 4)
    g1, l1 = ch.chfsi_mlp_gradient(_t(X), _t(T), _t(p))
    g2, l2 = ch.chfsi_mlp_gradient(_t(X), _t(T), _t(p))
    assert np.array_equal(g1.cpu().numpy(), g2.cpu().numpy()) and l1 == l2
    sse, gref = mlp.loss_and_grad(p.astype(np.float64), X.astype(np.float64),
                                  T.astype(np.float64))
    g = g1.cpu().numpy()
    assert l1 == pytest.approx(sse, rel=1e-4)
    scale = np.abs(gref).max()
    assert np.abs(g - gref).max() <= 1e-4 * scale, np.abs(g - gref).max() / scale
    assert np.all(g[:16] == 0) and g[-1] == 0


def test_adam_matches_oracle():
    import torch
    p = _blob(5)
    g = np.random.default_rng(6).normal(size=mlp.N_PARAMS).astype(np.float32)
    pd, gd = _t(p), _t(g)
    m = torch.zeros_like(pd)
    v = torch.zeros_like(pd)
    pr, mr, vr = p.astype(np.float64), np.zeros(mlp.N_PARAMS), np.zeros(mlp.N_PARAMS)
    for t in (1, 2, 3):
        ch.chfsi_mlp_adam(pd, gd, m, v, 1e-3, t)
        pr, mr, vr = mlp.adam_step(pr, g.astype(np.float64), mr, vr, 1e-3, t)
    assert np.abs(pd.cpu().numpy() - pr).max() <= 1e-6
    assert np.abs(m.cpu().numpy() - mr).max() <= 1e-6 * np.abs(mr).max()


def test_training_loop_follows_oracle():
    p0 = _blob(7, scale=0.1)
    X, T = _data(600, 8)
    pd = _t(p0)
    steps, lr = 60, 3e-3
    losses = ch.chfsi_mlp_train(_t(X), _t(T), pd, steps, lr)
    pr = p0.astype(np.float64)
    mr = np.zeros(mlp.N_PARAMS)
    vr = np.zeros(mlp.N_PARAMS)
    ref = []
    for t in range(1, steps + 1):
        sse, g = mlp.loss_and_grad(pr, X.astype(np.float64), T.astype(np.float64))
        ref.append(sse / X.shape[0])
        pr, mr, vr = mlp.adam_step(pr, g, mr, vr, lr, t)
    ref = np.array(ref)
    assert np.abs(losses - ref).max() <= 1e-3 * ref[0]
    assert losses[-1] < 0.5 * losses[0]
    final_ref = mlp.loss_and_grad(pr, X.astype(np.float64), T.astype(np.float64))[0]
    final = mlp.loss_and_grad(pd.cpu().numpy().astype(np.float64), X.astype(np.float64),
                              T.astype(np.float64))[0]
    assert final == pytest.approx(final_ref, rel=1e-2)


def _block(k, seed):
    g = np.random.default_rng(seed)
    mu = np.sort(np.concatenate([g.uniform(-24, -11, k - 5), g.uniform(-9, 20, 5)]))
    res = 10.0 ** g.uniform(-9, -1, k)
    return mu, res


def test_learned_degrees_match_oracle():
    k, nw = 90, 70
    mu, res = _block(k, 9)
    alpha, beta, gamma, norm_h, tol_abs = mu[-1], 60.0, mu[0] - 1.0, 60.0, 6e-9
    # statistics of the block's own features keep every input in range
    feats = np.array([f for f in (mlp.features(mu[j], res[j], mlp.ritz_gap(mu, j, 0.5 * (beta - alpha)),
                                               alpha, beta, gamma, norm_h, tol_abs, 2)
                                  for j in range(nw)) if f is not None])
    p = _blob(10, scale=0.2)
    p[mlp.SL_MEAN] = feats.mean(axis=0)
    p[mlp.SL_SCALE] = np.maximum(feats.std(axis=0), 1e-3)
    p[mlp.I_MARGIN] = 0.2
    rule = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol_abs, 40)
    deg, pred, src = ch.chfsi_degrees_learned(mu, res, nw, alpha, beta, gamma, norm_h, tol_abs, 2,
                                              p, deg_max=40)
    rdeg, ry, rsrc, cont = mlp.learned_degrees(p.astype(np.float64), mu, res, nw, alpha, beta,
                                               gamma, norm_h, tol_abs, 2, 40, rule=rule)
    assert np.array_equal(src, rsrc)
    net = src == 1
    assert net.sum() >= 50
    assert np.abs(pred[net] - ry[net]).max() <= 2e-5
    # the same decision wherever rounding cannot move it across an integer
    safe = net & (np.abs(cont - np.round(cont)) > 1e-4 * np.maximum(cont, 1.0))
    safe |= rsrc != 1
    assert safe.sum() >= 0.9 * k
    assert np.array_equal(deg[safe], rdeg[safe])
    # with the GPU's outputs the oracle's rule gives the GPU's degrees exactly
    rdeg2, _, _, _ = mlp.learned_degrees(p.astype(np.float64), mu, res, nw, alpha, beta, gamma,
                                         norm_h, tol_abs, 2, 40, rule=rule,
                                         y_override=pred.astype(np.float64))
    assert np.array_equal(deg, rdeg2)


# ---------------------------------------------------------------------------
# the solver's convergence log and learned mode

def _problem(n=300, nev=16, nex=6, cfg=91):
    conf = gen.small_config("l", n, nev, nex, False, length=1, cfg=cfg)
    seq = gen.Sequence(conf)
    return conf, next(seq.problems())[1]


def test_log_records_are_consistent_with_the_oracle():
    conf, a = _problem()
    log = np.zeros((2000, ch.binding.CHFSI_LOG_FIELDS))
    st, lam, _, info = ch.chfsi_solve(dev(a), None, conf.nev, conf.nex, 1e-10, log=log)
    assert st == 0
    nrec = info["log_records"]
    assert nrec > conf.nev
    rec = log[:nrec]
    for r in rec:
        loop, j, nw, ka = (int(x) for x in r[:4])
        assert 0 <= j < nw <= ka
        assert r[12] >= 1 and np.isfinite(r[14])
        if loop > 1:                                # the first loop uses deg0
            assert r[12] == r[13]
        f = mlp.features(r[4], r[5], r[6], r[7], r[8], r[9], r[10], r[11], loop)
        if f is None:
            assert np.all(np.isnan(r[16:24]))
        else:
            assert np.abs(f - r[16:24]).max() <= 1e-12 * max(1.0, np.abs(f).max())
    # the rule's degrees in the log are the oracle's rule on the same values
    for loop in np.unique(rec[:, 0]):
        blk = rec[rec[:, 0] == loop]
        nw = int(blk[0, 2])
        assert len(blk) == nw   # every wanted position of the loop is logged
        # a wanted vector's degree depends only on its own pair and on the
        # largest wanted degree (for those inside the damped interval)
        rule = ochfsi.degree_rule(blk[:, 4], blk[:, 5], nw, blk[0, 7], blk[0, 8], blk[0, 11], 40)
        assert np.array_equal(rule, blk[:, 13])
    # in the last loop every remaining wanted vector converged
    last = rec[rec[:, 0] == rec[:, 0].max()]
    assert np.all(last[:, 14] <= last[:, 11])
    X, y, keep = learned.targets(rec)
    assert keep.sum() > 0 and np.all(np.isfinite(y))


def _zero_net(scale=1e3, b3=0.0, margin=0.0):
    p = np.zeros(mlp.N_PARAMS, dtype=np.float32)
    p[mlp.SL_SCALE] = scale
    p[mlp.I_B3] = b3
    p[mlp.I_MARGIN] = margin
    return p


def _opts(**kw):
    o = ch.chfsi_default_opts()
    for key, v in kw.items():
        setattr(o, key, v)
    return o


def test_learned_mode_with_a_zero_network_is_the_rule():
    """Output 0 means 'the analytic rate': the learned mode then takes the
    rule's degrees and gives bitwise the same result."""
    conf, a = _problem(cfg=92)
    ad = dev(a)
    st0, lam0, x0, i0 = ch.chfsi_solve(ad, None, conf.nev, conf.nex, 1e-10)
    st2, lam2, x2, i2 = ch.chfsi_solve(ad, None, conf.nev, conf.nex, 1e-10,
                                       opts=_opts(degree_mode=2), mlp=_zero_net())
    assert st0 == st2 == 0
    assert np.array_equal(lam0, lam2)
    assert i0["iters"] == i2["iters"] and i0["matvecs"] == i2["matvecs"]
    assert i2["learned_cols"] > 0 and i2["fallback_cols"] == 0 and i2["learned_raised"] == 0
    # inputs out of the network's range fall back to the rule, same result
    st3, lam3, _, i3 = ch.chfsi_solve(ad, None, conf.nev, conf.nex, 1e-10,
                                      opts=_opts(degree_mode=2), mlp=_zero_net(scale=1e-4))
    assert np.array_equal(lam0, lam3) and i3["learned_cols"] == 0 and i3["fallback_cols"] > 0


def test_rule_is_the_floor_of_learned_degrees():
    """A network that claims 20x the analytic speed would pick far too low
    degrees; the rule's degree is the floor, so the call reproduces the
    rule bitwise.  A network that claims half the speed raises degrees and
    still converges to the oracle's eigenvalues."""
    conf, a = _problem(cfg=93)
    ad = dev(a)
    st0, lam0, _, i0 = ch.chfsi_solve(ad, None, conf.nev, conf.nex, 1e-10)
    st, lam, _, info = ch.chfsi_solve(ad, None, conf.nev, conf.nex, 1e-10,
                                      opts=_opts(degree_mode=2), mlp=_zero_net(b3=3.0))
    assert st == st0 == 0
    assert np.array_equal(lam, lam0) and info["matvecs"] == i0["matvecs"]
    assert info["learned_cols"] > 0 and info["learned_raised"] == 0
    st, lam, _, info = ch.chfsi_solve(ad, None, conf.nev, conf.nex, 1e-10,
                                      opts=_opts(degree_mode=2), mlp=_zero_net(b3=-math.log(2.0)))
    assert st == 0 and info["learned_raised"] > 0
    assert info["filter_matvecs"] > i0["filter_matvecs"] or info["iters"] < i0["iters"]
    ref = eigh.eigvalsh(a)[:conf.nev]
    assert np.abs(lam[:conf.nev] - ref).max() <= 1e-10 * np.abs(ref).min()


def test_jitter_changes_degrees_but_not_the_result():
    conf, a = _problem(cfg=94)
    log = np.zeros((4000, ch.binding.CHFSI_LOG_FIELDS))
    st, lam, _, info = ch.chfsi_solve(dev(a), None, conf.nev, conf.nex, 1e-10,
                                      opts=_opts(degree_jitter=0.5, seed=5), log=log)
    assert st == 0
    rec = log[:info["log_records"]]
    jit = rec[(rec[:, 15].astype(int) & 8) != 0]
    assert len(jit) > 0 and np.any(jit[:, 12] != jit[:, 13])
    ratio = jit[:, 12] / jit[:, 13]
    assert np.all(ratio <= math.exp(0.5) + 1.0) and np.all(ratio >= math.exp(-0.5) - 0.5)
    ref = eigh.eigvalsh(a)[:conf.nev]
    assert np.abs(lam[:conf.nev] - ref).max() <= 1e-10 * np.abs(ref).min()


def test_learned_mode_rejects_missing_or_bad_network():
    conf, a = _problem(n=120, nev=6, nex=3, cfg=95)
    with pytest.raises(ch.ChfsiError) as ei:
        ch.chfsi_solve(dev(a), None, conf.nev, conf.nex, 1e-10, opts=_opts(degree_mode=2))
    assert ei.value.status == ch.binding.CHFSI_INVALID_ARG
    bad = _zero_net()
    bad[100] = np.nan
    with pytest.raises(ch.ChfsiError) as ei:
        ch.chfsi_solve(dev(a), None, conf.nev, conf.nex, 1e-10, opts=_opts(degree_mode=2), mlp=bad)
    assert ei.value.status == ch.binding.CHFSI_NONFINITE
