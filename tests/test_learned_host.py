"""The product's training-data path against the oracle's definitions (CPU).

paper_1404_4161_amd.learned turns the solver's convergence records into
training targets and sets the safety margin from held-out errors; the
oracle (oracle.mlp.training_target, oracle.mlp.holdout_margin) writes the
same quantities from eq. (resl)'s model.  Records are built by hand in the
library's record layout with rates known exactly, plus random ones."""
import math

import numpy as np
import pytest

from oracle import mlp
from paper_1404_4161_amd import learned as L


def _record(res, after, deg, ln_rho, tol, fp32=False, feats_ok=True):
    r = np.zeros(L.F)
    r[L.R_RES], r[L.R_AFTER], r[L.R_DEG], r[L.R_TOL] = res, after, deg, tol
    r[L.R_FLAGS] = 1.0 if fp32 else 0.0
    f = np.linspace(0.1, 0.8, 8)
    f[1] = math.log(ln_rho)                  # f1 = ln ln|rho|
    if not feats_ok:
        f[5] = np.nan
    r[L.R_FEAT:L.R_FEAT + 8] = f
    return r


def _oracle_targets(recs):
    keep, ys = [], []
    for r in recs:
        feats = r[L.R_FEAT:L.R_FEAT + 8]
        y = None
        if np.all(np.isfinite(feats)):
            y = mlp.training_target(r[L.R_RES], r[L.R_AFTER], r[L.R_DEG],
                                    math.exp(feats[1]), r[L.R_TOL],
                                    fp32_loop=bool(int(r[L.R_FLAGS]) & 1))
        keep.append(y is not None)
        if y is not None:
            ys.append(y)
    return np.array(keep), np.array(ys)


def _hand_records():
    tol = 4e-9
    recs = []
    for eff in (0.05, 0.3, 1.0, 2.5, 4.0):
        res, m, lr = 2e-4, 7, 0.3
        recs.append(_record(res, res * math.exp(-eff * m * lr), m, lr, tol))
    recs += [
        _record(1e-3, 1e-30, 6, 0.25, tol),               # floored, then clipped at 8
        _record(1e-3, 3e-11, 6, 0.25, tol),               # just above the floor
        _record(1e-3, 5e-3, 4, 0.2, tol),                 # grew: clipped at 0.05
        _record(1e-3, 1e-6, 5, 0.2, tol, fp32=True),      # FP32 loop: left out
        _record(1e-3, 1e-6, 5, 0.2, tol, feats_ok=False), # no features: left out
        _record(1e-3, 0.0, 5, 0.2, tol),                  # no residual after: left out
        _record(1e-3, 1e-6, 0, 0.2, tol),                 # no degree: left out
    ]
    return np.array(recs)


def test_targets_match_the_oracle_on_hand_built_records():
    recs = _hand_records()
    X, y, ok = L.targets(recs)
    keep, ys = _oracle_targets(recs)
    assert ok.tolist() == keep.tolist()
    assert np.abs(y.astype(np.float64) - ys).max() < 1e-6        # float32 targets
    # the exact rates come back
    assert np.allclose(ys[:5], np.log([0.05, 0.3, 1.0, 2.5, 4.0]), atol=1e-12)
    assert X.shape == (int(keep.sum()), 8)


def test_targets_match_the_oracle_on_random_records():
    g = np.random.default_rng(5)
    recs = []
    for _ in range(400):
        res = 10 ** g.uniform(-9, -1)
        after = res * 10 ** g.uniform(-9, 1)
        recs.append(_record(res, after, int(g.integers(0, 41)), g.uniform(0.01, 2.0),
                            10 ** g.uniform(-12, -8), fp32=bool(g.random() < 0.2),
                            feats_ok=bool(g.random() > 0.1)))
    recs = np.array(recs)
    _, y, ok = L.targets(recs)
    keep, ys = _oracle_targets(recs)
    assert ok.tolist() == keep.tolist()
    assert np.abs(y.astype(np.float64) - ys).max() < 1e-5


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_holdout_margin_matches_the_oracle(seed):
    g = np.random.default_rng(seed)
    pred, y = g.normal(size=300), g.normal(size=300) * 0.7 + 0.1
    assert L.holdout_margin(pred, y) == pytest.approx(mlp.holdout_margin(pred, y), rel=1e-14)
    assert L.holdout_margin(pred, y, z=1.0) == pytest.approx(mlp.holdout_margin(pred, y, z=1.0),
                                                             rel=1e-14)
    assert L.holdout_margin(y - 5.0, y) == mlp.holdout_margin(y - 5.0, y) == 0.0
