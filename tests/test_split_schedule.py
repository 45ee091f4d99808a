"""The per-step split schedule of the mixed-precision defect filter (host
logic of the library, no GPU): which recurrence steps run with BF16 words
(precision 2) or FP16 words of scaled operands (precision 3).  Rule (eq.
resl applied to one step's rounding): step i may be split when, for every
wanted vector j still filtered (deg_j > i), the split's error eps rel_j,
damped by the deg_j - i - 1 steps after it (|rho_j|^-(deg_j - i - 1)),
stays 10x below max(tol, rel_j |rho_j|^-deg_j)."""
import ctypes
import math

import numpy as np
import pytest

import paper_1404_4161_amd as ch

EPS = {1: 3.0 * 2.0 ** -16, 2: 3.0 * 2.0 ** -22}


def _rule(mu, res, deg, n_wanted, c, e, tol, norm_h, form):
    out = np.full(max(deg), form, dtype=np.int64)
    out[0] = 0
    for j in range(min(n_wanted, len(deg))):
        t = (mu[j] - c) / e
        rho = abs(t) + math.sqrt(t * t - 1.0) if abs(t) > 1.0 else 1.0
        rel = res[j] / norm_h
        target = max(tol, rel * rho ** -deg[j])
        for i in range(1, deg[j]):
            if not (10.0 * EPS[form] * rel * rho ** -(deg[j] - i - 1) <= target):
                out[i] = 0
    return out


def test_single_column_worked_case():
    # t = 3: |rho| = 3 + sqrt(8); rel 1e-6, tol 1e-10, degree 10.  BF16:
    # 10 eps rel |rho|^-(9 - i) <= 1e-10 needs 9 - i >= ln(4.58) / ln|rho|
    # = 0.86, so steps 1..8 are split and the last one (9) is not.  FP16:
    # 10 eps rel = 7.2e-12 <= 1e-10 already undamped: every step.
    mu, res, deg = [3.0], [1e-6], [10]
    bf = ch.chfsi_split_schedule(mu, res, deg, 1, 0.0, 1.0, 1e-10, 1.0, 1)
    h = ch.chfsi_split_schedule(mu, res, deg, 1, 0.0, 1.0, 1e-10, 1.0, 2)
    assert bf.tolist() == [0, 1, 1, 1, 1, 1, 1, 1, 1, 0]
    assert h.tolist() == [0] + [2] * 9


def test_schedule_follows_the_rule_and_fp16_admits_more():
    g = np.random.default_rng(11)
    for trial in range(300):
        ka = int(g.integers(1, 30))
        n_wanted = int(g.integers(0, ka + 1))
        c, e = 20.0, 15.0
        mu = np.sort(g.uniform(-20.0, 30.0, ka))
        res = 10.0 ** g.uniform(-13, -1, ka)
        deg = g.integers(1, 41, ka).tolist()
        norm_h = 40.0
        tol = 10.0 ** g.uniform(-12, -8)
        sets = {}
        for form in (1, 2):
            got = ch.chfsi_split_schedule(mu, res, deg, n_wanted, c, e, tol, norm_h, form)
            want = _rule(mu, res, deg, n_wanted, c, e, tol, norm_h, form)
            assert got.tolist() == want.tolist(), (trial, form)
            sets[form] = got > 0
        # the FP16 words' error bound is 64x smaller: never fewer split steps
        assert np.all(sets[2] >= sets[1]), trial


def test_invalid_arguments():
    lib = ch.lib()
    d = (ctypes.c_double * 2)(1.0, 2.0)
    ok = (ctypes.c_int * 2)(3, 4)
    bad = (ctypes.c_int * 2)(0, 4)
    out = (ctypes.c_byte * 8)()
    inv = ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_split_schedule(2, 2, d, d, ok, 0.0, 1.0, 1e-10, 1.0, 3, out) == inv
    assert lib.chfsi_split_schedule(2, 2, d, d, bad, 0.0, 1.0, 1e-10, 1.0, 1, out) == inv
    assert lib.chfsi_split_schedule(2, 2, d, d, ok, 0.0, 0.0, 1e-10, 1.0, 1, out) == inv
    assert lib.chfsi_split_schedule(2, 0, d, d, ok, 0.0, 1.0, 1e-10, 1.0, 1, out) == inv
    assert lib.chfsi_split_schedule(2, 2, d, d, ok, 0.0, 1.0, 1e-10, 1.0, 2, None) == inv
    assert lib.chfsi_split_schedule(2, 2, d, d, ok, 0.0, 1.0, 1e-10, 1.0, 2, out) == 0
