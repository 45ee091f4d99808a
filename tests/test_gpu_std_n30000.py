"""Full-size checks of the learned-degree workload: the standard n = 30 000
sequence (nev 1500, nex 300, 20 problems, A(l+1) = A(l) + 1e-3 H_l), all
20 problems with the mixed-precision filter and its FP16-split steps
(precision 3) and the degree network (degree_mode 2), and the first three
problems with the paper's FP64 filter and analytic degrees.

The network is trained on the GPU from the logs of two small sequences of
the same recipe; at this size most of its inputs are outside that
training range, so the analytic rule (the floor and fallback of every
learned degree) decides most degrees.  Each problem is generated when it
is solved (only A(1) and the current problem are held).  For every problem,
a certificate over all wanted pairs that holds at any size (torch FP64
products as the checker): every residual ||A x - lam x|| <= 2 tol N_H,
X^H X = I over all k columns and a Kato-Temple bound of 1e-10 relative on
every wanted eigenvalue from the computed gaps; problem 1 also against its
prescribed spectrum (A = Q diag(lam) Q^H) to 1e-10 relative, and the FP64
and mixed+learned eigenvalues of problems 1-3 against each other."""
import dataclasses

import numpy as np
import pytest

import paper_1404_4161_amd as ch
from paper_1404_4161_amd import learned
from workloads import gen

from .gpu_util import certify, check_certificate

pytestmark = pytest.mark.gpu


def _small_network():
    import torch
    buf = learned.LogBuffer(100_000)
    for cfg in (610, 611):
        conf = gen.small_config("lg", 600, 30, 8, False, length=4, cfg=cfg)
        conf = dataclasses.replace(conf, delta=gen._decay(1e-2))
        seq = gen.Sequence(conf, kind="torch", device="cuda:0")
        probs = [a.clone() for _, a in seq.problems()]
        torch.cuda.synchronize()
        for jit in (0.0, 0.3):
            o = ch.chfsi_default_opts()
            o.first_rule, o.degree_jitter, o.seed = 1, jit, cfg
            learned.solve_sequence_logged(probs, None, 30, 8, 1e-10, o, buf)
    blob, _ = learned.fit(buf.records(), steps=800)
    return blob


def _run(seq, conf, opts, count, blob=None):
    import torch
    nev, nex = conf.nev, conf.nex
    x, lam, lams = None, None, []
    for l, a in seq.problems(count):
        torch.cuda.synchronize()
        print(f"std-n30000 problem {l}: solving (precision {opts.precision}, degree mode "
              f"{opts.degree_mode})", flush=True)
        st, lam, xd, info = ch.chfsi_solve(a, None, nev, nex, conf.tol, X0=x,
                                           Lambda0=lam if x is not None else None, opts=opts,
                                           mlp=blob)
        assert st == 0, (l, st)
        print(f"  iters {info['iters']} fp32 loops {info['filter_iters_fp32']} fp16 steps "
              f"{info['filter_steps_fp16']} learned/fallback cols {info['learned_cols']}/"
              f"{info['fallback_cols']} {info['total_seconds']:.2f}s", flush=True)
        if l == 1:
            ref = np.asarray(seq.lam[:nev])
            err = np.abs(lam[:nev] - ref) / np.abs(ref)
            assert err.max() <= 1e-10, err.max()
        check_certificate(certify(a, None, lam, xd, nev, conf.tol, info["norm_h"]),
                          f"problem {l}")
        lams.append(lam[:nev].copy())
        x = xd
        del a
    return lams


@pytest.mark.timeout(800)
def test_std_n30000_sequence_certified():
    import torch
    blob = _small_network()
    conf = gen.CONFIGS["std-n30000"]
    seq = gen.Sequence(conf, kind="torch", device="cuda:0", draw="device")
    torch.cuda.synchronize()
    opts = ch.chfsi_default_opts()
    opts.precision, opts.degree_mode = 3, 2
    mixed = _run(seq, conf, opts, conf.length, blob)
    assert len(mixed) == conf.length
    opts = ch.chfsi_default_opts()
    fp64 = _run(seq, conf, opts, 3)
    for l, (a, b) in enumerate(zip(fp64, mixed), start=1):
        err = float(np.max(np.abs(a - b) / np.abs(a)))
        print(f"problem {l}: max rel diff FP64 vs mixed+learned {err:.1e}", flush=True)
        assert err <= 1e-10, (l, err)
