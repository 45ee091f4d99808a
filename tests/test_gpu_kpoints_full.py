"""Full-size check of the batched k-point workload: 32 generalized problems
with n uniform in [2000, 9000] (nev 5 %, nex 1 % of n, B = I + 0.05 G,
perturbations 1e-2 0.5^l), solved in one lockstep batch per step as the
benchmark runs them: all five steps with the paper's FP64 filter and with
the mixed-precision filter and its FP16-split steps (precision 3), the
first two with BF16-split steps (precision 2).

Every problem of every step gets a certificate over all its wanted pairs
that holds at any size (torch FP64 products as the checker): residuals
||A x - lam B x|| <= 2 tol N_H ||B|| (||B|| <= 1.05), X^H B X = I over all
k columns, and a Kato-Temple bound of 1e-10 relative on every wanted
eigenvalue from the computed gaps.  (B moves the spectrum away from the
prescribed one, so the first step has no known eigenvalues; the small-size batch tests compare the same path element by element with
the oracle.)"""
import numpy as np
import pytest

import paper_1404_4161_amd as ch
from workloads import gen

from .gpu_util import certify, check_certificate

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,steps", [(0, 5), (3, 5), (2, 2)])
def test_kpoints_full_size_batched_certified(precision, steps):
    import torch
    confs = gen.kpoint_configs()
    seqs = [gen.Sequence(c, kind="torch", device="cuda:0", draw="device") for c in confs]
    gens = [s.problems() for s in seqs]
    Bs = [s.B for s in seqs]
    opts = ch.chfsi_default_opts()
    opts.precision = precision
    x0s = lam0s = None
    for step in range(1, steps + 1):
        As = [next(g)[1] for g in gens]
        torch.cuda.synchronize()
        print(f"k-points step {step}: solving {len(As)} problems (precision {precision})",
              flush=True)
        st, lams, Xs, infos, sts = ch.chfsi_solve_batch(
            As, Bs, [c.nev for c in confs], [c.nex for c in confs], 1e-10, X0s=x0s,
            Lambda0s=lam0s, opts=opts)
        assert st == 0 and all(s == 0 for s in sts), sts
        if step > 1 and precision:
            w = "filter_steps_bf16" if precision == 2 else "filter_steps_fp16"
            assert sum(i[w] for i in infos) > 0
        worst = {"resid_ratio": 0.0, "orth": 0.0, "kato_temple_rel_max": 0.0}
        for q, c in enumerate(confs):
            cert = certify(As[q], Bs[q], lams[q], Xs[q], c.nev, 1e-10, infos[q]["norm_h"],
                           b_norm=1.05)
            assert cert["resid_ratio"] <= 1.0, (step, q, cert)
            assert cert["orth"] <= 1e-12, (step, q, cert)
            assert cert["no_kt_bound"] == 0 and cert["kato_temple_rel_max"] <= 1e-10, \
                (step, q, cert)
            for kk in worst:
                worst[kk] = max(worst[kk], cert[kk])
        check_certificate(dict(worst, no_kt_bound=0, resid_max=0.0, resid_bound=0.0),
                          f"step {step} (worst of {len(confs)} problems)")
        x0s, lam0s = Xs, lams
        del As
