"""Full-size check of the learned-degree workload: the standard n = 30 000
problem (nev 1500, nex 300) with the mixed-precision filter and its
FP16-split steps (precision 3) and the degree network (degree_mode 2),
cold first problem and one warm-started problem.  The network is trained on the GPU from the logs of
two small sequences of the same recipe; at this size most of its inputs
are outside that training range, so the analytic rule (the floor and
fallback of every learned degree) decides most degrees -- which is what
the test checks besides the results: the first problem's eigenvalues
against the prescribed spectrum (A = Q diag(lam) Q^H, exact eigenvalues
known) to 1e-10 relative, and for both problems residuals of sampled pairs
<= 2 tol N_H with orthonormal vectors."""
import dataclasses

import numpy as np
import pytest

import paper_1404_4161_amd as ch
from paper_1404_4161_amd import learned
from workloads import gen

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


@pytest.mark.timeout(1200)
def test_std_n30000_mixed_learned_first_two_problems():
    import torch
    blob = _small_network()
    conf = gen.CONFIGS["std-n30000"]
    seq = gen.Sequence(conf, kind="torch", device="cuda:0", draw="device")
    problems = seq.problems()
    opts = ch.chfsi_default_opts()
    opts.precision, opts.degree_mode = 3, 2
    nev, nex = conf.nev, conf.nex
    x, lam = None, None
    for l in (1, 2):
        _, a = next(problems)
        torch.cuda.synchronize()
        print(f"std-n30000 problem {l}: solving (precision 3, learned degrees)", flush=True)
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
        cols = [0, nev // 2, nev - 1]
        xs = xd[:, cols]
        r = torch.linalg.norm(a @ xs - xs * torch.as_tensor(lam[cols], device=xs.device),
                              dim=0).cpu().numpy()
        assert r.max() <= 2 * conf.tol * info["norm_h"], (l, r)
        gram = (xs.conj().transpose(0, 1) @ xs).cpu().numpy()
        assert np.abs(gram - np.eye(len(cols))).max() <= 1e-12
        x = xd
        del a
