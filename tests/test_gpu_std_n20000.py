"""Full-size checks of the standard n = 20 000 workload (nev 1000, nex 200,
six problems, A(l+1) = A(l) + 1e-3 H_l) in the benchmark's launch path:
every problem of the sequence with the paper's FP64 filter and with the
mixed-precision filter with FP16-split steps (precision 3), and the first
two problems with BF16-split steps (precision 2).

For every problem, a certificate over all wanted pairs that holds at any
size (torch FP64 products as the checker): every residual
||A x - lam x|| <= 2 tol N_H, X^H X = I over all k columns, and a
Kato-Temple bound of 1e-10 relative on every wanted eigenvalue from the
computed gaps.  Besides: problem 1 against its prescribed spectrum
(A = Q diag(lam) Q^H, exact eigenvalues known), and problems 1 and 2
against the CPU oracle's eigenvalues for the same host draws
(tests/golden/std_n20000_eigs.txt, written by make_std_n20000.py with the
oracle and certified there by a Sylvester inertia count), to 1e-10
relative."""
import os

import numpy as np
import pytest

import paper_1404_4161_amd as ch
from workloads import gen

from .gpu_util import certify, check_certificate

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "std_n20000_eigs.txt")


def _golden():
    data = np.loadtxt(GOLDEN)
    return {int(l): data[data[:, 0] == l][:, 2] for l in np.unique(data[:, 0])}


@pytest.fixture(scope="module")
def seq20k():
    import torch
    conf = gen.CONFIGS["std-n20000"]
    print("std-n20000: generating problem 1 from host draws", flush=True)
    seq = gen.Sequence(conf, kind="torch", device="cuda:0", draw="host")
    torch.cuda.synchronize()
    return conf, seq


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision,count", [(0, 6), (3, 6), (2, 2)])
def test_std_n20000_sequence_certified(precision, count, seq20k):
    import torch
    conf, seq = seq20k
    golden = _golden()
    assert sorted(golden) == [1, 2]
    opts = ch.chfsi_default_opts()
    opts.precision = precision
    nev, nex = conf.nev, conf.nex
    x, lam = None, None
    for l, a in seq.problems(count):
        torch.cuda.synchronize()
        print(f"std-n20000 problem {l}: solving (precision {precision})", flush=True)
        st, lam, xd, info = ch.chfsi_solve(a, None, nev, nex, conf.tol, X0=x,
                                           Lambda0=lam if x is not None else None, opts=opts)
        assert st == 0, (l, st)
        print(f"  iters {info['iters']} fp32 loops {info['filter_iters_fp32']} bf16/fp16 steps "
              f"{info['filter_steps_bf16']}/{info['filter_steps_fp16']} rr refined/dense "
              f"{info['rr_refined']}/{info['rr_dense']} {info['total_seconds']:.2f}s", flush=True)
        if l == 1:
            ref = np.asarray(seq.lam[:nev])
            err = np.abs(lam[:nev] - ref) / np.abs(ref)
            assert err.max() <= 1e-10, err.max()
        if l in golden:
            err = np.abs(lam[:nev] - golden[l]) / np.abs(golden[l])
            print(f"  max rel diff vs oracle {err.max():.2e}", flush=True)
            assert err.max() <= 1e-10, (l, err.max())
        if l > 1 and precision:
            assert info["filter_steps_bf16" if precision == 2 else "filter_steps_fp16"] > 0
        check_certificate(certify(a, None, lam, xd, nev, conf.tol, info["norm_h"]),
                          f"problem {l}")
        x = xd
        del a
