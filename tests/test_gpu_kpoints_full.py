"""Full-size check of the batched k-point workload: 32 generalized problems
with n uniform in [2000, 9000] (nev 5 %, nex 1 % of n), solved in one
lockstep batch with the mixed-precision filter and its BF16-split steps
(precision 2) or FP16-split steps (precision 3), the cold first step and
one warm-started step, as the benchmark runs them.  Checked by properties that hold at any size: every
problem converges; sampled pairs have residuals ||A x - lam B x|| <= 2 tol
N_H ||B|| (||B|| <= 1.05 for B = I + 0.05 G) and B-orthonormal vectors.
(The small-size batch tests compare the same path element by element with
the oracle.)"""
import numpy as np
import pytest

import paper_1404_4161_amd as ch
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [2, 3])
def test_kpoints_full_size_batched_split_steps(precision):
    import torch
    confs = gen.kpoint_configs()
    seqs = [gen.Sequence(c, kind="torch", device="cuda:0", draw="device") for c in confs]
    gens = [s.problems() for s in seqs]
    Bs = [s.B for s in seqs]
    opts = ch.chfsi_default_opts()
    opts.precision = precision
    x0s = lam0s = None
    for step in (1, 2):
        As = [next(g)[1] for g in gens]
        torch.cuda.synchronize()
        print(f"k-points step {step}: solving {len(As)} problems", flush=True)
        st, lams, Xs, infos, sts = ch.chfsi_solve_batch(
            As, Bs, [c.nev for c in confs], [c.nex for c in confs], 1e-10, X0s=x0s,
            Lambda0s=lam0s, opts=opts)
        assert st == 0 and all(s == 0 for s in sts), sts
        if step == 2:
            w = "filter_steps_bf16" if precision == 2 else "filter_steps_fp16"
            assert sum(i[w] for i in infos) > 0
        worst_r = worst_o = 0.0
        for q, c in enumerate(confs):
            cols = [0, c.nev // 2, c.nev - 1]
            xs = Xs[q][:, cols]
            lam = torch.as_tensor(lams[q][cols], device=xs.device)
            bx = Bs[q] @ xs
            r = torch.linalg.norm(As[q] @ xs - bx * lam, dim=0).cpu().numpy()
            bound = 2 * 1e-10 * infos[q]["norm_h"] * 1.05
            assert r.max() <= bound, (step, q, r, bound)
            gram = (xs.conj().transpose(0, 1) @ bx).cpu().numpy()
            orth = np.abs(gram - np.eye(len(cols))).max()
            assert orth <= 1e-12, (step, q, orth)
            worst_r = max(worst_r, r.max() / bound)
            worst_o = max(worst_o, orth)
        print(f"  worst residual / bound {worst_r:.2e}, worst B-orthonormality {worst_o:.1e}",
              flush=True)
        x0s, lam0s = Xs, lams
        del As
