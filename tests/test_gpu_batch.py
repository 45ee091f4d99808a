"""Batched solves (chfsi_solve_batch): problems of uneven size run their
outer loops in lockstep and share one grouped filter launch per recurrence
step (FP64), or per recurrence step and step form (the mixed-precision
defect filters: FP16-split, BF16-split, FP32).  Every problem must match the
oracle's eigenvalues to 1e-10 and the single-problem solver's to rounding;
graph capture and per-problem defect filters must not change the result;
errors stay per problem."""
import numpy as np
import pytest

import paper_1404_4161_amd as ch
from oracle import chfsi as ochfsi, eigh
from workloads import gen

from .gpu_util import dev, host

pytestmark = pytest.mark.gpu

RTOL = 1e-10
SIZES = [(230, 12, 4, True), (410, 20, 5, False), (333, 16, 4, True), (150, 8, 3, False),
         (520, 26, 6, True)]


def _batch(length=1, delta=1e-2, cfg0=700):
    seqs, probs = [], []
    for q, (n, nev, nex, g) in enumerate(SIZES):
        conf = gen.small_config("b", n, nev, nex, g, length=length, cfg=cfg0 + q, delta=delta)
        seq = gen.Sequence(conf)
        seqs.append(seq)
        probs.append([a.copy() for _, a in seq.problems()])
    return seqs, probs


def _ref(a, b, nev):
    h = a if b is None else ochfsi.reduce_to_standard(a, b)[0]
    return eigh.eigvalsh(h)[:nev]


def _opts(**kw):
    o = ch.chfsi_default_opts()
    for key, v in kw.items():
        setattr(o, key, v)
    return o


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_batch_sequence_matches_oracle_and_single_solves(precision):
    import torch
    seqs, probs = _batch(length=3)
    nevs = [p[1] for p in SIZES]
    nexs = [p[2] for p in SIZES]
    Bs = [dev(s.B) if s.B is not None else None for s in seqs]
    o = _opts(precision=precision)
    x0s = lam0s = None
    sx = [None] * len(SIZES)
    slam = [None] * len(SIZES)
    for l in range(3):
        As = [dev(p[l]) for p in probs]
        st, lams, xs, infos, sts = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10, X0s=x0s,
                                                        Lambda0s=lam0s, opts=o)
        assert st == 0 and sts == [0] * len(SIZES)
        for q, (n, nev, nex, g) in enumerate(SIZES):
            ref = _ref(probs[q][l], seqs[q].B, nev)
            assert np.abs(lams[q][:nev] - ref).max() <= RTOL * np.abs(ref).min(), (l, q)
            assert infos[q]["converged"] == nev
            # the single-problem solver on the same inputs
            st1, lam1, x1, i1 = ch.chfsi_solve(As[q], Bs[q], nev, nex, 1e-10, X0=sx[q],
                                               Lambda0=slam[q], opts=o)
            assert st1 == 0
            assert np.abs(lam1[:nev] - lams[q][:nev]).max() <= 1e-12 * np.abs(ref).min()
            sx[q], slam[q] = x1, lam1
            # vectors: residuals in the original coordinates
            xq = host(xs[q])[:, :nev]
            a = probs[q][l]
            bx = xq if seqs[q].B is None else seqs[q].B @ xq
            r = np.linalg.norm(a @ xq - bx * lams[q][:nev], axis=0)
            bn = 1.0 if seqs[q].B is None else np.sqrt(np.linalg.norm(seqs[q].B, 2))
            assert r.max() <= 2e-10 * infos[q]["norm_h"] * bn
        x0s, lam0s = xs, lams
        torch.cuda.synchronize()


def test_batch_graph_capture_gives_the_same_result():
    import torch
    seqs, probs = _batch(length=1, cfg0=720)
    nevs = [p[1] for p in SIZES]
    nexs = [p[2] for p in SIZES]
    As = [dev(p[0]) for p in probs]
    Bs = [dev(s.B) if s.B is not None else None for s in seqs]
    stream = torch.cuda.Stream()
    r0 = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10, stream=stream)
    r1 = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10, stream=stream, graph=True)
    r2 = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10, stream=stream, serial=True)
    assert r0[0] == r1[0] == r2[0] == 0
    for q in range(len(SIZES)):      # one driving thread: the same arithmetic
        assert np.array_equal(r0[1][q], r2[1][q])
    for q in range(len(SIZES)):
        assert np.array_equal(r0[1][q], r1[1][q])
        assert torch.equal(r0[2][q], r1[2][q])
        assert r0[3][q]["iters"] == r1[3][q]["iters"]


def test_batch_errors_stay_per_problem():
    seqs, probs = _batch(length=1, cfg0=740)
    nevs = [p[1] for p in SIZES]
    nexs = [p[2] for p in SIZES]
    As = [dev(p[0]) for p in probs]
    bad = probs[1][0].copy()
    bad[3, 5] = np.nan
    As[1] = dev(bad)
    Bs = [dev(s.B) if s.B is not None else None for s in seqs]
    st, lams, xs, infos, sts = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10,
                                                    raise_on_error=False)
    assert st == ch.binding.CHFSI_NONFINITE
    assert sts[1] == ch.binding.CHFSI_NONFINITE
    for q in (0, 2, 3, 4):
        assert sts[q] == 0
        ref = _ref(probs[q][0], seqs[q].B, nevs[q])
        assert np.abs(lams[q][:nevs[q]] - ref).max() <= RTOL * np.abs(ref).min()


def test_batch_rejects_bad_arguments():
    import torch
    seqs, probs = _batch(length=1, cfg0=760)
    nevs = [p[1] for p in SIZES][:2]
    nexs = [p[2] for p in SIZES][:2]
    As = [dev(p[0]) for p in probs][:2]
    Bs = [dev(s.B) if s.B is not None else None for s in seqs][:2]
    o = ch.chfsi_default_opts()
    w = torch.empty(max(ch.chfsi_workspace_bytes(a.shape[0], nv, nx, True, o)
                        for a, nv, nx in zip(As, nevs, nexs)), dtype=torch.uint8, device="cuda")
    with pytest.raises(ch.ChfsiError) as ei:      # one workspace for two problems
        ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10, works=[w, w])
    assert ei.value.status == ch.binding.CHFSI_INVALID_ARG
    with pytest.raises(ch.ChfsiError):             # graph capture on the null stream
        ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10, graph=True,
                             stream=torch.cuda.default_stream())


@pytest.mark.parametrize("variant", [1, 3, 4, 5, 6])
def test_batch_with_another_tile_variant(variant):
    """The grouped launch with the 16-deep K stage or the 3M split (forced
    through the autotuner's table) gives the same eigenvalues as the
    default."""
    seqs, probs = _batch(length=1, cfg0=780)
    nevs = [p[1] for p in SIZES]
    nexs = [p[2] for p in SIZES]
    As = [dev(p[0]) for p in probs]
    Bs = [dev(s.B) if s.B is not None else None for s in seqs]
    r0 = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10)
    try:
        for (n, nev, nex, g) in SIZES:
            ch.chfsi_autotune_set(n, nev + nex, variant)
        r1 = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10)
    finally:
        ch.chfsi_autotune_reset()
    for q, (n, nev, nex, g) in enumerate(SIZES):
        ref = _ref(probs[q][0], seqs[q].B, nev)
        assert np.abs(r1[1][q][:nev] - ref).max() <= RTOL * np.abs(ref).min()
        assert np.abs(r1[1][q][:nev] - r0[1][q][:nev]).max() <= 1e-12 * np.abs(ref).min()


@pytest.mark.parametrize("precision", [2, 3])
def test_grouped_defect_filters_match_per_problem_ones(precision):
    """The grouped defect filter (default) against the same batch with each
    problem's defect filter on its own stream (flag bit 2), and both against
    the oracle, along a 3-problem sequence; the split steps did run."""
    seqs, probs = _batch(length=3, cfg0=800)
    nevs = [p[1] for p in SIZES]
    nexs = [p[2] for p in SIZES]
    Bs = [dev(s.B) if s.B is not None else None for s in seqs]
    o = _opts(precision=precision)
    state = {False: (None, None), True: (None, None)}
    for l in range(3):
        As = [dev(p[l]) for p in probs]
        out = {}
        for own in (False, True):
            x0s, lam0s = state[own]
            out[own] = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10, X0s=x0s, Lambda0s=lam0s,
                                            opts=o, own_defect=own)
            assert out[own][0] == 0
            state[own] = (out[own][2], out[own][1])
        key = "filter_steps_bf16" if precision == 2 else "filter_steps_fp16"
        if l > 0:
            assert sum(i[key] for i in out[False][3]) > 0
        for q, (n, nev, nex, g) in enumerate(SIZES):
            ref = _ref(probs[q][l], seqs[q].B, nev)
            for own in (False, True):
                assert np.abs(out[own][1][q][:nev] - ref).max() <= RTOL * np.abs(ref).min()
            assert (np.abs(out[False][1][q][:nev] - out[True][1][q][:nev]).max()
                    <= 1e-12 * np.abs(ref).min())


def test_grouped_defect_filter_with_wide_windows():
    """Two problems with k = 300 (windows of at least 257 columns take the
    128 x 128 tile in the grouped FP16-split launch) and a small one, three
    warm-started problems each, against the oracle and the single solver."""
    import torch
    sizes = [(1200, 280, 20, False), (1100, 270, 30, True), (300, 16, 4, False)]
    seqs, probs = [], []
    for q, (n, nev, nex, g) in enumerate(sizes):
        conf = gen.small_config("w", n, nev, nex, g, length=3, cfg=820 + q, delta=1e-2)
        seq = gen.Sequence(conf)
        seqs.append(seq)
        probs.append([a.copy() for _, a in seq.problems()])
    nevs = [p[1] for p in sizes]
    nexs = [p[2] for p in sizes]
    Bs = [dev(s.B) if s.B is not None else None for s in seqs]
    o = _opts(precision=3)
    x0s = lam0s = None
    sx = [None] * len(sizes)
    slam = [None] * len(sizes)
    for l in range(3):
        print(f"wide grouped defect filter: problem {l + 1}", flush=True)
        As = [dev(p[l]) for p in probs]
        st, lams, xs, infos, sts = ch.chfsi_solve_batch(As, Bs, nevs, nexs, 1e-10, X0s=x0s,
                                                        Lambda0s=lam0s, opts=o)
        assert st == 0
        if l > 0:
            assert sum(i["filter_steps_fp16"] for i in infos) > 0
        for q, (n, nev, nex, g) in enumerate(sizes):
            ref = _ref(probs[q][l], seqs[q].B, nev)
            assert np.abs(lams[q][:nev] - ref).max() <= RTOL * np.abs(ref).min(), (l, q)
            st1, lam1, x1, _ = ch.chfsi_solve(As[q], Bs[q], nev, nex, 1e-10, X0=sx[q],
                                              Lambda0=slam[q], opts=o)
            assert st1 == 0
            assert np.abs(lam1[:nev] - lams[q][:nev]).max() <= 1e-12 * np.abs(ref).min()
            sx[q], slam[q] = x1, lam1
        x0s, lam0s = xs, lams
        torch.cuda.synchronize()
