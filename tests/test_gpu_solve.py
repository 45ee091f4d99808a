"""GPU parity of chfsi_solve (through the C ABI) against the CPU oracle:
eigenvalues to 1e-10 relative on the same seeded inputs, residuals and
B-orthonormality of the vectors, warm-started sequences, edge cases and
error paths."""
import numpy as np
import pytest

import paper_1404_4161_amd as ch
from oracle import chfsi as ochfsi, eigh
from workloads import gen

from .gpu_util import dev, host

pytestmark = pytest.mark.gpu

RTOL = 1e-10


def _opts(**kw):
    o = ch.chfsi_default_opts()
    for key, v in kw.items():
        setattr(o, key, v)
    return o


def _check_pairs(a, b, lam, x, nev, tol, norm_h):
    """Residuals of the returned pairs in the original coordinates and
    B-orthonormality of X."""
    xb = x if b is None else b @ x
    r = np.linalg.norm(a @ x[:, :nev] - xb[:, :nev] * lam[:nev], axis=0)
    if b is None:
        assert r.max() <= 2 * tol * norm_h
    else:
        # ||A x - lam B x|| <= ||L|| ||H y - lam y||, ||L|| <= sqrt(||B||)
        assert r.max() <= 2 * tol * norm_h * np.sqrt(np.linalg.norm(b, 2))
    g = x.conj().T @ xb
    assert np.abs(g - np.eye(x.shape[1])).max() < 1e-11


@pytest.mark.parametrize("n,nev,nex,generalized", [(150, 8, 3, False), (333, 20, 6, False),
                                                   (260, 12, 4, True)])
def test_solve_small_matches_oracle(n, nev, nex, generalized):
    conf = gen.small_config("s", n, nev, nex, generalized, length=1, cfg=60 + n)
    seq = gen.Sequence(conf)
    a = next(seq.problems())[1]
    ref = ochfsi.chfsi(a, nev, nex, b=seq.B)
    st, lam, xd, info = ch.chfsi_solve(dev(a), dev(seq.B) if generalized else None, nev, nex, 1e-10)
    assert st == 0 and ref.status == 0
    assert np.abs(lam[:nev] - ref.lam[:nev]).max() <= RTOL * np.abs(ref.lam[:nev]).min()
    assert info["converged"] == nev
    assert info["norm_h"] == pytest.approx(ref.norm_h, rel=1e-9)
    _check_pairs(a, seq.B, lam, host(xd), nev, 1e-10, info["norm_h"])
    if not generalized:
        assert np.abs(lam[:nev] - seq.lam[:nev]).max() <= RTOL * np.abs(seq.lam[:nev]).min()


def test_solve_std_n1000_sequence_warm_start():
    """The n = 1000 standard workload: 4 problems, each warm-started from the
    previous Ritz vectors, against the oracle on the same inputs."""
    conf = gen.CONFIGS["std-n1000"]
    seq = gen.Sequence(conf)
    probs = [a.copy() for _, a in seq.problems()]
    refs = ochfsi.solve_sequence(probs, conf.nev, conf.nex)
    x = None
    iters, refined = [], []
    for l, (a, ref) in enumerate(zip(probs, refs)):
        st, lam, xd, info = ch.chfsi_solve(dev(a), None, conf.nev, conf.nex, conf.tol, X0=x)
        assert st == 0
        assert np.abs(lam[:conf.nev] - ref.lam[:conf.nev]).max() <= \
            RTOL * np.abs(ref.lam[:conf.nev]).min()
        _check_pairs(a, None, lam, host(xd), conf.nev, conf.tol, info["norm_h"])
        iters.append(info["matvecs"])
        refined.append((info["rr_refined"], info["rr_dense"]))
        x = xd
    lam1 = seq.lam[:conf.nev]
    assert np.abs(refs[0].lam[:conf.nev] - lam1).max() <= RTOL * np.abs(lam1).min()
    # warm starts need far fewer mat-vecs than the cold first problem (Sec. 4.2)
    assert max(iters[1:]) < 0.5 * iters[0]
    # the cold start's first Rayleigh-Ritz needs the dense eigensolver; in
    # the warm-started problems the projected matrices are nearly diagonal
    assert refined[0][1] >= 1
    assert all(r > 0 for r, _ in refined[1:]), refined


def test_solve_generalized_sequence_against_dense_oracle():
    conf = gen.small_config("g", 400, 20, 6, True, length=3, cfg=71, delta=1e-2)
    seq = gen.Sequence(conf)
    x = None
    for l, a in seq.problems():
        st, lam, xd, info = ch.chfsi_solve(dev(a), dev(seq.B), conf.nev, conf.nex, 1e-10, X0=x)
        assert st == 0
        h, _ = ochfsi.reduce_to_standard(a, seq.B)
        ref = eigh.eigvalsh(h)[:conf.nev]
        assert np.abs(lam[:conf.nev] - ref).max() <= RTOL * np.abs(ref).min()
        _check_pairs(a, seq.B, lam, host(xd), conf.nev, 1e-10, info["norm_h"])
        x = xd


def test_solve_x_aliases_x0_and_is_repeatable():
    conf = gen.small_config("r", 300, 10, 5, False, length=2, cfg=80)
    probs = [a.copy() for _, a in gen.Sequence(conf).problems()]
    ad = dev(probs[0])
    st, lam1, x1, _ = ch.chfsi_solve(ad, None, 10, 5, 1e-10)
    st2, lam2, x2, _ = ch.chfsi_solve(ad, None, 10, 5, 1e-10)
    assert st == st2 == 0
    assert np.array_equal(lam1, lam2)                 # bitwise repeatable
    assert np.array_equal(host(x1), host(x2))
    # warm start in place: X0 and X are the same buffer
    a2 = dev(probs[1])
    st3, lam3, x3, _ = ch.chfsi_solve(a2, None, 10, 5, 1e-10, X0=x1, X=x1)
    assert st3 == 0 and x3.data_ptr() == x1.data_ptr()
    ref = ochfsi.chfsi(probs[1], 10, 5)
    assert np.abs(lam3[:10] - ref.lam[:10]).max() <= RTOL * np.abs(ref.lam[:10]).min()


@pytest.mark.parametrize("precision,rr_refine", [(0, 1), (2, 1), (3, 1), (0, 0)])
def test_solve_edge_cases_tiny_and_full_block(precision, rr_refine):
    o = _opts(precision=precision, rr_refine=rr_refine)
    # tiny: n = 6, k = n (the subspace is the whole space)
    lamv = np.array([-3.0, -1.0, 0.5, 2.0, 4.0, 9.0])
    a = gen.prescribed_problem(6, lamv, 3)
    st, lam, xd, info = ch.chfsi_solve(dev(a), None, 4, 2, 1e-10, opts=o)
    assert st == 0
    assert np.abs(lam - lamv).max() < 1e-12
    # n not a multiple of the tile, k = n - 1
    lamv = np.linspace(-5, 5, 65)
    a = gen.prescribed_problem(65, lamv, 4)
    st, lam, xd, info = ch.chfsi_solve(dev(a), None, 60, 4, 1e-10, opts=o)
    assert st == 0
    assert np.abs(lam[:60] - lamv[:60]).max() < 1e-10 * 5
    # a warm start of the same problem (nearly diagonal projected matrices)
    st, lam2, _, info = ch.chfsi_solve(dev(a), None, 60, 4, 1e-10, X0=xd, Lambda0=lam, opts=o)
    assert st == 0
    assert np.abs(lam2[:60] - lamv[:60]).max() < 1e-10 * 5
    if rr_refine == 0:
        assert info["rr_refined"] == 0


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_solve_degenerate_and_clustered_spectrum(precision):
    """Exactly repeated eigenvalues (multiplicity 4 at the bottom, 3 at the
    edge of the wanted set, a pair split across nev) and a tight cluster:
    the eigenvalues match the prescribed spectrum, and the returned vectors
    of a repeated eigenvalue span its eigenspace (residuals + B-orthonormality)."""
    n, nev, nex = 300, 20, 6
    g = np.random.default_rng(17)
    lamv = np.sort(np.concatenate([
        [-20.0] * 4,                       # multiplicity 4 at the bottom
        np.linspace(-19.5, -17.0, 11),
        [-16.5] * 3,                       # multiplicity 3 inside the wanted set
        [-16.0, -16.0],                    # a pair split by nev (indices 19, 20)
        -15.9 + 1e-9 * np.arange(4),       # a cluster 1e-9 wide
        g.uniform(-14.0, 30.0, n - 24)]))
    a = gen.prescribed_problem(n, lamv, 18)
    opts = _opts(precision=precision)
    st, lam, xd, info = ch.chfsi_solve(dev(a), None, nev, nex, 1e-10, opts=opts)
    assert st == 0
    assert np.abs(lam[:nev] - lamv[:nev]).max() <= RTOL * np.abs(lamv[:nev]).min()
    _check_pairs(a, None, lam, host(xd), nev, 1e-10, info["norm_h"])
    # the 4-fold eigenspace is spanned: A = Q diag(lamv) Q^H, so it is the
    # span of the first 4 columns of the generator's Q
    x4 = host(xd)[:, :4]
    q = gen._NumpyBackend().qr_unitary(gen.complex_gaussian(
        np.random.Generator(np.random.PCG64(18)), n, n))
    u4 = q[:, :4]
    assert np.abs(u4 @ (u4.conj().T @ x4) - x4).max() < 1e-8
    # warm start on the same matrix: the projected matrices are nearly
    # diagonal with exactly repeated diagonal groups (refinement path)
    st, lam2, xd2, info2 = ch.chfsi_solve(dev(a), None, nev, nex, 1e-10, X0=xd, Lambda0=lam,
                                          opts=opts)
    assert st == 0
    assert np.abs(lam2[:nev] - lamv[:nev]).max() <= RTOL * np.abs(lamv[:nev]).min()
    _check_pairs(a, None, lam2, host(xd2), nev, 1e-10, info2["norm_h"])
    assert info2["rr_refined"] >= 1


def test_solve_fixed_degree_and_literal_alpha_modes():
    conf = gen.small_config("m", 250, 10, 4, False, length=1, cfg=90)
    a = next(gen.Sequence(conf).problems())[1]
    ref = ochfsi.chfsi(a, 10, 4)
    for kw in [dict(degree_mode=1, deg0=12), dict(alpha_rule=1)]:
        st, lam, xd, info = ch.chfsi_solve(dev(a), None, 10, 4, 1e-10, opts=_opts(**kw))
        assert st == 0, kw
        assert np.abs(lam[:10] - ref.lam[:10]).max() <= RTOL * np.abs(ref.lam[:10]).min()


def test_solve_error_paths():
    conf = gen.small_config("e", 120, 6, 2, False, length=1, cfg=91)
    a = next(gen.Sequence(conf).problems())[1]
    st, lam, xd, info = ch.chfsi_solve(dev(a), None, 6, 2, 1e-10, opts=_opts(max_iter=1),
                                       raise_on_error=False)
    assert st == ch.binding.CHFSI_NO_CONVERGENCE
    assert info["converged"] < 6 and np.all(np.isfinite(lam))
    bad = a.copy()
    bad[5, 7] = np.inf
    st, *_ = ch.chfsi_solve(dev(bad), None, 6, 2, 1e-10, raise_on_error=False)
    assert st == ch.binding.CHFSI_NONFINITE
    b = np.eye(120, dtype=complex)
    b[100, 100] = -2.0
    st, *_ = ch.chfsi_solve(dev(a), dev(b), 6, 2, 1e-10, raise_on_error=False)
    assert st == ch.binding.CHFSI_NOT_HPD
    x0 = gen.random_block(120, 8, 1)
    x0[:, 3] = x0[:, 2]                          # rank-deficient start block
    st, lam, xd, info = ch.chfsi_solve(dev(a), None, 6, 2, 1e-10, X0=dev(x0))
    assert st == 0
    ref = ochfsi.chfsi(a, 6, 2)
    assert np.abs(lam[:6] - ref.lam[:6]).max() <= RTOL * np.abs(ref.lam[:6]).min()


def test_b_factor_reused_only_for_identical_b():
    import torch
    conf = gen.small_config("f", 300, 12, 4, True, length=2, cfg=92, delta=1e-2)
    seq = gen.Sequence(conf)
    probs = [a.copy() for _, a in seq.problems()]
    bd = dev(seq.B)
    wb = ch.chfsi_workspace_bytes(300, 12, 4, True)
    work = torch.empty(wb, dtype=torch.uint8, device="cuda:0")
    st, lam1, x1, info1 = ch.chfsi_solve(dev(probs[0]), bd, 12, 4, 1e-10, work=work)
    assert st == 0 and info1["b_factor_reused"] == 0
    st, lam2, x2, info2 = ch.chfsi_solve(dev(probs[1]), bd, 12, 4, 1e-10, X0=x1, work=work)
    assert st == 0 and info2["b_factor_reused"] == 1
    fresh = ch.chfsi_solve(dev(probs[1]), bd, 12, 4, 1e-10, X0=x1)
    assert np.array_equal(lam2, fresh[1]) and fresh[3]["b_factor_reused"] == 0
    # a one-ulp change of B must invalidate the stored factor
    b2 = seq.B.copy()
    b2[5, 5] = np.nextafter(b2[5, 5].real, 2.0)
    st, lam3, x3, info3 = ch.chfsi_solve(dev(probs[1]), dev(b2), 12, 4, 1e-10, X0=x1, work=work)
    assert st == 0 and info3["b_factor_reused"] == 0
    h, _ = ochfsi.reduce_to_standard(probs[1], b2)
    ref = eigh.eigvalsh(h)[:12]
    assert np.abs(lam3[:12] - ref).max() <= RTOL * np.abs(ref).min()
    # reuse disabled by option
    o = _opts(reuse_b_factor=0)
    st, lam4, _, info4 = ch.chfsi_solve(dev(probs[1]), dev(b2), 12, 4, 1e-10, X0=x1, work=work,
                                        opts=o)
    assert st == 0 and info4["b_factor_reused"] == 0


def test_solve_sequence_with_previous_eigenvalues():
    """Warm start with X0 and Lambda0 (Alg. 1 inputs) against the oracle
    doing the same, on the n = 1000 standard workload."""
    conf = gen.CONFIGS["std-n1000"]
    probs = [a.copy() for _, a in gen.Sequence(conf).problems()]
    refs = ochfsi.solve_sequence(probs, conf.nev, conf.nex, with_lambda=True)
    x, lam = None, None
    for a, ref in zip(probs, refs):
        st, lam, xd, info = ch.chfsi_solve(dev(a), None, conf.nev, conf.nex, conf.tol, X0=x,
                                           Lambda0=lam if x is not None else None)
        assert st == 0
        assert np.abs(lam[:conf.nev] - ref.lam[:conf.nev]).max() <= \
            RTOL * np.abs(ref.lam[:conf.nev]).min()
        _check_pairs(a, None, lam, host(xd), conf.nev, conf.tol, info["norm_h"])
        x = xd


@pytest.mark.parametrize("with_lambda,precision", [(False, 1), (True, 1), (True, 2), (True, 3)])
def test_solve_mixed_precision_matches_oracle(with_lambda, precision):
    """precision = 1: filters run in FP32 defect form once residuals allow;
    precision = 2 also runs the early steps of those filters with BF16-split
    products, precision = 3 most of their steps with FP16-split products.
    The eigenvalues still match the FP64 oracle to 1e-10."""
    conf = gen.CONFIGS["std-n1000"]
    probs = [a.copy() for _, a in gen.Sequence(conf).problems()]
    refs = ochfsi.solve_sequence(probs, conf.nev, conf.nex)
    o = _opts(precision=precision)
    x, lam = None, None
    used32 = used16 = usedh = 0
    for a, ref in zip(probs, refs):
        st, lam, xd, info = ch.chfsi_solve(dev(a), None, conf.nev, conf.nex, conf.tol, X0=x,
                                           Lambda0=lam if (with_lambda and x is not None) else None,
                                           opts=o)
        assert st == 0
        assert np.abs(lam[:conf.nev] - ref.lam[:conf.nev]).max() <= \
            RTOL * np.abs(ref.lam[:conf.nev]).min()
        _check_pairs(a, None, lam, host(xd), conf.nev, conf.tol, info["norm_h"])
        used32 += info["filter_iters_fp32"]
        used16 += info["filter_steps_bf16"]
        usedh += info["filter_steps_fp16"]
        x = xd
    assert used32 > 0
    assert (used16 > 0) == (precision == 2)
    assert (usedh > 0) == (precision == 3)
