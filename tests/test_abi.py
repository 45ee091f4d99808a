"""The C-ABI library: loads without a GPU, exports every declared symbol,
and its host-only logic matches the oracle (no device calls here)."""
import ctypes

import numpy as np
import pytest

import paper_1404_4161_amd as ch
from oracle import chfsi as ochfsi


def test_library_exports_every_declared_function():
    lib = ch.lib()
    names = ch.header_functions()
    assert "chfsi_solve" in names and "chfsi_filter" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def _header_struct(name):
    """(C type, field name) pairs of `typedef struct name {...} name;` in the
    public header, comments removed."""
    import os
    import re
    path = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "chfsi.h")
    src = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
    body = re.search(r"typedef struct %s \{(.*?)\} %s;" % (name, name), src, re.S).group(1)
    out = []
    for decl in body.split(";"):
        decl = " ".join(decl.split())
        if not decl:
            continue
        m = re.match(r"(.*?)\s*\b(\w+)(\[\d+\])?$", decl)
        out.append((m.group(1).replace(" *", "*").strip(), m.group(2) + (m.group(3) or "")))
    return out


@pytest.mark.parametrize("cname,pystruct", [("chfsi_opts", ch.binding.ChfsiOpts),
                                            ("chfsi_info", ch.binding.ChfsiInfo)])
def test_binding_structs_follow_the_header(cname, pystruct):
    """The ctypes mirrors of the option and statistics structs have the
    header's fields in the header's order, with matching C types."""
    import ctypes as C
    ctype_of = {"double": C.c_double, "int": C.c_int, "long long": C.c_longlong,
                "unsigned long long": C.c_ulonglong, "double*": C.c_void_p,
                "const float*": C.c_void_p}
    fields = _header_struct(cname)
    py = pystruct._fields_
    assert [f for _, f in fields] == [f + ("[8]" if f == "step_seconds" else "") for f, _ in py]
    for (ct, f), (pf, pt) in zip(fields, py):
        if f.endswith("]"):
            assert pt == C.c_double * 8, f
        elif ct in ("double*", "const float*"):
            assert C.sizeof(pt) == C.sizeof(C.c_void_p), f
        else:
            assert C.sizeof(pt) == C.sizeof(ctype_of[ct]) and \
                (pt in (C.c_double,)) == (ct == "double"), f


def test_default_options_and_status_strings():
    o = ch.chfsi_default_opts()
    assert (o.tol, o.deg0, o.deg_max, o.max_iter, o.lanczos_steps, o.alpha_rule,
            o.degree_mode, o.reuse_b_factor) == (1e-10, 10, 40, 100, 20, 0, 0, 1)
    assert ch.chfsi_status_string(0) == "success"
    assert "converge" in ch.chfsi_status_string(3)
    assert ch.chfsi_status_string(99) == "unknown status"


def test_workspace_query():
    assert ch.chfsi_workspace_bytes(0, 1, 1, False) == 0
    assert ch.chfsi_workspace_bytes(10, 8, 3, False) == 0           # k > n
    small = ch.chfsi_workspace_bytes(1000, 50, 20, False)
    gen = ch.chfsi_workspace_bytes(1000, 50, 20, True)
    assert 6 * 1000 * 70 * 16 < small < gen
    assert gen - small >= 3 * 1000 * 1000 * 16                      # H, L, W for the reduction
    assert ch.chfsi_step_workspace_bytes(1000, 70) > 2 * 1000 * 70 * 16
    assert ch.chfsi_reduce_workspace_bytes(300) >= 300 * 300 * 16
    # mixed precision adds fp32(H); the BF16- and FP16-split forms also their
    # split panel
    o = ch.chfsi_default_opts()
    sizes = []
    for p in (0, 1, 2, 3):
        o.precision = p
        sizes.append(ch.chfsi_workspace_bytes(1000, 50, 20, False, o))
    assert sizes[1] - sizes[0] >= 1000 * 1000 * 8
    assert sizes[2] - sizes[1] >= 1000 * 1024 * 8
    assert sizes[3] == sizes[2]
    lib = ch.lib()
    assert lib.chfsi_defect_split_workspace_bytes(1000, 70) >= \
        lib.chfsi_defect_workspace_bytes(1000, 70) + 1000 * 1024 * 8


def test_invalid_arguments_are_rejected_before_any_device_call():
    lib = ch.lib()
    lam = (ctypes.c_double * 4)()
    dummy = ctypes.c_void_p(256)
    # n < 1, nex < 1, k > n, tol <= 0, null pointers
    assert lib.chfsi_solve(0, 1, 1, dummy, 1, None, 0, 1e-10, None, 0, None, lam, dummy, 1, dummy,
                           1 << 20, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_solve(10, 2, 0, dummy, 10, None, 0, 1e-10, None, 0, None, lam, dummy, 10, dummy,
                           1 << 20, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_solve(10, 8, 3, dummy, 10, None, 0, 1e-10, None, 0, None, lam, dummy, 10, dummy,
                           1 << 20, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_solve(10, 2, 2, dummy, 10, None, 0, 0.0, None, 0, None, lam, dummy, 10, dummy,
                           1 << 20, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_solve(10, 2, 2, None, 10, None, 0, 1e-10, None, 0, None, lam, dummy, 10, dummy,
                           1 << 20, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    # lda < n
    assert lib.chfsi_solve(10, 2, 2, dummy, 9, None, 0, 1e-10, None, 0, None, lam, dummy, 10, dummy,
                           1 << 20, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    # misaligned pointer
    assert lib.chfsi_solve(10, 2, 2, ctypes.c_void_p(8), 10, None, 0, 1e-10, None, 0, None, lam, dummy,
                           10, dummy, 1 << 20, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    # Lambda0 without X0, or not ascending
    lam0 = (ctypes.c_double * 4)(1.0, 2.0, 3.0, 4.0)
    assert lib.chfsi_solve(10, 2, 2, dummy, 10, None, 0, 1e-10, None, 0, lam0, lam, dummy, 10,
                           dummy, 1 << 30, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    bad0 = (ctypes.c_double * 4)(1.0, 3.0, 2.0, 4.0)
    assert lib.chfsi_solve(10, 2, 2, dummy, 10, None, 0, 1e-10, dummy, 10, bad0, lam, dummy, 10,
                           dummy, 1 << 30, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    # workspace too small is only detectable after carving: still no device call
    assert lib.chfsi_solve(10, 2, 2, dummy, 10, None, 0, 1e-10, None, 0, None, lam, dummy, 10, dummy,
                           16, None, None, None) == ch.binding.CHFSI_INVALID_ARG
    deg = (ctypes.c_int * 2)(3, 2)
    assert lib.chfsi_filter(10, 2, dummy, 10, dummy, 10, deg, 0.0, 1.0, -2.0, dummy, 1 << 30,
                            None, None, None) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_zgemm(b"X", b"N", 2, 2, 2, (ctypes.c_double * 2)(), dummy, 2, dummy, 2,
                           (ctypes.c_double * 2)(), dummy, 2, None, 0, None) == \
        ch.binding.CHFSI_INVALID_ARG
    # BF16-split defect filter: negative step count, unsorted degrees, small workspace
    mu = (ctypes.c_double * 2)(1.0, 2.0)
    ok = (ctypes.c_int * 2)(2, 3)
    for fn in (lib.chfsi_filter_defect_split, lib.chfsi_filter_defect_fp16):
        for steps, dg, wb in ((-1, ok, 1 << 40), (1, deg, 1 << 40), (1, ok, 64)):
            assert fn(10, 2, dummy, 10, dummy, 10, dummy, 10, mu, dg, 5.0, 1.0, -2.0, steps,
                      dummy, 10, dummy, wb, None, None, None) == ch.binding.CHFSI_INVALID_ARG


def test_degree_rule_bit_exact_with_oracle():
    g = np.random.default_rng(0)
    for trial in range(200):
        k = int(g.integers(1, 40))
        alpha = float(g.uniform(-16, -14))
        beta = float(g.uniform(30, 50))
        mu = np.sort(g.uniform(-21, alpha, k))
        if trial % 7 == 0:
            mu[-1] = alpha                      # a vector on the interval edge (|t| = 1)
        res = 10.0 ** g.uniform(-9, 0, k)
        nw = int(g.integers(0, k + 1))
        tol = float(10.0 ** g.uniform(-10, -7))
        dm = int(g.integers(5, 41))
        ref = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol, dm)
        got = ch.chfsi_degrees(mu, res, nw, alpha, beta, tol, dm)
        assert np.array_equal(ref, got), (trial, ref, got)


def test_degrees_rejects_bad_interval():
    with pytest.raises(ch.ChfsiError):
        ch.chfsi_degrees([1.0], [1.0], 1, 2.0, 1.0, 1e-9)


def test_learned_degree_options_defaults_and_validation():
    o = ch.chfsi_default_opts()
    assert (o.degree_jitter, o.first_rule, o.log_capacity) == (0.0, 0, 0)
    assert not o.log and not o.mlp
    lib = ch.lib()
    lam = (ctypes.c_double * 4)()
    dummy = ctypes.c_void_p(256)

    def solve_with(**kw):
        oo = ch.chfsi_default_opts()
        for key, v in kw.items():
            setattr(oo, key, v)
        return lib.chfsi_solve(10, 2, 2, dummy, 10, None, 0, 1e-10, None, 0, None, lam, dummy, 10,
                               dummy, 1 << 30, ctypes.byref(oo), None, None)

    assert ch.chfsi_default_opts().rr_refine == 1
    assert solve_with(rr_refine=2) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_eigh_projected(4, dummy, 4, dummy, 4, lam, 3, dummy, 1 << 30, None,
                                    None) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_eigh_projected(4, dummy, 3, dummy, 4, lam, 1, dummy, 1 << 30, None,
                                    None) == ch.binding.CHFSI_INVALID_ARG
    assert solve_with(precision=4) == ch.binding.CHFSI_INVALID_ARG
    assert solve_with(precision=-1) == ch.binding.CHFSI_INVALID_ARG
    assert solve_with(precision=2, deg_max=300) == ch.binding.CHFSI_INVALID_ARG
    assert solve_with(precision=3, deg_max=300) == ch.binding.CHFSI_INVALID_ARG
    assert solve_with(degree_mode=3) == ch.binding.CHFSI_INVALID_ARG
    assert solve_with(degree_mode=2) == ch.binding.CHFSI_INVALID_ARG        # no network
    assert solve_with(degree_jitter=-0.1) == ch.binding.CHFSI_INVALID_ARG
    assert solve_with(first_rule=2) == ch.binding.CHFSI_INVALID_ARG
    assert solve_with(log_capacity=5) == ch.binding.CHFSI_INVALID_ARG       # no buffer
    bad = (ctypes.c_float * ch.binding.CHFSI_MLP_PARAMS)()
    bad[7] = float("inf")
    assert solve_with(degree_mode=2, mlp=ctypes.cast(bad, ctypes.POINTER(ctypes.c_float))) == \
        ch.binding.CHFSI_NONFINITE
    # network entry points check their sizes before touching the device
    assert lib.chfsi_mlp_gradient(0, dummy, dummy, dummy, dummy, dummy, dummy, 1 << 30, None) == \
        ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_mlp_adam(dummy, dummy, dummy, dummy, 1e-3, 0, None) == \
        ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_mlp_train(5, dummy, dummy, dummy, 3, 1e-3, dummy, 16, None, None) == \
        ch.binding.CHFSI_INVALID_ARG
    assert ch.lib().chfsi_mlp_workspace_bytes(1000) > 1000 * (8 + 4 * 64) * 4


def test_degree_features_match_oracle():
    from oracle import mlp
    g = np.random.default_rng(11)
    alpha, beta, gamma, norm_h, tol_abs = -9.0, 45.0, -26.0, 45.0, 4.5e-9
    n_ok = 0
    for _ in range(300):
        mu = g.uniform(-40, 50)
        res = 10.0 ** g.uniform(-12, 0)
        gap = 10.0 ** g.uniform(-14, 1)
        loop = int(g.integers(1, 9))
        got = ch.chfsi_degree_features(mu, res, gap, alpha, beta, gamma, norm_h, tol_abs, loop)
        ref = mlp.features(mu, res, gap, alpha, beta, gamma, norm_h, tol_abs, loop)
        if ref is None:
            assert got is None
            continue
        n_ok += 1
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), (mu, res, gap)
    assert n_ok > 100


def test_autotuner_and_batch_argument_checks():
    lib = ch.lib()
    assert lib.chfsi_autotune_set(0, 5, 0) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_autotune_set(10, 5, ch.binding.FILTER_VARIANTS) == \
        ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_autotune_set(10, 5, -1) == ch.binding.CHFSI_INVALID_ARG
    assert lib.chfsi_autotune_workspace_bytes(100, 10) >= 16 * (100 * 100 + 2 * 100 * 10)
    n = (ctypes.c_int * 1)(10)
    N = (ctypes.c_int * 1)(20)                       # N > n
    v = (ctypes.c_int * 1)()
    assert lib.chfsi_autotune_filter(1, n, N, ctypes.c_void_p(256), 1 << 30, None, v, None) == \
        ch.binding.CHFSI_INVALID_ARG
    assert ch.chfsi_batch_workspace_bytes(0) == 0
    assert ch.chfsi_batch_workspace_bytes(4) > 0
    st = (ctypes.c_int * 1)()
    assert lib.chfsi_solve_batch(0, None, None, None, None, None, None, None, 1e-10, None, None,
                                 None, None, None, None, None, None, None, 0, None, 0, None, None,
                                 st) == ch.binding.CHFSI_INVALID_ARG


def test_sequence_calibrated_degrees_follow_their_definition():
    """degree_mode 3's rule (parity unpinned: the paper defers Multiple
    Optimization to another paper; checked against its stated definition
    and the analytic rule it falls back to)."""
    import math
    from oracle import chebyshev
    g = np.random.default_rng(4)
    k, nw = 40, 30
    mu = np.sort(np.concatenate([g.uniform(-24, -11, k - 4), g.uniform(-9, 20, 4)]))
    res = 10.0 ** g.uniform(-9, -3, k)
    alpha, beta, tol_abs = mu[-1], 60.0, 6e-9
    rule = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol_abs, 40)
    # unknown speeds: the rule
    d, src = ch.chfsi_degrees_sequence(mu, res, None, nw, alpha, beta, tol_abs, 40)
    assert np.array_equal(d, rule)
    # half speed everywhere, every vector can finish: ceil(1.25 * 2 m_a)
    c, e = 0.5 * (alpha + beta), 0.5 * (beta - alpha)
    r = chebyshev.rho((mu - c) / e)
    speed = np.full(k, 0.5)
    d, src = ch.chfsi_degrees_sequence(mu, res, speed, nw, alpha, beta, tol_abs, 400)
    rule400 = ochfsi.degree_rule(mu, res, nw, alpha, beta, tol_abs, 400)
    for j in range(nw):
        if r[j] > 1:
            m_a = math.log(max(res[j] / tol_abs, 1.0)) / math.log(r[j])
            lo, hi = math.ceil(2.5 * m_a - 1e-9), math.ceil(2.5 * m_a + 1e-9)
            assert max(lo, 1, rule400[j]) <= d[j] <= max(hi, 1, rule400[j])
            assert src[j] == 1
    assert np.all(d[nw:] == d[:nw].max())
    # a vector that cannot finish under the cap: no margin, speed only
    d2, _ = ch.chfsi_degrees_sequence(mu, res, speed, nw, alpha, beta, tol_abs, 5)
    assert np.all(d2 <= 5) and np.all(d2 >= np.minimum(rule, 5))
