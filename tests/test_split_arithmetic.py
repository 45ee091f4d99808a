"""The error bounds of the split products used by the mixed-precision
filter's FP16 and BF16 steps, checked on the host.  FP16 (IEEE binary16,
numpy float16, round to nearest even): an FP32 value x, scaled by a power
of two so that
its vector's largest magnitude lies in [2^14, 2^15), splits into
hi = fp16(x), lo = fp16(x - hi); hi_a hi_b + hi_a lo_b + lo_a hi_b then
differs from a b by at most 3 * 2^-22 |a| |b| for normal words, and a dot
product of such terms by at most that fraction of sum |a_k| |b_k| plus
n 2^-39 max|a| max|b| (words in FP16's subnormal range).  The sums here
are exact (float64 of binary16 products), so only the split is measured.
BF16 (rounded from FP32 bits, nearest even): 3 * 2^-16 |a| |b|.

These tests pin the derivation of the bounds with numpy's own binary16
arithmetic; they do not call the library.  The kernels' splits are
covered on the GPU by the split-step tests of test_gpu_kernels.py, which
hold one kernel step to the same bounds (H scaled by 1e6 and 1e-5, defect
columns spanning seven decades, exactly zero defect columns); their NaN
and infinity branches are not exercised by any test."""
import numpy as np


def _scale_exp(v):
    m = float(np.max(np.abs(v)))
    return 0 if m == 0.0 else min(14 - int(np.floor(np.log2(m))), 100)


def _split(v):
    s = _scale_exp(v)
    x = (v.astype(np.float32) * np.float32(2.0 ** s)).astype(np.float32)
    hi = x.astype(np.float16)
    lo = (x - hi.astype(np.float32)).astype(np.float16)
    return hi.astype(np.float64), lo.astype(np.float64), s


def test_scaled_split_keeps_the_largest_magnitude_in_range():
    g = np.random.default_rng(1)
    for e in (-40, -12, 0, 9, 30):
        v = (g.standard_normal(300) * 2.0 ** e).astype(np.float32)
        hi, lo, s = _split(v)
        m = np.max(np.abs(v.astype(np.float64))) * 2.0 ** s
        assert 2.0 ** 14 <= m < 2.0 ** 15
        assert np.all(np.isfinite(hi)) and np.all(np.isfinite(lo))


def test_elementwise_product_error_within_three_times_two_to_minus_22():
    g = np.random.default_rng(2)
    a = (g.standard_normal(20000) * 10.0 ** g.uniform(-3, 3, 20000)).astype(np.float32)
    b = (g.standard_normal(20000) * 10.0 ** g.uniform(-3, 3, 20000)).astype(np.float32)
    ha, la, sa = _split(a)
    hb, lb, sb = _split(b)
    approx = (ha * hb + ha * lb + la * hb) * 2.0 ** -(sa + sb)
    exact = a.astype(np.float64) * b.astype(np.float64)
    # normal words only (subnormal ones are covered by the dot-product floor)
    big = (np.abs(a) * 2.0 ** sa > 2.0 ** -3) & (np.abs(b) * 2.0 ** sb > 2.0 ** -3)
    err = np.abs(approx - exact)[big]
    bound = 3.0 * 2.0 ** -22 * np.abs(exact)[big]
    assert np.all(err <= bound), (err / bound).max()
    # and the split is not exact: errors reach a good fraction of the bound
    assert (err / bound).max() > 0.05


def test_dot_products_within_the_bound_with_the_subnormal_floor():
    g = np.random.default_rng(3)
    n = 4000
    for trial in range(20):
        a = (g.standard_normal(n) * 10.0 ** g.uniform(-6, 6, n)).astype(np.float32)
        b = (g.standard_normal(n) * 10.0 ** g.uniform(-6, 6, n)).astype(np.float32)
        ha, la, sa = _split(a)
        hb, lb, sb = _split(b)
        approx = float(np.sum(ha * hb + ha * lb + la * hb)) * 2.0 ** -(sa + sb)
        a64, b64 = a.astype(np.float64), b.astype(np.float64)
        exact = float(np.sum(a64 * b64))
        bound = (3.0 * 2.0 ** -22 * float(np.sum(np.abs(a64) * np.abs(b64)))
                 + n * 2.0 ** -39 * float(np.max(np.abs(a64)) * np.max(np.abs(b64)))
                 + 1e-15 * float(np.sum(np.abs(a64 * b64))))
        assert abs(approx - exact) <= bound, (trial, abs(approx - exact) / bound)


def _bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32)


def test_bf16_split_product_error_within_three_times_two_to_minus_16():
    """The BF16 form (precision 2) needs no scaling (BF16 has FP32's
    exponent range); its dropped terms are at most 3 * 2^-16 |a| |b|."""
    g = np.random.default_rng(4)
    a = (g.standard_normal(20000) * 10.0 ** g.uniform(-20, 20, 20000)).astype(np.float32)
    b = (g.standard_normal(20000) * 10.0 ** g.uniform(-20, 20, 20000)).astype(np.float32)
    ha = _bf16(a)
    la = _bf16(a - ha)
    hb = _bf16(b)
    lb = _bf16(b - hb)
    h = [x.astype(np.float64) for x in (ha, la, hb, lb)]
    approx = h[0] * h[2] + h[0] * h[3] + h[1] * h[2]
    exact = a.astype(np.float64) * b.astype(np.float64)
    err = np.abs(approx - exact)
    bound = 3.0 * 2.0 ** -16 * np.abs(exact)
    assert np.all(err <= bound), (err / bound).max()
    assert (err / bound).max() > 0.05
