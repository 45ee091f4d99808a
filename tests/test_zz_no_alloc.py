"""chfsi_filter_noalloc (the filter without a workspace, on the library's
static device scratch) against chfsi_filter (the same operation with a
caller-provided workspace) through the C ABI: two calls in a row on one
GPU, the second on a smaller block (the scratch keeps the first call's
contents), each compared column by column with the workspace entry point
(1e-13 relative: the same kernels, the split-K partial sums in the same
order whenever the scratch has room for them, as at these sizes) and with
the CPU oracle (1e-11, the filter tests' bound)."""
import numpy as np
import pytest

import paper_1404_4161_amd as ch
from oracle import chebyshev
from workloads import gen

from .gpu_util import dev, host, rel_col_err

pytestmark = pytest.mark.gpu


def _case(n, k, seed):
    lam = np.sort(np.random.default_rng(seed).uniform(-20, 40, n))
    h = gen.prescribed_problem(n, lam, seed + 1)
    y0 = gen.random_block(n, k, seed + 2)
    degrees = np.sort(np.random.default_rng(seed + 3).integers(1, 14, k)).tolist()
    return h, y0, degrees


@pytest.mark.parametrize("first,second", [((1000, 70), (333, 37))])
def test_noalloc_filter_matches_workspace_filter_twice(first, second):
    c, e, gamma = 13.0, 28.0, -20.5
    for (n, k), seed in ((first, 5), (second, 9)):
        print(f"no-alloc filter n={n} k={k} seed={seed}", flush=True)
        assert ch.chfsi_filter_noalloc_need_bytes(n, k) <= (64 << 20)
        h, y0, degrees = _case(n, k, seed)
        hd = dev(h)
        y_ws = dev(y0)
        fl_ws, ln_ws = ch.chfsi_filter(hd, y_ws, degrees, c, e, gamma)
        y_na = dev(y0)
        fl_na, ln_na = ch.chfsi_filter_noalloc(hd, y_na, degrees, c, e, gamma)
        assert fl_na == fl_ws and ln_na == ln_ws
        got, ref_ws = host(y_na), host(y_ws)
        assert rel_col_err(got, ref_ws).max() <= 1e-13
        ref = chebyshev.chebyshev_filter(h, y0, degrees, c, e, gamma)
        assert rel_col_err(got, ref).max() < 1e-11


def test_noalloc_filter_rejects_blocks_beyond_the_scratch():
    n, k = 3000, 700          # 2 n k 16 bytes = 67.2 MB > 64 MiB
    assert ch.chfsi_filter_noalloc_need_bytes(n, k) > (64 << 20)
    import torch
    y = ch.colmajor(torch.zeros((n, k), dtype=torch.complex128, device="cuda:0"))
    hd = ch.colmajor(torch.zeros((n, n), dtype=torch.complex128, device="cuda:0"))
    with pytest.raises(ch.ChfsiError) as ex:
        ch.chfsi_filter_noalloc(hd, y, [1] * k, 0.0, 1.0, -2.0)
    assert ex.value.status == 1
