"""The allocation-free entry point tsqr_factor_r_noalloc through the C ABI:
its R equals, bit for bit, the R of the plan-based entry point
(tsqr_plan_create with want_q = 0, tsqr_factor) on the same geometry, and
agrees with the default R-only plan to 1e-13 (uniqueness of R up to signs,
Sec. 2) -- on two calls in a row, the second on a smaller problem, so the
second call reuses the fixed device array the first one filled."""
import numpy as np
import pytest

import synth
from gpu_util import announce, need_gpu
from metrics import rel_diff

pytestmark = pytest.mark.gpu


def _plan_r(T, torch, Ad, m, n, **kw):
    with T.Plan(m, n, want_q=False, **kw) as p:
        R = p.factor(Ad)
        torch.cuda.synchronize()
    return R.cpu().numpy()


def test_noalloc_r_equals_plan_r_on_two_calls_in_a_row():
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    cases = [(1 << 21, 32, 12.0, 51), (300007, 20, 8.0, 52)]  # the second call is smaller
    for m, n, dec, seed in cases:
        announce(f"noalloc R m={m} n={n}")
        A, _ = synth.prescribed_sigma(m, n, seed=seed, decades=dec)
        Ad = T.to_colmajor(torch.from_numpy(A))
        before = Ad.clone()
        R, info = T.factor_r_noalloc(Ad)
        torch.cuda.synchronize()
        Rn = R.cpu().numpy()
        assert torch.equal(Ad, before)  # A is only read
        assert info["m"] == m and info["n"] == n and info["workspace_bytes"] <= 64 << 20
        # the plan-based entry point on the same geometry: the same kernels, the same bits
        Rp = _plan_r(T, torch, Ad, m, n, leaf_rows=info["leaf_rows"])
        assert np.array_equal(Rn, Rp)
        # the default R-only plan (another tree): R is unique up to roundoff
        assert rel_diff(Rn, _plan_r(T, torch, Ad, m, n)) <= 1e-13
        assert np.all(np.diag(Rn) >= 0) and np.all(np.tril(Rn, -1) == 0)


def test_noalloc_rejects_arguments_and_sizes_beyond_the_array():
    torch = need_gpu()
    from paper_0809_2407_amd import _lib
    from paper_0809_2407_amd import tsqr as T

    lib = _lib.load()
    m, n = 4096, 16
    Ad = T.colmajor(m, n)
    Ad.normal_()
    R = T.colmajor(n, n)
    s = torch.cuda.current_stream().cuda_stream
    assert lib.tsqr_factor_r_noalloc(m, n, Ad.data_ptr(), m - 1, R.data_ptr(), n, s, None) == -4
    assert lib.tsqr_factor_r_noalloc(m, n, Ad.data_ptr(), m, R.data_ptr(), n - 1, s, None) == -6
    assert lib.tsqr_factor_r_noalloc(m, 65, Ad.data_ptr(), m, R.data_ptr(), 65, s, None) == 3
    # 64 columns, 2^26 rows: chains past 256 tiles would be needed (status 6,
    # checked on the host before any launch; the pointer is never dereferenced)
    assert lib.tsqr_factor_r_noalloc(1 << 26, 64, Ad.data_ptr(), 1 << 26, R.data_ptr(), 64, s, None) == 6
    torch.cuda.synchronize()
