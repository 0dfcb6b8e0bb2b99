"""Out-of-HBM TSQR (the flat tree over host-resident blocks of Sec. 7.1)
through the C ABI: the R of a matrix streamed from host memory in blocks,
against the oracle's R and the in-HBM TSQR's R (R is unique up to signs,
Sec. 2), for ragged last blocks, a last block too short to stand alone,
a single block, pinned and pageable host memory, and a repeated call."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import rel_diff

pytestmark = pytest.mark.gpu


def _host(A, pinned):
    import torch

    H = torch.empty((A.shape[1], A.shape[0]), dtype=torch.float64, pin_memory=pinned).t()
    H.copy_(torch.from_numpy(A))
    return H


@pytest.mark.parametrize("m,n,block,pinned,nblocks", [
    (1_000_003, 24, 1 << 17, True, 8),      # 7 full blocks and a ragged last one
    (300_010, 32, 100_000, True, 3),        # a last block of 10 rows < n joins the one before
    (50_000, 17, 0, False, 1),              # one block (automatic size), pageable memory
    (400_000, 64, 65_536, False, 7),        # pageable, the widest kernels
])
def test_streamed_r_equals_oracle_and_in_hbm_r(m, n, block, pinned, nblocks):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    A, _ = synth.prescribed_sigma(m, n, seed=800 + n, decades=12)
    announce(f"stream m={m} n={n} block={block} pinned={pinned}")
    H = _host(A, pinned)
    with T.StreamPlan(m, n, block_rows=block) as sp:
        info = sp.info()
        assert info["num_blocks"] == nblocks
        R1 = sp.factor(H)
        R2 = sp.factor(H)  # the buffers and plans are reused
        torch.cuda.synchronize()
    R1, R2 = R1.cpu().numpy(), R2.cpu().numpy()
    assert np.array_equal(R1, R2)
    assert np.all(np.diag(R1) >= 0) and np.all(np.tril(R1, -1) == 0)
    assert rel_diff(R1, oracle.qr_reference(A, want_q=False)) <= 1e-13
    with T.Plan(m, n, want_q=False) as p:
        Rh = p.factor(T.to_colmajor(torch.from_numpy(A))).cpu().numpy()
    assert rel_diff(R1, Rh) <= 1e-13
