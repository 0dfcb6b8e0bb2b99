"""CAQR (Sec. 6, Alg. 3) on the GPU through the C ABI: TSQR panels with the
trailing update applied up each panel's tree.  R against the oracle's plain
Householder R of the whole matrix (R is unique up to signs, Sec. 2); Q^T B:
the top n rows against the oracle's thin Q, the rest through the invariants
that pin them (their norm is the least-squares residual norm, ||Q^T B|| =
||B||); least squares against numpy's solver; ragged last panels and
narrow-and-tall to square shapes."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import rel_diff

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,panel,npanels", [
    (20000, 200, 32, 7),    # a last panel of 8 columns
    (4096, 512, 64, 8),     # wider panels
    (2000, 1000, 32, 32),   # the last panels see few rows; a last panel of 8 columns
    (50000, 96, 0, 3),      # the automatic panel width (32)
])
def test_caqr_r_and_qtb_match_the_oracle(m, n, panel, npanels):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    k = 5
    Bh = synth.gaussian(m, k, 901)
    announce(f"caqr m={m} n={n} panel={panel}")
    with T.CaqrPlan(m, n, panel) as p:
        assert p.info()["num_panels"] == npanels
        # kappa = 1e6: R only (Q's columns of the small singular values are
        # determined to about kappa eps, so Q^T B is checked on the next matrix)
        A6, _ = synth.prescribed_sigma(m, n, seed=902 + n, decades=6)
        R6 = p.factor(T.to_colmajor(torch.from_numpy(A6))).cpu().numpy()
        assert rel_diff(R6, oracle.qr_reference(A6, want_q=False)) <= 1e-13
        A, _ = synth.prescribed_sigma(m, n, seed=900 + n, decades=1)
        Ad = T.to_colmajor(torch.from_numpy(A))
        Bd = T.to_colmajor(torch.from_numpy(Bh))
        R = p.factor(Ad)
        p.apply_qt(Ad, Bd)
        torch.cuda.synchronize()
    R, X = R.cpu().numpy(), Bd.cpu().numpy()
    Ro, Qo = oracle.qr_reference(A)
    assert np.all(np.diag(R) >= 0) and np.all(np.tril(R, -1) == 0)
    assert rel_diff(R, Ro) <= 1e-13
    # the top n rows are D Q^T B with the signs that make diag(R) >= 0: those of the oracle
    top = Qo.T @ Bh
    assert np.abs(X[:n] - top).max() <= 1e-12 * np.abs(Bh).max() * np.sqrt(m)
    # Q^T is orthogonal: the norm of each column is kept, and the rest of the
    # rows carry the part of B outside the column space of A
    assert np.allclose(np.linalg.norm(X, axis=0), np.linalg.norm(Bh, axis=0), rtol=1e-12)
    resid = np.linalg.norm(Bh - Qo @ top, axis=0)
    assert np.allclose(np.linalg.norm(X[n:], axis=0), resid, rtol=1e-9)
    # least squares: x = R^{-1} (Q^T b)_{0:n}
    x = np.linalg.solve(np.triu(R), X[:n, 0])
    xr = np.linalg.lstsq(A, Bh[:, 0], rcond=None)[0]
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)


def test_caqr_refactor_and_errors():
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T
    from paper_0809_2407_amd._lib import TsqrError

    m, n = 6000, 100
    with T.CaqrPlan(m, n, 16) as p:
        with pytest.raises(TsqrError) as e:
            B = T.colmajor(m, 2)
            p.apply_qt(T.colmajor(m, n), B)
        assert e.value.status == 4
        for seed in (1, 2):  # the plan is reused
            A = synth.gaussian(m, n, 910 + seed)
            Ad = T.to_colmajor(torch.from_numpy(A))
            R = p.factor(Ad).cpu().numpy()
            assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-13


@pytest.mark.parametrize("m,n,panel,k", [
    (20000, 200, 32, 5),    # trailing widths 168, 136, ..., 8: B shares the last 32-column chunk
    (4096, 512, 64, 40),    # more right-hand sides than one chunk
    (2000, 1000, 32, 3),    # the last panels see few rows
    (3000, 64, 64, 7),      # one panel: its only pass is over B
])
def test_caqr_with_right_hand_sides_equals_factor_then_apply(m, n, panel, k):
    """B carried as columns n .. n+k-1 of the factored array: R, the reflectors
    and Q^T B bit for bit those of tsqr_caqr_factor followed by
    tsqr_caqr_apply_qt (the same operations on every column, in the same order),
    and Q^T B's top rows against the oracle's thin Q."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    announce(f"caqr with {k} right-hand sides m={m} n={n} panel={panel}")
    A, _ = synth.prescribed_sigma(m, n, seed=930 + n, decades=1)
    Bh = synth.gaussian(m, k, 931)
    with T.CaqrPlan(m, n, panel) as p:
        Ad, Bd = T.to_colmajor(torch.from_numpy(A)), T.to_colmajor(torch.from_numpy(Bh))
        R0 = p.factor(Ad)
        p.apply_qt(Ad, Bd)
        AB = T.colmajor(m, n + k)
        AB[:, :n].copy_(torch.from_numpy(A))
        AB[:, n:].copy_(torch.from_numpy(Bh))
        R1 = p.factor_rhs(AB)
        # the plan then holds this factorisation: Q^T of a fresh copy of B
        B2 = T.to_colmajor(torch.from_numpy(Bh))
        p.apply_qt(AB[:, :n], B2)
        assert p._lib.tsqr_caqr_factor_rhs(p._h, AB.data_ptr(), m, R1.data_ptr(), n, -1) == -6
        torch.cuda.synchronize()
        assert torch.equal(R0, R1)
        assert torch.equal(Ad, AB[:, :n])
        assert torch.equal(Bd, AB[:, n:])
        assert torch.equal(B2, Bd)
    X = Bd.cpu().numpy()
    Ro, Qo = oracle.qr_reference(A)
    assert rel_diff(R0.cpu().numpy(), Ro) <= 1e-13
    assert np.abs(X[:n] - Qo.T @ Bh).max() <= 1e-12 * np.abs(Bh).max() * np.sqrt(m)
    assert np.allclose(np.linalg.norm(X, axis=0), np.linalg.norm(Bh, axis=0), rtol=1e-12)
