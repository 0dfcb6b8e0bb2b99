"""Parity of tsqr_apply_qt (B <- Q_full^T B, the reduction of Sec. 4.1) with the
oracle run on the same tree.  On well-conditioned inputs every row is compared
(same tree, same reflectors); on ill-conditioned ones the unique top rows
D Q^T B are compared with the GPU's own explicit Q, together with the
invariants: Q^T preserves norms, Q^T A = [R; 0]."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import fp64_bound

pytestmark = pytest.mark.gpu


def run_apply(A, B, ldb=None, **plan_kw):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = A.shape
    k = B.shape[1]
    Ad = T.to_colmajor(torch.from_numpy(A))
    Bd = T.colmajor(m, k, ld=ldb or m)
    Bd.copy_(torch.from_numpy(np.ascontiguousarray(B)))
    with T.Plan(m, n, **plan_kw) as p:
        info = p.info()
        R = p.factor(Ad)
        p.apply_qt(Ad, Bd)
        Q = p.form_q(Ad, T.colmajor(m, n))
        torch.cuda.synchronize()
    return Bd.cpu().numpy(), R.cpu().numpy(), Q.cpu().numpy(), info


CASES = [(4096, 16, 32, dict(leaf_rows=512)), (3000, 17, 5, dict(tree="binary")), (5000, 8, 37, dict()),
         (20000, 32, 70, dict(tree="hybrid", flat_len=3)), (777, 3, 1, dict(tree="flat")), (6000, 64, 32, dict()),
         (9000, 48, 16, dict(tree="binary")), (2048, 20, 33, dict(tree="hybrid", flat_len=2))]


@pytest.mark.parametrize("m,n,k,kw", CASES)
def test_apply_qt_matches_oracle_all_rows(m, n, k, kw):
    need_gpu()
    A = synth.gaussian(m, n, seed=300 + n)
    B = synth.gaussian(m, k, seed=400 + k)
    announce(f"apply_qt {m}x{n} k={k} {kw}")
    X, R, Q, info = run_apply(A, B, **kw)
    t = oracle.TSQR(A, info["leaf_rows"], info["tile_rows"])
    Xo = t.apply_qt(B)
    scale = np.linalg.norm(B)
    assert np.abs(X - Xo).max() <= 1e-13 * scale
    # top rows are D Q^T B with the Q of tsqr_form_q
    assert np.abs(X[:n] - Q.T @ B).max() <= 1e-13 * scale


@pytest.mark.parametrize("m,n", [(50000, 32), (30000, 17), (8000, 64)])
def test_apply_qt_ill_conditioned_invariants(m, n):
    need_gpu()
    A, _ = synth.prescribed_sigma(m, n, seed=500 + n, decades=12)
    B = synth.gaussian(m, 32, seed=501)
    announce(f"apply_qt kappa=1e12 {m}x{n}")
    X, R, Q, info = run_apply(A, B)
    nb = np.linalg.norm(B)
    assert abs(np.linalg.norm(X) - nb) <= 64 * 2.0 ** -53 * nb
    assert np.abs(X[:n] - Q.T @ B).max() <= 1e-13 * nb
    # Q^T A = [R; 0] (the complement rows within the backward-error bound)
    XA, R2, _, _ = run_apply(A, A.copy())
    na = np.linalg.norm(A)
    assert np.abs(XA[:n] - R2).max() <= 1e-13 * na
    assert np.linalg.norm(XA[n:]) <= fp64_bound(n) * na


def test_apply_qt_leading_dimension_and_zero_columns():
    torch = need_gpu()
    A = synth.gaussian(4000, 24, seed=7)
    B = synth.gaussian(4000, 10, seed=8)
    announce("apply_qt ldb > m")
    X1, _, _, _ = run_apply(A, B, ldb=4003)
    X2, _, _, _ = run_apply(A, B)
    assert np.array_equal(X1, X2)
    from paper_0809_2407_amd import tsqr as T
    Ad = T.to_colmajor(torch.from_numpy(A))
    with T.Plan(4000, 24) as p:
        p.factor(Ad)
        E = T.colmajor(4000, 0)
        p.apply_qt(Ad, E)  # k = 0: nothing to do
        torch.cuda.synchronize()


def test_least_squares_through_apply_qt():
    """x = R^-1 (Q^T b)[:n] solves min ||A x - b|| (Sec. 4.1: the R-only reduction
    plus Q^T applied to the right-hand side)."""
    need_gpu()
    A, _ = synth.prescribed_sigma(20000, 12, seed=9, decades=4)
    xt = np.arange(1, 13, dtype=np.float64)
    b = A @ xt + 1e-3 * synth.gaussian(20000, 1, seed=10)[:, 0]
    announce("least squares")
    X, R, _, _ = run_apply(A, b[:, None])
    x = np.linalg.solve(np.triu(R), X[:12, 0])
    xr = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.abs(x - xr).max() <= 1e-9 * np.abs(xr).max()
    assert abs(np.linalg.norm(X[12:, 0]) - np.linalg.norm(b - A @ xr)) <= 1e-10 * np.linalg.norm(b)
