"""The mixed-precision path (FP32 first pass, FP64 re-orthogonalising second
pass) through the C ABI.  FP32 rounding values are parity unpinned: the checks
are the bounds of the method against the FP64 oracle -- backward error
<= 1e-6, orthogonality <= 1e-13 after the second pass, R close to the oracle's
-- and the second pass's own check, ||R2^T R2 - I||_F, against ||Q1^T Q1 - I||_F
computed on the host from the first-pass Q1."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import backward_error, is_upper, orthogonality, rel_diff

pytestmark = pytest.mark.gpu

BWD_MIXED = 1e-6
ORTH_MIXED = 1e-13


def run_mixed(A, want_q=True, **plan_kw):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = A.shape
    Ad = T.to_colmajor(torch.from_numpy(A))
    A_before = Ad.clone()
    with T.Plan(m, n, precision="mixed", want_q=want_q, **plan_kw) as p:
        R = p.factor(Ad)
        Q = Q1 = None
        if want_q:
            Q = p.form_q(None)
            Q1 = p.mixed_q1()
        torch.cuda.synchronize()
        info = p.info()
    assert torch.equal(Ad, A_before)  # A is only read on a MIXED plan
    return (R.cpu().numpy(), None if Q is None else Q.cpu().numpy(),
            None if Q1 is None else Q1.cpu().numpy().astype(np.float64), info)


CASES = [(50000, 64), (40000, 32), (30000, 17), (20000, 8), (9000, 48), (5000, 3), (777, 20)]


@pytest.mark.parametrize("m,n", CASES)
def test_mixed_bounds_on_prescribed_sigma(m, n):
    """sigma log-spaced from 1 to 1e-6 (the matrix of the mixed comparison)."""
    need_gpu()
    A, _ = synth.prescribed_sigma(m, n, seed=700 + n, decades=6)
    announce(f"mixed {m}x{n} kappa=1e6")
    R, Q, Q1, info = run_mixed(A)
    assert info["precision"] == 1 and info["reorth_applied"] == 1
    assert is_upper(R) and np.all(np.diag(R) >= 0)
    bwd = backward_error(A, Q, R)
    orth = orthogonality(Q)
    Rref = oracle.qr_reference(A, want_q=False)
    dr = rel_diff(R, Rref)
    print(f"mixed {m}x{n}: backward {bwd:.2e} orthogonality {orth:.2e} |R-R_fp64|/|R| {dr:.2e} "
          f"orth_estimate {info['orth_estimate']:.3e}")
    assert bwd <= BWD_MIXED
    assert orth <= ORTH_MIXED
    assert dr <= 1e-5


@pytest.mark.parametrize("m,n", [(50000, 64), (30000, 17), (4000, 5)])
def test_second_pass_check_matches_first_pass_orthogonality(m, n):
    """The device-side check ||G - I||_F (= ||R2^T R2 - I||_F) agrees with
    ||Q1^T Q1 - I||_F computed on the host from the copied first-pass Q1."""
    need_gpu()
    A = synth.gaussian(m, n, seed=800 + n)
    announce(f"mixed check {m}x{n}")
    R, Q, Q1, info = run_mixed(A)
    host = orthogonality(Q1)
    est = info["orth_estimate"]
    print(f"orth estimate {est:.6e} host {host:.6e}")
    assert host > ORTH_MIXED  # an FP32 Q1 is never orthogonal to 1e-13
    assert abs(est - host) <= 1e-3 * host
    # Q1 itself is a QR factor to FP32 accuracy, and Q = Q1 R2^{-1}
    assert orthogonality(Q1) <= 1e-4
    assert orthogonality(Q) <= ORTH_MIXED


def test_mixed_ill_conditioned_and_ragged():
    need_gpu()
    A, _ = synth.prescribed_sigma(5 * 4096 + 321, 32, seed=901, decades=12)
    announce("mixed kappa=1e12 ragged")
    R, Q, _, info = run_mixed(A, tree="hybrid", flat_len=3)
    assert backward_error(A, Q, R) <= BWD_MIXED
    assert orthogonality(Q) <= ORTH_MIXED


@pytest.mark.parametrize("tree", [dict(tree="binary"), dict(tree="flat"), dict(tree="hybrid", flat_len=2)],
                         ids=["binary", "flat", "hybrid2"])
def test_mixed_trees(tree):
    need_gpu()
    A, _ = synth.prescribed_sigma(12000, 24, seed=902, decades=6)
    announce(f"mixed trees {tree}")
    R, Q, _, info = run_mixed(A, **tree)
    assert backward_error(A, Q, R) <= BWD_MIXED
    assert orthogonality(Q) <= ORTH_MIXED
    assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-5


def test_mixed_r_only_and_tiny():
    need_gpu()
    A, _ = synth.prescribed_sigma(30000, 40, seed=903, decades=6)
    announce("mixed R only")
    R, Q, _, info = run_mixed(A, want_q=False)
    assert Q is None
    assert is_upper(R) and np.all(np.diag(R) >= 0)
    # one FP32 pass: R to FP32-level accuracy
    assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-5
    for m, n in [(64, 64), (16, 16), (70, 9)]:
        A = synth.gaussian(m, n, seed=904 + n)
        announce(f"mixed tiny {m}x{n}")
        R, Q, _, _ = run_mixed(A)
        assert backward_error(A, Q, R) <= BWD_MIXED
        assert orthogonality(Q) <= ORTH_MIXED


def test_mixed_q1_is_refused_on_an_fp64_plan():
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T
    from paper_0809_2407_amd._lib import TsqrError

    announce("mixed_q1 on an FP64 plan")
    with T.Plan(8000, 16) as p:
        with pytest.raises(TsqrError) as e:
            p.mixed_q1()
        assert e.value.status == 3
    torch.cuda.synchronize()


@pytest.mark.parametrize("m,n,k,ldb_pad,decades", [(8000, 16, 2, 0, 0), (20000, 17, 33, 5, 6), (9001, 8, 40, 0, 0),
                                                   (30000, 64, 32, 3, 6), (4100, 33, 1, 0, 0), (70, 9, 5, 0, 0)])
def test_mixed_apply_qt(m, n, k, ldb_pad, decades):
    """Q^T B on a MIXED plan: the top n rows against the plan's own explicit Q
    (Q^T B in FP64 on the host; the same Q1 R2^{-1}), the other rows
    untouched, and, on well-conditioned inputs, against the FP64 oracle's
    Q^T B within the mixed bound (the same space, the same sign convention;
    at kappa = 1e6 the FP32 pass moves the space by about kappa times its
    rounding, so only the plan's own Q is the reference there)."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    if decades:
        A, _ = synth.prescribed_sigma(m, n, seed=960 + n, decades=decades)
    else:
        A = synth.gaussian(m, n, seed=960 + n)
    B = synth.gaussian(m, k, seed=961 + k)
    Ad = T.to_colmajor(torch.from_numpy(A))
    Bd = T.colmajor(m, k, ld=m + ldb_pad)
    Bd.copy_(torch.from_numpy(B))
    announce(f"mixed apply_qt {m}x{n} k={k} ldb=m+{ldb_pad}")
    with T.Plan(m, n, precision="mixed") as p:
        p.factor(Ad)
        Q = p.form_q(None)
        p.apply_qt(None, Bd)
        torch.cuda.synchronize()
        reorth = p.info()["reorth_applied"]
    X, Qh = Bd.cpu().numpy(), Q.cpu().numpy()
    scale = np.linalg.norm(B)
    assert np.abs(X[:n] - Qh.T @ B).max() <= 1e-13 * scale
    assert np.array_equal(X[n:], B[n:])
    if decades == 0:
        # well conditioned: the FP32 pass moves Q by about its rounding
        Qo = oracle.qr_reference(A, want_q=True)[1]
        assert np.abs(X[:n] - Qo.T @ B).max() <= 10 * BWD_MIXED * scale
    del reorth


def test_mixed_leading_dimensions_and_q_over_a():
    """lda > m and ldq > m; Q may overwrite the original A on a mixed plan
    (its reflectors live in the plan)."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = 9000, 24
    A, _ = synth.prescribed_sigma(m, n, seed=950, decades=6)
    Ad = T.colmajor(m, n, ld=m + 7)
    Ad.copy_(torch.from_numpy(A))
    Qd = T.colmajor(m, n, ld=m + 3)
    announce("mixed ld > m")
    with T.Plan(m, n, precision="mixed") as p:
        R1 = p.factor(Ad)
        p.form_q(None, Qd)
        R2 = p.factor(Ad)
        p.form_q(None, Ad)  # overwrite A with Q
        torch.cuda.synchronize()
    R1, R2 = R1.cpu().numpy(), R2.cpu().numpy()
    Q1, Q2 = Qd.cpu().numpy(), Ad.cpu().numpy()
    assert np.array_equal(R1, R2) and np.array_equal(Q1, Q2)
    assert backward_error(A, Q1, R1) <= BWD_MIXED
    assert orthogonality(Q1) <= ORTH_MIXED
