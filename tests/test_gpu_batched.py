"""Batched plans (one captured graph for many problems) through the C ABI:
every problem's R and Q equal, bit for bit, those of a single-problem plan
with the same geometry (the per-item device code is the same), and meet the
oracle's bounds; replays with new matrices reuse the captured graphs."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import backward_error, fp64_bound, is_upper, orthogonality, rel_diff

pytestmark = pytest.mark.gpu

SHAPES = [(30000, 64), (1000, 8), (25000, 16), (4100, 17), (12000, 32), (777, 3), (20000, 40), (6000, 64),
          (2000, 16), (15000, 8), (64, 64), (9000, 32)]


def _inputs(seed0):
    mats = []
    for k, (m, n) in enumerate(SHAPES):
        if k % 2:
            A = synth.gaussian(m, n, seed=seed0 + k)
        else:
            A, _ = synth.prescribed_sigma(m, n, seed=seed0 + k, decades=12)
        mats.append(A)
    return mats


def _single(A, leaf_rows):
    """A single plan with the geometry the batched plan chose for the problem
    (a problem in a batch keeps longer leaf chains than one on its own)."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = A.shape
    Ad = T.to_colmajor(torch.from_numpy(A))
    with T.Plan(m, n, leaf_rows=leaf_rows) as p:
        R = p.factor(Ad)
        Q = p.form_q(Ad, T.colmajor(m, n))
        torch.cuda.synchronize()
    return R.cpu().numpy(), Q.cpu().numpy()


def test_batched_equals_single_plans_and_meets_oracle_bounds():
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    mats = _inputs(1000)
    ms, ns = [A.shape[0] for A in mats], [A.shape[1] for A in mats]
    announce(f"batched {len(mats)} problems")
    with T.BatchedPlan(ms, ns) as bp:
        for rep, data in enumerate([mats, _inputs(2000)]):
            As = [T.to_colmajor(torch.from_numpy(A)) for A in data]
            Rs = bp.factor(As)
            Qs = bp.form_q(As, [T.colmajor(m, n) for m, n in zip(ms, ns)])
            torch.cuda.synchronize()
            for i, A in enumerate(data):
                announce(f"batched rep {rep} problem {i} {A.shape}")
                R, Q = Rs[i].cpu().numpy(), Qs[i].cpu().numpy()
                Rs1, Qs1 = _single(A, bp.problem_info(i)["leaf_rows"])
                assert np.array_equal(R, Rs1) and np.array_equal(Q, Qs1)
                n = A.shape[1]
                assert is_upper(R) and np.all(np.diag(R) >= 0)
                assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-13
                assert backward_error(A, Q, R) <= fp64_bound(n)
                assert orthogonality(Q) <= fp64_bound(n)
        info = bp.problem_info(0)
        assert info["m"] == 30000 and info["n"] == 64 and info["num_leaves"] >= 1


def test_batched_elementwise_against_oracle_tree():
    """Well-conditioned problems: R and Q element by element against the oracle
    run on each problem's own tree."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    shapes = [(5000, 16), (3000, 17), (8000, 32), (1000, 5)]
    mats = [synth.gaussian(m, n, seed=77 + n) for m, n in shapes]
    announce("batched elementwise")
    with T.BatchedPlan([m for m, _ in shapes], [n for _, n in shapes], tree="hybrid", flat_len=2) as bp:
        As = [T.to_colmajor(torch.from_numpy(A)) for A in mats]
        Rs = bp.factor(As)
        Qs = bp.form_q(As, As)  # Q may alias A
        torch.cuda.synchronize()
        for i, A in enumerate(mats):
            info = bp.problem_info(i)
            t = oracle.TSQR(A, info["leaf_rows"], info["tile_rows"])
            Ro, Qo = t.R(), t.form_q()
            assert np.abs(Rs[i].cpu().numpy() - Ro).max() <= 1e-13 * np.linalg.norm(Ro)
            assert np.abs(Qs[i].cpu().numpy() - Qo).max() <= 1e-13


def test_batched_r_only_and_errors():
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T
    from paper_0809_2407_amd._lib import TsqrError

    shapes = [(4000, 8), (9000, 24)]
    mats = [synth.gaussian(m, n, seed=5 + n) for m, n in shapes]
    announce("batched R only")
    with T.BatchedPlan([m for m, _ in shapes], [n for _, n in shapes], want_q=False) as bp:
        As = [T.to_colmajor(torch.from_numpy(A)) for A in mats]
        before = [X.clone() for X in As]
        Rs = bp.factor(As)
        torch.cuda.synchronize()
        for A, X, X0, R in zip(mats, As, before, Rs):
            assert torch.equal(X, X0)
            assert rel_diff(R.cpu().numpy(), oracle.qr_reference(A, want_q=False)) <= 1e-13
        with pytest.raises(TsqrError) as e:
            bp.form_q(As)
        assert e.value.status == 4
    torch.cuda.synchronize()


def test_batched_mixed_equals_single_mixed_plans():
    """MIXED batched plans give each problem the results of a single MIXED plan,
    within the mixed bounds against the FP64 oracle."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    shapes = [(30000, 64), (1500, 8), (4100, 33), (20000, 32), (777, 3), (9000, 17)]
    mats = [synth.gaussian(m, n, seed=950 + i) for i, (m, n) in enumerate(shapes)]
    announce(f"batched mixed {len(mats)} problems")
    with T.BatchedPlan([m for m, _ in shapes], [n for _, n in shapes], precision="mixed") as bp:
        As = [T.to_colmajor(torch.from_numpy(A)) for A in mats]
        Rs = bp.factor(As)
        Qs = bp.form_q(As, [T.colmajor(m, n) for m, n in shapes])
        torch.cuda.synchronize()
        assert bp.problem_info(0)["precision"] == 1
        for i, A in enumerate(mats):
            m, n = A.shape
            announce(f"batched mixed problem {i} {A.shape}")
            Ad = T.to_colmajor(torch.from_numpy(A))
            with T.Plan(m, n, precision="mixed", leaf_rows=bp.problem_info(i)["leaf_rows"]) as p:
                R1 = p.factor(Ad)
                Q1 = p.form_q(Ad, T.colmajor(m, n))
                torch.cuda.synchronize()
            R, Q = Rs[i].cpu().numpy(), Qs[i].cpu().numpy()
            assert np.array_equal(R, R1.cpu().numpy()) and np.array_equal(Q, Q1.cpu().numpy())
            assert backward_error(A, Q, R) <= 1e-6
            assert orthogonality(Q) <= 1e-13
            assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-5


def test_batched_mixed_r_only_and_check():
    """MIXED batched R only (the first pass's R) equals single MIXED R-only
    plans; with Q, each problem's second-pass check is reported."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    shapes = [(6000, 32), (2000, 64), (999, 9)]
    mats = [synth.gaussian(m, n, seed=970 + i) for i, (m, n) in enumerate(shapes)]
    announce("batched mixed R only")
    with T.BatchedPlan([m for m, _ in shapes], [n for _, n in shapes], precision="mixed", want_q=False) as bp:
        Rs = bp.factor([T.to_colmajor(torch.from_numpy(A)) for A in mats])
        torch.cuda.synchronize()
        for i, (A, R) in enumerate(zip(mats, Rs)):
            m, n = A.shape
            with T.Plan(m, n, precision="mixed", want_q=False, leaf_rows=bp.problem_info(i)["leaf_rows"]) as p:
                R1 = p.factor(T.to_colmajor(torch.from_numpy(A)))
                torch.cuda.synchronize()
            assert np.array_equal(R.cpu().numpy(), R1.cpu().numpy())
            assert rel_diff(R.cpu().numpy(), oracle.qr_reference(A, want_q=False)) <= 1e-5
    announce("batched mixed check")
    with T.BatchedPlan([m for m, _ in shapes], [n for _, n in shapes], precision="mixed") as bp:
        bp.factor([T.to_colmajor(torch.from_numpy(A)) for A in mats])
        for i in range(len(shapes)):
            info = bp.problem_info(i)
            # Q1 is orthonormal to FP32 accuracy only: the check is above its bound and the pass applies
            assert info["precision"] == 1 and info["reorth_applied"] == 1
            assert 1e-13 < info["orth_estimate"] < 1e-4
