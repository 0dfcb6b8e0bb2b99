"""Every padded column count of the kernels (widths rounded up to a multiple of
4, widths 49-52 on the 56-column kernels and 57-60 on the 64-column ones), with widths that are not a multiple
of 4 so the zero columns past n are exercised in each: the FP64 path against
the oracle run on the same tree, element by element, and the mixed path
against the bounds of the method."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu, run_tsqr
from metrics import backward_error, fp64_bound, is_upper, orthogonality, rel_diff

pytestmark = pytest.mark.gpu

WIDTHS = [2, 7, 10, 13, 19, 22, 26, 31, 34, 38, 43, 46, 49, 50, 52, 53, 55, 57, 58, 60, 62, 63]


@pytest.mark.parametrize("n", WIDTHS)
def test_fp64_every_kernel_width(n):
    """A Gaussian matrix (well conditioned, so Q itself is determined to
    rounding and can be compared element by element)."""
    need_gpu()
    A = synth.gaussian(6000 + 3 * n, n, seed=1000 + n)
    announce(f"fp64 width {n}: {A.shape[0]}x{n} hybrid3")
    R, Q, _, info = run_tsqr(A, tree="hybrid", flat_len=3)
    assert info["n_padded"] == (64 if 57 <= n <= 60 else (56 if 49 <= n <= 52 else (n + 3) // 4 * 4))
    assert info["num_leaves"] > 1
    assert is_upper(R) and np.all(np.diag(R) >= 0)
    t = oracle.TSQR(A, info["leaf_rows"], info["tile_rows"])
    Ro, Qo = t.R(), t.form_q()
    assert np.abs(R - Ro).max() <= 1e-13 * np.linalg.norm(Ro)
    assert np.abs(Q - Qo).max() <= 1e-13
    assert backward_error(A, Q, R) <= fp64_bound(n)
    assert orthogonality(Q) <= fp64_bound(n)


@pytest.mark.parametrize("n", [13, 31, 50, 57, 60, 63])
def test_fp64_ill_conditioned_widths(n):
    """sigma from 1 to 1e-12: Q's last columns are determined only to about
    eps * kappa, so the checks are the method's bounds and R against the
    reference QR."""
    need_gpu()
    A, _ = synth.prescribed_sigma(5000 + 7 * n, n, seed=1200 + n, decades=12)
    announce(f"fp64 ill-conditioned width {n}: {A.shape[0]}x{n}")
    R, Q, _, _ = run_tsqr(A, tree="hybrid", flat_len=2)
    assert is_upper(R) and np.all(np.diag(R) >= 0)
    assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-13
    assert backward_error(A, Q, R) <= fp64_bound(n)
    assert orthogonality(Q) <= fp64_bound(n)


@pytest.mark.parametrize("n", [7, 22, 38, 53, 57, 60, 63])
def test_mixed_every_kernel_width(n):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m = 9000 + 5 * n
    A, _ = synth.prescribed_sigma(m, n, seed=1100 + n, decades=6)
    announce(f"mixed width {n}: {m}x{n}")
    Ad = T.to_colmajor(torch.from_numpy(A))
    with T.Plan(m, n, precision="mixed") as p:
        R = p.factor(Ad)
        Q = p.form_q(None)
        torch.cuda.synchronize()
        info = p.info()
    R, Q = R.cpu().numpy(), Q.cpu().numpy()
    assert info["reorth_applied"] == 1
    assert is_upper(R) and np.all(np.diag(R) >= 0)
    assert backward_error(A, Q, R) <= 1e-6
    assert orthogonality(Q) <= 1e-13
    assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-5


@pytest.mark.parametrize("n", [49, 51, 52, 57, 59, 60])
def test_apply_qt_on_widened_kernels(n):
    """Q^T B for widths padded by 4-7 columns, every row against the oracle's
    replay of the same tree."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, k = 7000 + n, 33
    A = synth.gaussian(m, n, seed=1300 + n)
    B = synth.gaussian(m, k, seed=1400 + n)
    announce(f"apply_qt width {n}: {m}x{n} k={k}")
    Ad = T.to_colmajor(torch.from_numpy(A))
    Bd = T.to_colmajor(torch.from_numpy(B))
    with T.Plan(m, n, tree="hybrid", flat_len=3) as p:
        info = p.info()
        p.factor(Ad)
        p.apply_qt(Ad, Bd)
        torch.cuda.synchronize()
    X = Bd.cpu().numpy()
    Xo = oracle.TSQR(A, info["leaf_rows"], info["tile_rows"]).apply_qt(B)
    assert np.abs(X - Xo).max() <= 1e-13 * np.linalg.norm(B)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_widened_widths_equal_single_plans(precision):
    """A batched plan whose 56-column class holds widths 49-52 and 56 and whose
    64-column class holds 57-60 and 64 gives every problem the bits of its
    single-problem plan."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    shapes = [(9000, 57), (3000, 60), (12000, 64), (5000, 58), (2500, 59), (7000, 49), (4000, 52), (6000, 56),
              (3500, 50)]
    mats = [synth.gaussian(m, n, seed=1500 + i) for i, (m, n) in enumerate(shapes)]
    announce(f"batched {precision} widths 49-52 and 57-60")
    with T.BatchedPlan([m for m, _ in shapes], [n for _, n in shapes], precision=precision) as bp:
        assert all(bp.problem_info(i)["n_padded"] == (64 if n > 56 else 56) for i, (_, n) in enumerate(shapes))
        As = [T.to_colmajor(torch.from_numpy(A)) for A in mats]
        Rs = bp.factor(As)
        Qs = bp.form_q(As, [T.colmajor(m, n) for m, n in shapes])
        torch.cuda.synchronize()
        lrs = [bp.problem_info(i)["leaf_rows"] for i in range(len(shapes))]
    for i, A in enumerate(mats):
        m, n = A.shape
        announce(f"batched {precision} problem {i} {A.shape} against a single plan")
        Ad = T.to_colmajor(torch.from_numpy(A))
        with T.Plan(m, n, precision=precision, leaf_rows=lrs[i]) as p:
            R1 = p.factor(Ad)
            Q1 = p.form_q(Ad if precision == "fp64" else None, T.colmajor(m, n))
            torch.cuda.synchronize()
        R, Q = Rs[i].cpu().numpy(), Qs[i].cpu().numpy()
        assert np.array_equal(R, R1.cpu().numpy()) and np.array_equal(Q, Q1.cpu().numpy())
        bound = fp64_bound(n) if precision == "fp64" else 1e-6
        assert backward_error(A, Q, R) <= bound
        assert orthogonality(Q) <= (fp64_bound(n) if precision == "fp64" else 1e-13)


@pytest.mark.parametrize("m,n", [(100_000, 50), (1_000_000, 50)])
def test_paper_local_qr_shapes_against_the_oracle(m, n):
    """The n = 50 shapes of the paper's local-QR tables, in the geometry a plan
    picks by itself: R and Q element by element against the oracle on the same
    tree, orthogonality measured on the host (FP64 sums by row blocks) within
    the FP64 bound."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    A = synth.gaussian(m, n, seed=1700 + n)
    announce(f"paper shape {m}x{n}")
    R, Q, _, info = run_tsqr(A)
    assert info["n_padded"] == 56
    t = oracle.TSQR(A, info["leaf_rows"], info["tile_rows"])
    Ro, Qo = t.R(), t.form_q()
    assert np.abs(R - Ro).max() <= 1e-13 * np.linalg.norm(Ro)
    assert np.abs(Q - Qo).max() <= 1e-13
    G = np.zeros((n, n))
    for i in range(0, m, 4096):
        G += Q[i:i + 4096].T @ Q[i:i + 4096]
    orth = float(np.linalg.norm(G - np.eye(n)))
    print(f"[gpu-case] {m}x{n}: orthogonality {orth:.2e} (host, by row blocks), "
          f"max|Q - Q_oracle| {np.abs(Q - Qo).max():.2e}", flush=True)
    assert orth <= fp64_bound(n)
