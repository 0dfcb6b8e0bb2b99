"""Empty problems (n = 0) through the Python binding on a device: the plans
launch nothing and leave every buffer as it was (Q^T B = B without reflectors);
in a batched plan, empty problems beside ordinary ones change nothing for the
others (their R and Q stay bitwise those of single plans), and a batch of
empty problems only is valid too."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import rel_diff

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("m", [0, 1, 5000])
def test_single_plan_of_an_empty_problem(precision, m):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    announce(f"empty problem m={m} {precision}")
    with T.Plan(m, 0, precision=precision) as p:
        A = T.colmajor(m, 0)
        R = p.factor(A)
        assert tuple(R.shape) == (0, 0)
        Q = p.form_q(A if precision == "fp64" else None)
        assert tuple(Q.shape) == (m, 0)
        B0 = torch.randn((3, m), dtype=torch.float64, device="cuda").t()
        B = T.colmajor(m, 3)
        B.copy_(B0)
        p.apply_qt(A if precision == "fp64" else None, B)
        torch.cuda.synchronize()
        assert torch.equal(B, B0)
        info = p.info()
        assert (info["m"], info["n"], info["num_leaves"], info["workspace_bytes"]) == (m, 0, 0, 0)
    R, info = T.factor_r_noalloc(T.colmajor(m, 0))
    assert tuple(R.shape) == (0, 0) and info["m"] == m


def test_batched_plan_with_empty_problems():
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    shapes = [(5000, 32), (300, 0), (0, 0), (2000, 17), (4000, 0), (64, 64)]
    ms, ns = [s[0] for s in shapes], [s[1] for s in shapes]
    mats = [synth.gaussian(m, n, seed=940 + i) if n > 0 else np.zeros((m, 0)) for i, (m, n) in enumerate(shapes)]
    announce(f"batched with empty problems {shapes}")
    with T.BatchedPlan(ms, ns) as bp:
        As = [T.to_colmajor(torch.from_numpy(A)) if A.shape[1] > 0 else T.colmajor(A.shape[0], 0) for A in mats]
        Rs = bp.factor(As)
        Qs = bp.form_q(As, [T.colmajor(m, n) for m, n in zip(ms, ns)])
        torch.cuda.synchronize()
        infos = [bp.problem_info(i) for i in range(len(shapes))]
    for i, (A, (m, n)) in enumerate(zip(mats, shapes)):
        if n == 0:
            assert tuple(Rs[i].shape) == (0, 0) and tuple(Qs[i].shape) == (m, 0)
            assert infos[i]["num_leaves"] == 0 and infos[i]["workspace_bytes"] == 0
            continue
        announce(f"problem {i} {A.shape}")
        Ad = T.to_colmajor(torch.from_numpy(A))
        with T.Plan(m, n, leaf_rows=infos[i]["leaf_rows"]) as p:
            R1 = p.factor(Ad)
            Q1 = p.form_q(Ad, T.colmajor(m, n))
            torch.cuda.synchronize()
        assert torch.equal(Rs[i], R1) and torch.equal(Qs[i], Q1)
        assert rel_diff(Rs[i].cpu().numpy(), oracle.qr_reference(A, want_q=False)) <= 1e-13


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_plan_of_empty_problems_only(precision):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    announce(f"batched, empty problems only, {precision}")
    ms, ns = [0, 10, 700], [0, 0, 0]
    with T.BatchedPlan(ms, ns, precision=precision) as bp:
        As = [T.colmajor(m, 0) for m in ms]
        Rs = bp.factor(As)
        Qs = bp.form_q(As, [T.colmajor(m, 0) for m in ms])
        torch.cuda.synchronize()
        assert [tuple(R.shape) for R in Rs] == [(0, 0)] * 3
        assert [tuple(Q.shape) for Q in Qs] == [(m, 0) for m in ms]
        assert all(bp.problem_info(i)["n"] == 0 for i in range(3))
