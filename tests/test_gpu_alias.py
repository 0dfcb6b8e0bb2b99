"""Q written over the factored A.  Above 48 columns the FP64 Q kernel splits
a leaf's 16-column windows over two wavefronts, each of which reads every
reflector column of the rows whose Q window it writes; a call with Q aliasing
A therefore runs one wavefront per leaf.  The aliased Q must equal, bit for
bit, the Q written to a separate buffer, for single and batched plans, at
every workgroup size."""
import numpy as np
import pytest

import synth
from gpu_util import announce, need_gpu

pytestmark = pytest.mark.gpu

WIDTHS = [49, 52, 57, 64]


def _pair(T, torch, A, waves):
    m, n = A.shape
    out = []
    for alias in (False, True):
        Ad = T.to_colmajor(torch.from_numpy(A))
        with T.Plan(m, n, waves=waves) as p:
            p.factor(Ad)
            Q = p.form_q(Ad, Ad if alias else T.colmajor(m, n))
            torch.cuda.synchronize()
        out.append(Q.cpu().numpy())
    return out


@pytest.mark.parametrize("waves", [1, 4])
@pytest.mark.parametrize("n", WIDTHS)
def test_single_aliased_q_equals_separate_q(n, waves):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    A, _ = synth.prescribed_sigma(40000, n, seed=600 + n, decades=8)
    announce(f"alias single n={n} waves={waves}")
    Qs, Qa = _pair(T, torch, A, waves)
    assert np.array_equal(Qs, Qa)
    assert np.linalg.norm(Qa.T @ Qa - np.eye(n)) <= 20 * n * 2.0 ** -53


@pytest.mark.parametrize("waves", [1, 4])
def test_batched_aliased_q_equals_separate_q(waves):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    shapes = [(30000, 64), (9000, 49), (20000, 57), (5000, 20), (12000, 52), (3000, 64)]
    mats = [synth.gaussian(m, n, seed=640 + i) for i, (m, n) in enumerate(shapes)]
    ms, ns = [m for m, _ in shapes], [n for _, n in shapes]
    announce(f"alias batched waves={waves}")
    with T.BatchedPlan(ms, ns, waves=waves) as bp:
        res = []
        for alias in (False, True, False):  # both graphs, and back to the first
            As = [T.to_colmajor(torch.from_numpy(A)) for A in mats]
            bp.factor(As)
            Qs = bp.form_q(As, As if alias else [T.colmajor(m, n) for m, n in shapes])
            torch.cuda.synchronize()
            res.append([Q.cpu().numpy() for Q in Qs])
    for i in range(len(shapes)):
        assert np.array_equal(res[0][i], res[1][i]) and np.array_equal(res[0][i], res[2][i]), shapes[i]
