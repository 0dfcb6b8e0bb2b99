"""A plan's calls captured into a HIP graph on the plan's stream and replayed.

factor_into forks the T construction onto the plan's side stream and joins it
back with events; under stream capture that fork and join must become graph
edges.  Every replay (with eager work and synchronisations between replays) is
compared with the eager result of the same calls, and with the oracle's
bounds."""
import numpy as np
import pytest

import synth
from gpu_util import announce, need_gpu
from metrics import backward_error, fp64_bound, orthogonality

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,precision", [(20000, 32, "fp64"), (9000, 64, "fp64"), (12000, 40, "mixed")])
def test_captured_factor_and_q_replay_equal_eager(m, n, precision):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    A = synth.gaussian(m, n, seed=900 + n)
    announce(f"graph capture {m}x{n} {precision}")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        A0 = T.to_colmajor(torch.from_numpy(A))
        Ad = T.colmajor(m, n)
        V = T.colmajor(m, n) if precision == "fp64" else None
        Q = T.colmajor(m, n)
        R = T.colmajor(n, n)
        p = T.Plan(m, n, precision=precision, stream=s)

        def step():
            Ad.copy_(A0)
            p.factor_into(Ad, V, R)
            p.form_q(V, Q)

        step()
        s.synchronize()
        R_eager, Q_eager = R.cpu().numpy(), Q.cpu().numpy()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            step()
        for rep in range(3):
            R.zero_()
            Q.zero_()
            junk = torch.randn(1 << 20, device="cuda")  # eager work between replays
            junk.mul_(2.0)
            s.synchronize()
            g.replay()
            s.synchronize()
            announce(f"graph replay {rep}")
            Rg, Qg = R.cpu().numpy(), Q.cpu().numpy()
            assert np.array_equal(Rg, R_eager) and np.array_equal(Qg, Q_eager)
        p.close()
    bound = fp64_bound(n) if precision == "fp64" else 1e-6
    assert backward_error(A, Q_eager, R_eager) <= bound
    if precision == "fp64":
        assert orthogonality(Q_eager) <= fp64_bound(n)
    else:
        assert orthogonality(Q_eager) <= 1e-13
