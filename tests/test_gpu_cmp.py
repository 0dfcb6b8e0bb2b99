"""TSQR's competitors of Sec. 5 on the GPU (CholeskyQR, CholeskyQR2, CGS,
MGS) through the C ABI, against the plain CPU oracle of each: R and Q on
well-conditioned inputs element by element, the loss of orthogonality on
ill-conditioned ones (no worse than the oracle's, and the kappa^2 / kappa
growth the paper contrasts with Householder QR), breakdowns, and Q written
over A."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import backward_error, fp64_bound, orthogonality, rel_diff

pytestmark = pytest.mark.gpu

METHODS = ["cholqr", "cholqr2", "cgs", "mgs"]
ORACLE = {"cholqr": oracle.cholqr, "cholqr2": oracle.cholqr2, "cgs": oracle.cgs, "mgs": oracle.mgs}


def _gpu(A, method, alias=False):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = A.shape
    Ad = T.to_colmajor(torch.from_numpy(A))
    with T.CmpPlan(m, n, method) as p:
        Q, R = p.factor(Ad, Ad if alias else None)
        info = p.breakdown()
    return Q.cpu().numpy(), R.cpu().numpy(), info


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("m,n", [(10000, 5), (9001, 16), (4099, 17), (12345, 33), (8200, 64)])
def test_well_conditioned_matches_the_oracle(method, m, n):
    A, _ = synth.prescribed_sigma(m, n, seed=700 + n, decades=1)
    announce(f"cmp {method} m={m} n={n}")
    Q, R, info = _gpu(A, method)
    Qo, Ro, info_o = ORACLE[method](A)
    assert info == 0 and info_o == 0
    assert rel_diff(R, Ro) <= 1e-13
    assert np.abs(Q - Qo).max() <= 1e-12
    assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)
    assert backward_error(A, Q, R) <= fp64_bound(n)
    assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-13


def test_loss_of_orthogonality_tracks_the_oracle():
    """kappa 1e3 and 1e5: each method's GPU orthogonality is no worse than the
    oracle's; CholeskyQR and CGS grow with kappa^2, MGS with kappa,
    CholeskyQR2 stays at working precision."""
    got = {}
    for d in (3, 5):
        A, _ = synth.prescribed_sigma(20000, 10, seed=710, decades=d)
        for method in METHODS:
            announce(f"cmp orthogonality {method} kappa 1e{d}")
            Q, R, info = _gpu(A, method)
            Qo, Ro, _ = ORACLE[method](A)
            assert info == 0
            o, oo = orthogonality(Q), orthogonality(Qo)
            got[method, d] = o
            if method == "cholqr2":
                assert o <= fp64_bound(10) and oo <= fp64_bound(10)
            else:
                # the GPU's sums are pairwise over row chunks, the oracle's
                # sequential over all m rows: its loss can be far smaller,
                # never much larger
                assert o <= 10 * oo, (method, d, o, oo)
            assert backward_error(A, Q, R) <= 1e-12
    assert got["cholqr", 5] / got["cholqr", 3] >= 1e3
    assert got["cgs", 5] / got["cgs", 3] >= 1e3
    assert 10 <= got["mgs", 5] / got["mgs", 3] <= 1e3


def test_breakdowns_are_reported():
    A, _ = synth.prescribed_sigma(20000, 10, seed=720, decades=12)
    for method in ("cholqr", "cholqr2"):
        announce(f"cmp breakdown {method}")
        _, _, info = _gpu(A, method)
        assert info > 0  # kappa^2 eps >> 1: a Cholesky pivot that is not positive
    B = synth.gaussian(5000, 6, 721)
    B[:, 3] = 0.0
    for method in METHODS:
        _, _, info = _gpu(B, method)
        assert info == 4, method  # the zero column (index 3) is the first to break down


@pytest.mark.parametrize("method", METHODS)
def test_q_over_a_equals_separate_q(method):
    A, _ = synth.prescribed_sigma(7777, 24, seed=730, decades=2)
    Q1, R1, _ = _gpu(A, method)
    Q2, R2, _ = _gpu(A, method, alias=True)
    assert np.array_equal(Q1, Q2) and np.array_equal(R1, R2)


def test_full_size_against_tsqr():
    """m = 2^22, n = 32, Gaussian: every method's R against the FP64 TSQR R
    (uniqueness of R, Sec. 2) and its backward error."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = 1 << 22, 32
    g = torch.Generator(device="cuda")
    g.manual_seed(731)
    A = torch.randn((n, m), generator=g, device="cuda", dtype=torch.float64).t()
    with T.Plan(m, n, want_q=False) as p:
        Rt = p.factor(A).cpu().numpy()
    for method in METHODS:
        announce(f"cmp full size {method}")
        with T.CmpPlan(m, n, method) as p:
            Q, R = p.factor(A)
            assert p.breakdown() == 0
        Rh = R.cpu().numpy()
        assert rel_diff(Rh, Rt) <= 1e-13
        with torch.no_grad():
            bwd = float(torch.linalg.norm(torch.addmm(A, Q, R, alpha=-1.0)) / torch.linalg.norm(A))
        assert bwd <= fp64_bound(n)
