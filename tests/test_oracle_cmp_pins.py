"""Pins for the oracle of TSQR's competitors (Sec. 5: CholeskyQR, classical
and modified Gram-Schmidt, and CholeskyQR applied twice), each against
something other than itself: the exact-rational R, the Householder oracle on
well-conditioned inputs, the closed form R_11 = ||a_1||, and the stability
contrast the paper states -- the orthogonality of CholeskyQR's Q degrades
quadratically with the condition number (Sec. 5), that of MGS linearly, while
Householder QR (and TSQR) stays at machine precision."""
import numpy as np
import pytest

import oracle
import synth
from exact_qr import exact_qr
from metrics import EPS, backward_error, fp64_bound, orthogonality, rel_diff

METHODS = {"cholqr": oracle.cholqr, "cholqr2": oracle.cholqr2, "cgs": oracle.cgs, "mgs": oracle.mgs}


@pytest.mark.parametrize("name", sorted(METHODS))
@pytest.mark.parametrize("shape,seed", [((7, 4), 11), ((12, 5), 12), ((16, 3), 13)])
def test_exact_rational_R(name, shape, seed):
    m, n = shape
    for attempt in range(20):
        A = synth.small_int_matrix(m, n, seed * 100 + attempt)
        ex = exact_qr(A)
        if ex is not None:
            break
    Rx, _ = ex
    Q, R, info = METHODS[name](A)
    assert info == 0
    # these small integer matrices are well conditioned: every method is accurate
    assert np.abs(R - Rx).max() <= 1e3 * EPS * np.abs(Rx).max()
    assert np.all(np.diag(R) > 0) and np.all(np.tril(R, -1) == 0)


@pytest.mark.parametrize("name", sorted(METHODS))
def test_well_conditioned_agrees_with_householder(name):
    A, _ = synth.prescribed_sigma(3000, 12, seed=21, decades=1)
    Q, R, info = METHODS[name](A)
    assert info == 0
    assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-13
    assert backward_error(A, Q, R) <= fp64_bound(12)
    assert orthogonality(Q) <= 1e-12
    assert abs(R[0, 0] - np.linalg.norm(A[:, 0])) <= 1e-14 * R[0, 0]  # closed form


def _orth(name, decades, seed=22, m=2000, n=10):
    A, _ = synth.prescribed_sigma(m, n, seed=seed, decades=decades)
    Q, R, info = METHODS[name](A)
    return orthogonality(Q) if info == 0 else np.inf, info


def test_stability_contrast_in_the_condition_number():
    """kappa = 1e3 -> 1e5: CholeskyQR and CGS lose about kappa^2 more, MGS about
    kappa more, CholeskyQR2 stays at O(eps) while kappa^2 eps < 1."""
    ch3, _ = _orth("cholqr", 3)
    ch5, _ = _orth("cholqr", 5)
    cg3, _ = _orth("cgs", 3)
    cg5, _ = _orth("cgs", 5)
    mg3, _ = _orth("mgs", 3)
    mg5, _ = _orth("mgs", 5)
    assert ch5 / ch3 >= 1e3 and cg5 / cg3 >= 1e3      # quadratic in kappa (a factor 1e4 ideally)
    assert 10.0 <= mg5 / mg3 <= 1e3                   # linear in kappa (a factor 1e2 ideally)
    assert mg5 <= 1e5 * 1e3 * EPS                     # MGS: O(kappa eps)
    for d in (3, 5, 7):
        o, info = _orth("cholqr2", d)
        assert info == 0 and o <= fp64_bound(10)
    # the Householder oracle at the same kappa: machine precision
    A, _ = synth.prescribed_sigma(2000, 10, seed=22, decades=7)
    assert orthogonality(oracle.qr_reference(A)[1]) <= fp64_bound(10)


def test_cholesky_breaks_down_where_kappa_squared_exceeds_one_over_eps():
    A, _ = synth.prescribed_sigma(2000, 10, seed=23, decades=12)
    for name in ("cholqr", "cholqr2"):
        Q, R, info = METHODS[name](A)
        assert info > 0  # a pivot that is not positive: G is not numerically positive definite
    B = synth.krylov_basis(64, 16, seed=0)  # the s-step basis (n = 17): kappa ~ 1e11
    _, _, info = oracle.cholqr(B)
    Qc, _, _ = oracle.cgs(B)
    assert info > 0 or orthogonality(Qc) > 1e-2


def test_zero_column_is_reported():
    A = synth.gaussian(500, 4, 24)
    A[:, 2] = 0.0
    for name in ("cgs", "mgs"):
        _, _, info = METHODS[name](A)
        assert info == 3
    _, _, info = oracle.cholqr(A)
    assert info == 3


def _cmp_pins_pass() -> bool:
    try:
        A = synth.small_int_matrix(9, 4, 301)
        Rx, _ = exact_qr(A)
        for f in METHODS.values():
            Q, R, info = f(A)
            if info or np.abs(R - Rx).max() > 1e3 * EPS * np.abs(Rx).max():
                return False
        A2, _ = synth.prescribed_sigma(1500, 8, seed=25, decades=1)
        for f in METHODS.values():
            Q, R, info = f(A2)
            if info or backward_error(A2, Q, R) > fp64_bound(8) or orthogonality(Q) > 1e-12:
                return False
        c3, _ = _orth("cgs", 3)
        c5, _ = _orth("cgs", 5)
        if c5 / c3 < 1e3:
            return False
        return True
    except Exception:
        return False


@pytest.mark.parametrize("code", [8, 9, 10])
def test_planted_mistakes_fail_the_cmp_pins(code):
    assert _cmp_pins_pass()
    try:
        oracle.set_mutation(code)
        assert not _cmp_pins_pass(), f"planted mistake {code} went unnoticed"
    finally:
        oracle.set_mutation(0)
    assert _cmp_pins_pass()
