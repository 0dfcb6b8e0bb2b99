"""Pins for the CPU oracle: each test checks it against something other than
itself -- exact rational arithmetic, closed forms, invariants the paper states,
special inputs whose answer is known, and a library SVD for the spectrum."""
import os

import numpy as np
import pytest

import oracle
import synth
from exact_qr import exact_lstsq, exact_qr
from metrics import EPS, backward_error, fp64_bound, is_upper, orthogonality, rel_diff

# (leaf_rows, tile_rows) shapes of the hybrid tree used throughout:
# binary (tile == leaf), flat (one leaf), and hybrid chains
TREES_SMALL = [(64, 64), (10_000, 32), (128, 32), (96, 40)]


# ---------------------------------------------------------------- P1: exact rationals
@pytest.mark.parametrize("shape,seed", [((7, 4), 1), ((9, 5), 2), ((12, 3), 3), ((6, 6), 4), ((16, 4), 5)])
def test_exact_rational_R_and_Q(shape, seed):
    m, n = shape
    for attempt in range(20):
        A = synth.small_int_matrix(m, n, seed * 100 + attempt)
        ex = exact_qr(A)
        if ex is not None:
            break
    Rx, Qx = ex
    R, Q = oracle.qr_reference(A)
    scale = np.abs(Rx).max()
    assert np.abs(R - Rx).max() <= 8 * EPS * scale * n
    assert np.abs(Q - Qx).max() <= 64 * EPS * np.sqrt(m)
    # every tree shape gives the same R and Q (uniqueness, Sec. 2)
    for leaf, tile in [(n, n), (2 * n, n), (m, n), (max(n, m // 2), n)]:
        t = oracle.TSQR(A, leaf, tile)
        assert np.abs(t.R() - Rx).max() <= 16 * EPS * scale * n
        assert np.abs(t.form_q() - Qx).max() <= 128 * EPS * np.sqrt(m)


def test_exact_least_squares():
    A = synth.small_int_matrix(11, 4, 7)
    b = synth.small_int_matrix(11, 1, 8)[:, 0]
    x_exact = np.array([float(v) for v in exact_lstsq(A, b)])
    t = oracle.TSQR(A, 4, 4)
    qtb = t.apply_qt(b[:, None])[:, 0]
    x = _back_subst(t.R(), qtb[:4])
    assert np.abs(x - x_exact).max() <= 1e-12 * max(1.0, np.abs(x_exact).max())
    # residual norm equals the norm of the complement rows (P7)
    r_exact = b - A @ x_exact
    assert abs(np.linalg.norm(qtb[4:]) - np.linalg.norm(r_exact)) <= 1e-12 * np.linalg.norm(b)


def _back_subst(R, y):
    n = R.shape[0]
    x = np.zeros(n)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - R[i, i + 1:] @ x[i + 1:]) / R[i, i]
    return x


# ---------------------------------------------------------------- P2 / P3: uniqueness and stability
@pytest.mark.parametrize("m,n", [(2048, 16), (3000, 17), (1537, 8), (4096, 32)])
@pytest.mark.parametrize("tree", TREES_SMALL)
def test_tree_invariance_and_stability(m, n, tree):
    A, _ = synth.prescribed_sigma(m, n, seed=11 + n, decades=12)
    leaf, tile = tree
    R0, _ = oracle.qr_reference(A)
    t = oracle.TSQR(A, max(leaf, n), max(tile, n))
    R, Q = t.R(), t.form_q()
    assert is_upper(R)
    assert np.all(np.diag(R) >= 0)
    assert rel_diff(R, R0) <= 1e-13
    assert backward_error(A, Q, R) <= fp64_bound(n)
    assert orthogonality(Q) <= fp64_bound(n)


# ---------------------------------------------------------------- P4: closed forms
def test_closed_forms():
    A = synth.gaussian(777, 12, 3)
    t = oracle.TSQR(A, 100, 25)
    R = t.R()
    assert abs(R[0, 0] - np.sqrt(np.sum(A[:, 0] ** 2))) <= 4 * EPS * R[0, 0]
    # column norms are preserved by an orthogonal Q
    cn = np.sqrt(np.sum(A ** 2, axis=0))
    assert np.allclose(np.sqrt(np.sum(R ** 2, axis=0)), cn, rtol=1e-14, atol=0)


def test_single_column_is_norm_and_scaling():
    a = synth.gaussian(1000, 1, 5)
    t = oracle.TSQR(a, 64, 16)
    R, Q = t.R(), t.form_q()
    nrm = np.sqrt(np.sum(a[:, 0] ** 2))
    assert abs(R[0, 0] - nrm) <= 8 * EPS * nrm
    assert np.abs(Q[:, 0] - a[:, 0] / nrm).max() <= 1e-15


def test_one_leaf_one_tile_is_plain_householder():
    A = synth.gaussian(300, 9, 6)
    R0, Q0 = oracle.qr_reference(A)
    t = oracle.TSQR(A, 300, 300)
    assert np.array_equal(t.R(), R0)
    assert np.array_equal(t.form_q(), Q0)


# ---------------------------------------------------------------- P5: spectrum (Weyl)
def test_singular_values_of_R_match_prescribed():
    n = 24
    A, sig = synth.prescribed_sigma(4096, n, seed=21, decades=12)
    t = oracle.TSQR(A, 512, 128)
    s = np.linalg.svd(t.R(), compute_uv=False)
    assert np.max(np.abs(s - sig)) <= 100 * n * EPS * sig[0]


# ---------------------------------------------------------------- P6: special inputs
def test_orthonormal_input_gives_identity():
    U, _ = synth.prescribed_sigma(2000, 10, seed=1, decades=0)  # sigma = 1: orthonormal columns
    t = oracle.TSQR(U, 256, 64)
    assert np.abs(t.R() - np.eye(10)).max() <= 50 * EPS * 10


def test_triangle_on_zeros_gives_signed_triangle():
    n = 8
    rng = np.random.default_rng(3)
    R0 = np.triu(rng.standard_normal((n, n)))
    A = np.zeros((512, n))
    A[:n] = R0
    t = oracle.TSQR(A, 128, 32)
    D = np.where(np.diag(R0) < 0, -1.0, 1.0)
    assert np.abs(t.R() - D[:, None] * R0).max() <= 4 * EPS * np.abs(R0).max()


def test_apply_qt_of_A_and_of_Q():
    m, n = 1500, 7
    A = synth.gaussian(m, n, 9)
    t = oracle.TSQR(A, 200, 50)
    R, Q = t.R(), t.form_q()
    X = t.apply_qt(A)
    assert np.abs(X[:n] - R).max() <= 50 * EPS * np.linalg.norm(A)
    assert np.linalg.norm(X[n:]) <= fp64_bound(n) * np.linalg.norm(A)
    Y = t.apply_qt(Q)
    assert np.abs(Y[:n] - np.eye(n)).max() <= 50 * EPS * n
    assert np.linalg.norm(Y[n:]) <= fp64_bound(n)
    B = synth.gaussian(m, 5, 10)
    Z = t.apply_qt(B)
    assert abs(np.linalg.norm(Z) - np.linalg.norm(B)) <= 50 * EPS * np.linalg.norm(B)
    assert np.abs(Z[:n] - Q.T @ B).max() <= 1e-13 * np.linalg.norm(B)


# ---------------------------------------------------------------- P8: structure of a tree node
def test_tree_node_structure_and_block_update():
    n = 6
    A = synth.gaussian(8 * n, n, 12)
    t = oracle.TSQR(A, n, n)
    V, tau = t.node(0, 0)
    Vtop, Y1 = V[:n], V[n:]
    # the part of each reflector inside R_a is e_j: zero below the diagonal
    assert np.all(np.tril(Vtop, -1) == 0.0)
    # the part inside R_b is upper triangular (eq. fact_2rs)
    assert np.all(np.tril(Y1, -1) == 0.0)
    # compact-WY: H_0..H_{n-1} = I - Y T Y^T with Y = [I; Y1]; T by the forward recurrence
    Y = np.vstack([np.eye(n), np.triu(Y1)])
    T = np.zeros((n, n))
    for j in range(n):
        T[j, j] = tau[j]
        T[:j, j] = -tau[j] * T[:j, :j] @ (Y[:, :j].T @ Y[:, j])
    C = synth.gaussian(2 * n, 5, 13)
    # the update formulas of the trailing-matrix section: D = C0 + Y1^T C1,
    # C0 -= T^T D, C1 -= Y1 T^T D, must equal the reflector-by-reflector Q^T C
    C0, C1 = C[:n], C[n:]
    D = C0 + np.triu(Y1).T @ C1
    ref = oracle.apply_qt(V, tau, C)
    assert np.abs((C0 - T.T @ D) - ref[:n]).max() <= 1e-14 * np.abs(C).max()
    assert np.abs((C1 - np.triu(Y1) @ T.T @ D) - ref[n:]).max() <= 1e-14 * np.abs(C).max()


# ---------------------------------------------------------------- P9: tree indices
def test_tree_indices_worked_example():
    """P = 8: at level k = 2 processors 4..7 meet at first_proc 4 and
    target_first_proc 6; level(i,k) = floor(i/2^k), first = 2^k level,
    target = first + 2^(k-1)."""
    A = synth.gaussian(8 * 8, 4, 1)
    t = oracle.TSQR(A, 8, 8)
    assert t.num_leaves == 8 and t.num_levels == 3
    for k in (1, 2, 3):
        for i in range(8):
            lev = i // 2 ** k
            first = 2 ** k * lev
            target = first + 2 ** (k - 1)
            a, b = t.node_homes(k - 1, lev)
            assert (a, b) == (first, target)
    assert t.node_homes(1, 1) == (4, 6)
    # the rows of the worked example as the paper prints them (golden fixture)
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tree_index_p8.txt")
    rows = [list(map(int, ln.split())) for ln in open(golden) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 4
    for P, k, i, first, target in rows:
        assert P == t.num_leaves
        assert t.node_homes(k - 1, i // 2 ** k) == (first, target)


def test_odd_leaf_count_passes_up():
    assert oracle.tree_level_counts(5) == [3, 2, 1]
    A = synth.gaussian(5 * 16, 4, 2)
    t = oracle.TSQR(A, 16, 16)
    assert t.node(0, 2) is None  # leaf 4 passes up at the first stage
    assert t.node_homes(1, 1) == (4, -1)
    assert t.node_homes(2, 0) == (0, 4)


# ---------------------------------------------------------------- P10: negative control
def test_cholesky_qr_loses_orthogonality_on_krylov_basis():
    B = synth.krylov_basis(64, 16, seed=0)  # 4096 x 17, very ill-conditioned
    n = B.shape[1]
    G = B.T @ B
    try:
        Rc = np.linalg.cholesky(G).T
        Qc = np.linalg.solve(Rc.T, B.T).T
        chol_orth = orthogonality(Qc)
    except np.linalg.LinAlgError:
        chol_orth = np.inf
    assert chol_orth > 1e-6
    t = oracle.TSQR(B, 512, 128)
    Q, R = t.form_q(), t.R()
    assert orthogonality(Q) <= fp64_bound(n)
    assert backward_error(B, Q, R) <= fp64_bound(n)


# ---------------------------------------------------------------- rank deficiency (reading C2)
def test_exactly_dependent_column():
    A = synth.gaussian(400, 5, 4)
    A[:, 3] = 2.0 * A[:, 1] - A[:, 0]
    t = oracle.TSQR(A, 100, 50)
    R, Q = t.R(), t.form_q()
    assert abs(R[3, 3]) <= 1e-13 * np.linalg.norm(A)
    assert backward_error(A, Q, R) <= fp64_bound(5)
    assert orthogonality(Q) <= fp64_bound(5)


def test_zero_matrix_gives_zero_R_and_orthonormal_Q():
    A = np.zeros((300, 4))
    t = oracle.TSQR(A, 100, 50)
    assert np.all(t.R() == 0.0)
    Q = t.form_q()
    assert orthogonality(Q) <= fp64_bound(4)


# ---------------------------------------------------------------- planted mistakes are caught
def _pins_pass() -> bool:
    """A compact run of the pins above; False as soon as one fails."""
    try:
        A = synth.small_int_matrix(9, 4, 301)
        ex = exact_qr(A)
        Rx, Qx = ex
        t = oracle.TSQR(A, 4, 4)
        if np.abs(t.R() - Rx).max() > 1e-13 * np.abs(Rx).max():
            return False
        if np.abs(t.form_q() - Qx).max() > 1e-13:
            return False
        A2 = synth.gaussian(1000, 6, 302)  # ragged: leaf rows 128, last leaf absorbs 104
        t2 = oracle.TSQR(A2, 128, 32)
        R2, Q2 = t2.R(), t2.form_q()
        if backward_error(A2, Q2, R2) > fp64_bound(6) or orthogonality(Q2) > fp64_bound(6):
            return False
        if not (is_upper(R2) and np.all(np.diag(R2) >= 0)):
            return False
        X = t2.apply_qt(A2)
        if np.abs(X[:6] - R2).max() > 1e-13 * np.linalg.norm(A2):
            return False
        return True
    except Exception:
        return False


@pytest.mark.parametrize("code", [1, 2, 3, 4, 5, 6, 7])
def test_planted_mistakes_fail_the_pins(code):
    assert _pins_pass()
    try:
        oracle.set_mutation(code)
        assert not _pins_pass(), f"planted mistake {code} went unnoticed"
    finally:
        oracle.set_mutation(0)
    assert _pins_pass()
