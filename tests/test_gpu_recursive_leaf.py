"""The recursive leaf variant (Elmroth and Gustavson's recursive local QR, which
Sec. 3.1 and Sec. 7 bring into TSQR): each tile's compact-WY factor
T = [T_L, -T_L Y_L^T Y_R T_R; 0, T_R] is put together inside the leaf kernel
from its 16-column blocks, instead of by a T kernel after the leaves.

Against the oracle run on the same tree (identical reflector sequence), element
by element on well-conditioned inputs, and through the bounds on ill-conditioned
ones; against the compact-WY variant, which runs the same factorisation code:
R and the stored reflectors are bitwise the same, Q and Q^T B agree to
roundoff."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import backward_error, fp64_bound, is_upper, orthogonality, rel_diff

pytestmark = pytest.mark.gpu


def _run(A, kind, B=None, alias=False, lda=None, **kw):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = A.shape
    Ad = T.colmajor(m, n, ld=lda or m)
    Ad.copy_(torch.from_numpy(np.ascontiguousarray(A)))
    with T.Plan(m, n, leaf_kind=kind, **kw) as p:
        info = p.info()
        R = p.factor(Ad)
        V = Ad.cpu().numpy()
        X = None
        if B is not None:
            Bd = T.to_colmajor(torch.from_numpy(B))
            p.apply_qt(Ad, Bd)
            X = Bd.cpu().numpy()
        Q = p.form_q(Ad, Ad if alias else T.colmajor(m, n))
        torch.cuda.synchronize()
        Qh = Q.cpu().numpy()
    return R.cpu().numpy(), Qh, V, X, info


CASES = [
    (40 * 128 + 37, 29, dict(tree="flat")),          # pads to 32; ragged last tile
    (40 * 128 + 37, 32, dict(tree="hybrid", flat_len=3)),
    (5000, 31, dict()),                              # automatic geometry
    (4096 + 37, 16, dict(tree="binary")),            # 256-row tiles, one per leaf
    (3000, 13, dict(tree="hybrid", flat_len=2)),     # pads to 16
    (128, 32, dict()),                               # a single tile
    (100, 32, dict()),                               # less than a tile
    (32, 32, dict()),                                # square
]


@pytest.mark.parametrize("m,n,kw", CASES)
def test_matches_oracle_and_compact_wy(m, n, kw):
    need_gpu()
    A = synth.gaussian(m, n, seed=900 + n + m % 7)
    B = synth.gaussian(m, 7, seed=901)
    announce(f"recursive leaf {m}x{n} {kw}")
    R, Q, V, X, info = _run(A, "recursive", B=B, **kw)
    assert info["leaf_kind"] == "recursive"
    R2, Q2, V2, X2, info2 = _run(A, "compact_wy", B=B, **kw)
    assert info2["leaf_kind"] == "compact_wy"
    assert info["leaf_rows"] == info2["leaf_rows"] and info["tile_rows"] == info2["tile_rows"]
    # same factorisation code: R and the reflectors bit for bit
    assert np.array_equal(R, R2) and np.array_equal(V, V2)
    assert np.abs(Q - Q2).max() <= 1e-14
    # the oracle on the same tree
    assert is_upper(R) and np.all(np.diag(R) >= 0)
    t = oracle.TSQR(A, info["leaf_rows"], info["tile_rows"])
    Ro, Qo = t.R(), t.form_q()
    assert np.abs(R - Ro).max() <= 1e-13 * np.linalg.norm(Ro)
    assert np.abs(Q - Qo).max() <= 1e-13
    assert np.abs(X - t.apply_qt(B)).max() <= 1e-13 * np.linalg.norm(B)
    assert backward_error(A, Q, R) <= fp64_bound(n)
    assert orthogonality(Q) <= fp64_bound(n)


@pytest.mark.parametrize("n", [16, 32])
def test_ill_conditioned_bounds(n):
    need_gpu()
    A, _ = synth.prescribed_sigma(60000, n, seed=910 + n, decades=12)
    announce(f"recursive leaf kappa=1e12 60000x{n}")
    R, Q, _, _, info = _run(A, "recursive")
    assert info["leaf_kind"] == "recursive"
    assert rel_diff(R, oracle.qr_reference(A, want_q=False)) <= 1e-13
    assert backward_error(A, Q, R) <= fp64_bound(n)
    assert orthogonality(Q) <= fp64_bound(n)


def test_zero_columns_and_q_over_a():
    """Exactly zero columns inside both 16-column blocks (tau = 0 reflectors),
    a leading dimension above m, and Q written over the reflectors."""
    need_gpu()
    m, n = 20 * 128 + 5, 32
    A = synth.gaussian(m, n, seed=920)
    A[:, [3, 16, 31]] = 0.0
    announce("recursive leaf zero columns, lda > m, Q over A")
    R, Q, _, _, info = _run(A, "recursive", alias=True, lda=m + 3, tree="hybrid", flat_len=4)
    for c in (3, 16, 31):
        assert R[c, c] == 0.0
    t = oracle.TSQR(A, info["leaf_rows"], info["tile_rows"])
    assert np.abs(Q - t.form_q()).max() <= 1e-13
    assert np.abs(R - t.R()).max() <= 1e-13 * np.linalg.norm(R)
