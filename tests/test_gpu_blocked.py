"""The blocked factorization of chained tiles (16-column panels, the compact-WY
update of the later columns on the matrix cores) against the oracle run on the
same tree: widths that pad to 32 columns, ragged last tiles, and exactly zero
columns (tau = 0 reflectors inside a panel), for which the reflector sequence
is still unique, so R and Q are compared element by element."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu, run_tsqr
from metrics import backward_error, fp64_bound, is_upper, orthogonality, rel_diff

pytestmark = pytest.mark.gpu


def _elementwise(A, R, Q, info):
    n = A.shape[1]
    assert is_upper(R) and np.all(np.diag(R) >= 0)
    t = oracle.TSQR(A, info["leaf_rows"], info["tile_rows"])
    Ro, Qo = t.R(), t.form_q()
    assert np.abs(R - Ro).max() <= 1e-13 * np.linalg.norm(Ro)
    assert np.abs(Q - Qo).max() <= 1e-13
    assert backward_error(A, Q, R) <= fp64_bound(n)
    assert orthogonality(Q) <= fp64_bound(n)


@pytest.mark.parametrize("n", [29, 30, 31, 32])
@pytest.mark.parametrize("tree", [dict(tree="flat"), dict(tree="hybrid", flat_len=3)], ids=["flat", "hybrid3"])
def test_padded_widths_and_ragged_tiles(n, tree):
    need_gpu()
    m = 40 * 128 + 37  # the last tile of the chain has 37 rows
    A = synth.gaussian(m, n, seed=700 + n)
    announce(f"blocked {m}x{n} {tree}")
    R, Q, _, info = run_tsqr(A, **tree)
    assert info["tile_rows"] == 128
    _elementwise(A, R, Q, info)


@pytest.mark.parametrize("zero_cols", [(5,), (21,), (3, 16, 31)])
def test_zero_columns_inside_panels(zero_cols):
    need_gpu()
    m, n = 20 * 128 + 5, 32
    A = synth.gaussian(m, n, seed=800 + sum(zero_cols))
    A[:, list(zero_cols)] = 0.0
    announce(f"blocked zero columns {zero_cols}")
    R, Q, _, info = run_tsqr(A, tree="hybrid", flat_len=4)
    for c in zero_cols:
        assert R[c, c] == 0.0
    _elementwise(A, R, Q, info)


def test_r_only_matches_r_with_q():
    """The R-only leaf runs the same blocked factorization."""
    need_gpu()
    A, _ = synth.prescribed_sigma(30000, 32, seed=811, decades=12)
    announce("blocked R only vs R + Q")
    R1, _, _, _ = run_tsqr(A, want_q=False, tree="hybrid", flat_len=8)
    R2, _, _, _ = run_tsqr(A, want_q=True, tree="hybrid", flat_len=8)
    assert np.array_equal(R1, R2)
    assert rel_diff(R1, oracle.qr_reference(A, want_q=False)) <= 1e-13
