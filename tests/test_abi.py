"""C-ABI checks that need no GPU: the library loads, exports every function
include/tsqr.h declares, rejects bad arguments before touching a device, and
its layout (leaves, tiles, tree) follows the paper's partition rules."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "tsqr.h")).read()
    return sorted(set(re.findall(r"\b(tsqr_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    from paper_0809_2407_amd import _lib
    assert _declared_functions() == sorted(_lib.EXPORTED)


def test_library_exports_every_declared_symbol():
    from paper_0809_2407_amd import _lib
    lib = _lib.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_status_strings_and_version():
    from paper_0809_2407_amd import _lib
    lib = _lib.load()
    assert lib.tsqr_status_string(0) == b"success"
    assert b"invalid argument" in lib.tsqr_status_string(-2)
    assert b"out of order" in lib.tsqr_status_string(4)
    assert lib.tsqr_version() >= 100


def test_argument_errors_without_device():
    from paper_0809_2407_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.tsqr_plan_create(None, 100, 4, 0, None, None) == -1
    assert lib.tsqr_plan_create(ctypes.byref(h), 3, 4, 0, None, None) == -2  # m < n
    assert lib.tsqr_plan_create(ctypes.byref(h), -1, 0, 0, None, None) == -2
    assert lib.tsqr_plan_create(ctypes.byref(h), 100, -1, 0, None, None) == -3
    assert lib.tsqr_plan_create(ctypes.byref(h), 1000, 65, 0, None, None) == 3  # n > 64 unsupported
    assert lib.tsqr_plan_create(ctypes.byref(h), 1000, 8, 7, None, None) == -4
    bad = _lib.TsqrOpts(9, 0, 0, 0, 0, 1)
    assert lib.tsqr_plan_create(ctypes.byref(h), 1000, 8, 0, ctypes.byref(bad), None) == -5
    bad = _lib.TsqrOpts(0, 0, 0, 0, 3, 1)  # waves must be 1, 2 or 4
    assert lib.tsqr_plan_create(ctypes.byref(h), 1000, 8, 0, ctypes.byref(bad), None) == -5
    assert lib.tsqr_factor(None, 1, 1, 1, 1) == -1
    assert lib.tsqr_form_q(None, 1, 1, 1, 1) == -1
    assert lib.tsqr_apply_qt(None, 1, 1, 1, 1, 1) == -1
    assert lib.tsqr_plan_info(None, None) == -1
    assert lib.tsqr_plan_destroy(None) == -1
    out = _lib.TsqrInfo()
    assert lib.tsqr_plan_query(3, 4, 0, None, ctypes.byref(out)) == -1
    assert lib.tsqr_plan_query(100, -1, 0, None, ctypes.byref(out)) == -2
    assert lib.tsqr_plan_query(100, 4, 5, None, ctypes.byref(out)) == -3
    assert lib.tsqr_plan_query(100, 4, 0, None, None) == -5


def _query(**kw):
    from paper_0809_2407_amd.tsqr import plan_query
    return plan_query(**kw)


@pytest.mark.parametrize("n", [1, 3, 4, 8, 16, 17, 20, 32, 33, 48, 49, 52, 53, 56, 57, 60, 61, 64])
def test_tile_rows_respect_fast_memory_bound(n):
    """m/P * n + n(n+1)/2 <= W (Sec. 4.2) with W the per-wavefront register
    budget for the tile (64 doubles per lane, 4096 per wavefront)."""
    q = _query(m=1 << 20, n=n)
    np_ = q["n_padded"]
    # n rounded up to a multiple of 4; widths 49-52 run on the 56-column kernels, 57-60 on the 64-column ones
    assert np_ == (64 if 57 <= n <= 60 else (56 if 49 <= n <= 52 else (n + 3) // 4 * 4))
    assert q["tile_rows"] * np_ <= 64 * 64
    assert q["tile_rows"] >= np_


def test_leaf_partition_last_leaf_absorbs_remainder():
    q = _query(m=4096, n=16, leaf_rows=512)
    assert q["num_leaves"] == 8 and q["tree_levels"] == 3 and q["tree"] == 1 + 2  # hybrid: 2 tiles per leaf
    q = _query(m=4096 + 300, n=16, leaf_rows=512)
    assert q["num_leaves"] == 8  # 300 extra rows go to the last leaf
    assert q["num_tiles"] == 7 * 2 + (512 + 300 + 255) // 256
    q = _query(m=500, n=16, leaf_rows=512)
    assert q["num_leaves"] == 1 and q["tree_levels"] == 0


def test_tree_shapes():
    b = _query(m=1 << 16, n=32, tree="binary")
    assert b["leaf_rows"] == b["tile_rows"] and b["num_leaves"] == (1 << 16) // b["tile_rows"]
    f = _query(m=1 << 16, n=32, tree="flat")
    assert f["num_leaves"] == 1 and f["tree_levels"] == 0
    h = _query(m=1 << 16, n=32, tree="hybrid", flat_len=8)
    assert h["leaf_rows"] == 8 * h["tile_rows"]
    assert h["tree_levels"] == (h["num_leaves"] - 1).bit_length()


def test_levels_match_binary_pairing():
    for P in [1, 2, 3, 5, 8, 13, 4096, 4097]:
        q = _query(m=P * 128, n=32, leaf_rows=128)
        assert q["num_leaves"] == P
        L, c = 0, P
        while c > 1:
            c = (c + 1) // 2
            L += 1
        assert q["tree_levels"] == L


@pytest.mark.parametrize("prec,want_q", [(0, 1), (0, 0), (1, 1)])
def test_empty_problem_plans_need_no_device(prec, want_q):
    """n = 0 (any m >= 0): a plan with no workspace whose calls check their
    leading dimensions, reference no matrix (NULL pointers pass), launch
    nothing and return 0; call order is still enforced.  No device is touched,
    so this runs without a GPU."""
    from paper_0809_2407_amd import _lib
    lib = _lib.load()
    for m in (0, 10):
        out = _lib.TsqrInfo()
        assert lib.tsqr_plan_query(m, 0, prec, None, ctypes.byref(out)) == 0
        assert (out.m, out.n, out.num_leaves, out.num_tiles, out.workspace_bytes) == (m, 0, 0, 0, 0)
        h = ctypes.c_void_p()
        opts = _lib.TsqrOpts(0, 0, 0, 0, 0, want_q, 0)
        assert lib.tsqr_plan_create(ctypes.byref(h), m, 0, prec, ctypes.byref(opts), None) == 0
        assert lib.tsqr_form_q(h, None, m, None, m) == 4  # nothing factored yet
        assert lib.tsqr_factor(h, None, m - 1, None, 0) == -3  # lda < m
        assert lib.tsqr_factor(h, None, m, None, 0) == 0
        dummy = 8  # never dereferenced: Q^T B = B without reflectors
        if want_q:
            assert lib.tsqr_form_q(h, None, m, None, m) == 0
            assert lib.tsqr_apply_qt(h, None, m, 3, dummy, m) == 0
            assert lib.tsqr_apply_qt(h, None, m, 3, None, m) == (-5 if m > 0 else 0)  # 0 x 3: not referenced
            assert lib.tsqr_apply_qt(h, None, m, -1, dummy, m) == -4
            if m > 0:
                assert lib.tsqr_apply_qt(h, None, m, 3, dummy, m - 1) == -6
                assert lib.tsqr_form_q(h, None, m, None, m - 1) == -5
        else:
            assert lib.tsqr_form_q(h, None, m, None, m) == 4
        if prec == 1:
            assert lib.tsqr_mixed_q1(h, None, m) == 0
        assert lib.tsqr_plan_info(h, ctypes.byref(out)) == 0
        assert (out.m, out.n, out.workspace_bytes, out.reorth_applied) == (m, 0, 0, 0)
        assert lib.tsqr_plan_destroy(h) == 0
        # the allocation-free entry point and CAQR take the same convention
        assert lib.tsqr_factor_r_noalloc(m, 0, None, m, None, 0, None, ctypes.byref(out)) == 0
        assert (out.m, out.n) == (m, 0)
        c = ctypes.c_void_p()
        assert lib.tsqr_caqr_plan_create(ctypes.byref(c), m, 0, 0, None) == 0
        assert lib.tsqr_caqr_factor(c, None, m, None, 0) == 0
        assert lib.tsqr_caqr_factor_rhs(c, None, m, None, 0, 2) == 0
        assert lib.tsqr_caqr_apply_qt(c, None, m, 2, dummy, m) == 0
        assert lib.tsqr_caqr_plan_destroy(c) == 0


def test_batched_argument_errors_without_device():
    from paper_0809_2407_amd import _lib
    lib = _lib.load()
    P = ctypes.c_void_p()
    I64 = ctypes.c_int64 * 2
    ms, ns = I64(100, 200), I64(8, 16)
    assert lib.tsqr_batched_plan_create(None, 2, ms, ns, 0, None, None) == -1
    assert lib.tsqr_batched_plan_create(ctypes.byref(P), 0, ms, ns, 0, None, None) == -2
    assert lib.tsqr_batched_plan_create(ctypes.byref(P), 2, None, ns, 0, None, None) == -3
    assert lib.tsqr_batched_plan_create(ctypes.byref(P), 2, ms, None, 0, None, None) == -4
    assert lib.tsqr_batched_plan_create(ctypes.byref(P), 2, ms, ns, 7, None, None) == -5
    assert lib.tsqr_batched_plan_create(ctypes.byref(P), 2, I64(100, 10), ns, 0, None, None) == -3
    assert lib.tsqr_batched_plan_create(ctypes.byref(P), 2, ms, I64(8, -1), 0, None, None) == -3
    assert lib.tsqr_batched_plan_create(ctypes.byref(P), 2, ms, I64(8, 65), 0, None, None) == 3
    assert lib.tsqr_batched_factor(None, None, None, None, None) == -1
    assert lib.tsqr_batched_plan_destroy(None) == -1


def test_tune_cache_roundtrip(tmp_path):
    import json

    from paper_0809_2407_amd import tsqr as T
    path = str(tmp_path / "tune.json")
    assert T.tune_cache_lookup(path, 100000, 16) is None  # no file: empty cache
    T.tune_cache_store(path, 100000, 16, {"tree": "hybrid", "flat_len": 4, "waves": 2}, 1.25)
    T.tune_cache_store(path, 1 << 24, 32, {"tree": "binary", "waves": 4}, 6.5)
    T.tune_cache_store(path, 1 << 24, 32, {"tree": "flat", "waves": 1, "want_q": False}, 2.5)
    doc = json.load(open(path))  # the cache is plain JSON
    assert len(doc["entries"]) == 3
    hit = T.tune_cache_lookup(path, 120000, 16)  # same bucket: floor(log2 m) = 16
    assert hit["opts"]["tree"] == "hybrid" and hit["opts"]["flat_len"] == 4 and hit["ms"] == 1.25
    assert T.tune_cache_lookup(path, 200000, 16) is None  # bucket 17
    assert T.tune_cache_lookup(path, 100000, 16, precision="mixed") is None
    assert T.tune_cache_lookup(path, 1 << 24, 32)["opts"]["tree"] == "binary"
    assert T.tune_cache_lookup(path, 1 << 24, 32, want_q=False)["opts"]["tree"] == "flat"
    T.tune_cache_store(path, 100000, 16, {"tree": "binary", "waves": 4}, 0.5)  # replaces
    assert T.tune_cache_lookup(path, 100000, 16)["opts"]["tree"] == "binary"
    assert len(json.load(open(path))["entries"]) == 3
    with open(path, "w") as f:
        f.write("not json at all")
    assert T.tune_cache_lookup(path, 100000, 16) is None  # unreadable: treated as empty


def test_tune_cache_skips_entries_no_option_can_take(tmp_path):
    """Hand-edited or damaged cache entries (a tree out of range, a fractional
    leaf length, a huge wave count) read as absent; a store of an out-of-range
    tree is refused."""
    import json

    from paper_0809_2407_amd import _lib
    from paper_0809_2407_amd import tsqr as T
    path = str(tmp_path / "tune.json")
    T.tune_cache_store(path, 100000, 16, {"tree": "hybrid", "flat_len": 4, "waves": 2}, 1.25)
    doc = json.load(open(path))
    (key, good), = doc["entries"].items()
    for field, bad in (("tree", 9), ("tree", -1), ("leaf_rows", 1.5), ("waves", 1e30), ("flat_len", -3),
                       ("want_q", 2), ("leaf_kind", 7)):
        e = dict(good, **{field: bad})
        json.dump({"format": doc["format"], "entries": {key: e}}, open(path, "w"))
        assert T.tune_cache_lookup(path, 100000, 16) is None, (field, bad)
    json.dump(doc, open(path, "w"))
    assert T.tune_cache_lookup(path, 100000, 16)["opts"]["flat_len"] == 4
    lib = _lib.load()
    bad = _lib.TsqrOpts(9, 0, 0, 0, 0, 1)
    assert lib.tsqr_tune_cache_store(path.encode(), 100000, 16, 0, ctypes.byref(bad), 1.0) == -5


def test_tuned_options_reach_plan_query(tmp_path, monkeypatch):
    from paper_0809_2407_amd import tsqr as T
    path = str(tmp_path / "tune.json")
    base = T.plan_query(1 << 20, 32)
    T.tune_cache_store(path, 1 << 20, 32, {"tree": "hybrid", "flat_len": 3, "waves": 1}, 1.0)
    monkeypatch.setenv("TSQR_TUNE_CACHE", path)
    tuned = T.plan_query(1 << 20, 32)
    assert tuned["leaf_rows"] == 3 * tuned["tile_rows"] and tuned["waves"] == 1
    assert base["leaf_rows"] != tuned["leaf_rows"]


def test_mixed_plan_geometry():
    """A mixed plan: FP32 tiles of twice the FP64 height, FP32 chains capped at 64
    tiles, and a workspace that holds V32, Q1 and the second pass."""
    from paper_0809_2407_amd import tsqr as T
    f64 = T.plan_query(1 << 24, 64)
    mx = T.plan_query(1 << 24, 64, precision="mixed")
    # the FP32 tile of the mixed leaf holds twice the rows in the same registers
    assert mx["precision"] == 1 and mx["tile_rows"] == 2 * f64["tile_rows"] == 128
    assert mx["leaf_rows"] <= 64 * mx["tile_rows"]
    # V32 and Q1: 2 x 4 bytes per element at least
    assert mx["workspace_bytes"] >= 8 * (1 << 24) * 64
    # R only: no FP32 cap needed for accuracy of Q, still FP32 tiles
    r_only = T.plan_query(1 << 20, 16, precision="mixed", want_q=False)
    assert r_only["precision"] == 1


def test_binding_rejects_views_the_kernels_would_overrun():
    """Leading dimensions come from the tensor's strides: an expanded or
    overlapping view (column stride below the row count) is refused before
    any launch."""
    import torch

    from paper_0809_2407_amd.tsqr import _ld

    base = torch.zeros(10, 1, dtype=torch.float64)
    with pytest.raises(ValueError, match="column stride"):
        _ld(base.expand(10, 3), 10, "A")
    over = torch.zeros(40, dtype=torch.float64).as_strided((10, 3), (1, 5))
    with pytest.raises(ValueError, match="column stride"):
        _ld(over, 10, "A")
    ok = torch.zeros(3, 12, dtype=torch.float64).t()[:10]  # ld 12, the last column ends at 34 < 36
    with pytest.raises(ValueError, match="device tensor"):
        _ld(ok, 10, "A")


def test_comparison_and_streamed_plans_reject_arguments_without_device():
    """The Sec. 5 comparison plans and the out-of-HBM plans check their
    arguments before any device call."""
    from paper_0809_2407_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.tsqr_cmp_plan_create(None, 100, 4, 0, None) == -1
    assert lib.tsqr_cmp_plan_create(ctypes.byref(h), 3, 4, 0, None) == -2
    assert lib.tsqr_cmp_plan_create(ctypes.byref(h), 100, 0, 0, None) == -3
    assert lib.tsqr_cmp_plan_create(ctypes.byref(h), 100, 65, 0, None) == 3
    assert lib.tsqr_cmp_plan_create(ctypes.byref(h), 100, 4, 9, None) == -4
    assert lib.tsqr_cmp_factor(None, 1, 1, 1, 1, 1, 1) == -1
    assert lib.tsqr_cmp_breakdown(None, None) == -1
    assert lib.tsqr_cmp_plan_destroy(None) == -1
    assert lib.tsqr_stream_plan_create(None, 100, 4, 0, None) == -1
    assert lib.tsqr_stream_plan_create(ctypes.byref(h), 3, 4, 0, None) == -2
    assert lib.tsqr_stream_plan_create(ctypes.byref(h), 100, 0, 0, None) == -3
    assert lib.tsqr_stream_plan_create(ctypes.byref(h), 100, 65, 0, None) == 3
    assert lib.tsqr_stream_plan_create(ctypes.byref(h), 100, 8, 5, None) == -4  # blocks below n rows
    assert lib.tsqr_stream_factor(None, 1, 1, 1, 1) == -1
    assert lib.tsqr_stream_plan_info(None, None, None) == -1
    assert lib.tsqr_stream_plan_destroy(None) == -1


def test_caqr_plans_reject_arguments_without_device():
    from paper_0809_2407_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.tsqr_caqr_plan_create(None, 100, 4, 0, None) == -1
    assert lib.tsqr_caqr_plan_create(ctypes.byref(h), 3, 4, 0, None) == -2
    assert lib.tsqr_caqr_plan_create(ctypes.byref(h), 100, -1, 0, None) == -3
    assert lib.tsqr_caqr_plan_create(ctypes.byref(h), 100, 4, 65, None) == -4
    assert lib.tsqr_caqr_factor(None, 1, 1, 1, 1) == -1
    assert lib.tsqr_caqr_factor_rhs(None, 1, 1, 1, 1, 0) == -1
    assert lib.tsqr_caqr_apply_qt(None, 1, 1, 1, 1, 1) == -1
    assert lib.tsqr_caqr_plan_info(None, None, None) == -1
    assert lib.tsqr_caqr_plan_destroy(None) == -1


def test_leaf_kind_choice_and_errors():
    """The recursive leaf variant exists for FP64 with Q at padded widths 16
    and 32; asked for elsewhere (FP64 with Q) it is an argument error, and
    without Q or on a MIXED plan the variants coincide and the field is
    ignored."""
    from paper_0809_2407_amd import tsqr as T
    for n in (13, 16, 29, 32):
        assert T.plan_query(1 << 16, n, leaf_kind="recursive")["leaf_kind"] == "recursive"
        assert T.plan_query(1 << 16, n, leaf_kind="compact_wy")["leaf_kind"] == "compact_wy"
    for n in (8, 20, 33, 48, 64):
        assert T.plan_query(1 << 16, n)["leaf_kind"] == "compact_wy"
        with pytest.raises(RuntimeError):
            T.plan_query(1 << 16, n, leaf_kind="recursive")
    assert T.plan_query(1 << 16, 32, leaf_kind="recursive", want_q=False)["leaf_kind"] == "compact_wy"
    assert T.plan_query(1 << 16, 32, precision="mixed", leaf_kind="recursive")["leaf_kind"] == "compact_wy"
    from paper_0809_2407_amd import _lib
    lib = _lib.load()
    out = _lib.TsqrInfo()
    bad = _lib.TsqrOpts(0, 0, 0, 0, 0, 1, 3)
    assert lib.tsqr_plan_query(1000, 32, 0, ctypes.byref(bad), ctypes.byref(out)) == -4
    h = ctypes.c_void_p()
    rec = _lib.TsqrOpts(0, 0, 0, 0, 0, 1, 2)
    n = (ctypes.c_int64 * 1)(32)
    m = (ctypes.c_int64 * 1)(1000)
    assert lib.tsqr_batched_plan_create(ctypes.byref(h), 1, m, n, 0, ctypes.byref(rec), None) == -6
