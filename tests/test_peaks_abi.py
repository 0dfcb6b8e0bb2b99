"""The ceiling-measurement library (streaming copy and read, FP64 FMA and MFMA
loops) without a GPU: it loads, exports every function include/tsqr_peaks.h
declares, and rejects bad arguments before touching a device."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "tsqr_peaks.h")).read()
    return sorted(set(re.findall(r"\b(tsqr_peak_[a-z0-9_]+)\s*\(", text)))


def test_header_binding_and_library_agree():
    from paper_0809_2407_amd import peaks
    assert _declared_functions() == sorted(peaks.EXPORTED)
    lib = peaks.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_argument_errors_without_device():
    from paper_0809_2407_amd import peaks
    lib = peaks.load()
    assert lib.tsqr_peak_copy(None, 4096, 16, 0, None) == -1
    assert lib.tsqr_peak_copy(4104, 4096, 16, 0, None) == -1      # src not 16-byte aligned
    assert lib.tsqr_peak_copy(4096, None, 16, 0, None) == -2
    assert lib.tsqr_peak_copy(4096, 8192 + 8, 16, 0, None) == -2  # dst not aligned
    assert lib.tsqr_peak_copy(4096, 4096 + 16, 32, 0, None) == -2  # overlapping
    assert lib.tsqr_peak_copy(4096, 8192, 24, 0, None) == -3       # not a multiple of 16
    assert lib.tsqr_peak_copy(4096, 8192, 0, 0, None) == -3
    assert lib.tsqr_peak_copy(4096, 8192, 16, (1 << 20) + 1, None) == -4
    assert lib.tsqr_peak_read(None, 16, 8192, 0, None) == -1
    assert lib.tsqr_peak_read(4096, 8, 8192, 0, None) == -2
    assert lib.tsqr_peak_read(4096, 16, None, 0, None) == -3
    assert lib.tsqr_peak_read(4096, 16, 8192, (1 << 20) + 1, None) == -4
    assert lib.tsqr_peak_fma(None, 1, 1, 1.0, 1.0, None) == -1
    assert lib.tsqr_peak_fma(4096, (1 << 20) + 1, 1, 1.0, 1.0, None) == -2
    assert lib.tsqr_peak_fma(4096, 1, -1, 1.0, 1.0, None) == -3
    assert lib.tsqr_peak_mfma(None, 1, 1, 0.5, 0.5, None) == -1
    assert lib.tsqr_peak_mfma(4096, (1 << 20) + 1, 1, 0.5, 0.5, None) == -2
    assert lib.tsqr_peak_mfma(4096, 1, -1, 0.5, 0.5, None) == -3
    # copy_leaf(src, lds, dst, ldd, m, n, leaf_rows, tile_rows, stream)
    big = 1 << 40
    assert lib.tsqr_peak_copy_leaf(None, 100, big, 100, 100, 8, 64, 16, None) == -1
    assert lib.tsqr_peak_copy_leaf(4096, 99, big, 100, 100, 8, 64, 16, None) == -2
    assert lib.tsqr_peak_copy_leaf(4096, 100, None, 100, 100, 8, 64, 16, None) == -3
    assert lib.tsqr_peak_copy_leaf(4096, 100, 4096 + 800, 100, 100, 8, 64, 16, None) == -3  # overlapping
    assert lib.tsqr_peak_copy_leaf(4096, 100, big, 99, 100, 8, 64, 16, None) == -4
    assert lib.tsqr_peak_copy_leaf(4096, 100, big, 100, 0, 8, 64, 16, None) == -5
    assert lib.tsqr_peak_copy_leaf(4096, 100, big, 100, 100, 65, 64, 16, None) == -6
    assert lib.tsqr_peak_copy_leaf(4096, 100, big, 100, 100, 0, 64, 16, None) == -6
    assert lib.tsqr_peak_copy_leaf(4096, 100, big, 100, 100, 8, 40, 16, None) == -7  # not a multiple of tile
    assert lib.tsqr_peak_copy_leaf(4096, 100, big, 100, 100, 8, 64, 24, None) == -8
    assert lib.tsqr_peak_grid(3, 0) == -1
    assert lib.tsqr_peak_grid(0, -16) == -1
