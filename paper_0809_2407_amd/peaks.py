"""ctypes binding of libtsqr_peaks (include/tsqr_peaks.h): the streaming copy
and read and the FP64 FMA and MFMA loops that measure the part's own ceilings.
Argument marshalling only; loading fails loudly when the library has not been
built."""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsqr_peaks.so")

EXPORTED = ["tsqr_peak_copy", "tsqr_peak_read", "tsqr_peak_copy_leaf", "tsqr_peak_fma", "tsqr_peak_mfma",
            "tsqr_peak_grid"]

_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -m paper_0809_2407_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    i64, dp, d = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
    c_int = ctypes.c_int
    lib.tsqr_peak_copy.argtypes = [dp, dp, i64, c_int, dp]
    lib.tsqr_peak_read.argtypes = [dp, i64, dp, c_int, dp]
    lib.tsqr_peak_copy_leaf.argtypes = [dp, i64, dp, i64, i64, c_int, i64, c_int, dp]
    lib.tsqr_peak_fma.argtypes = [dp, c_int, c_int, d, d, dp]
    lib.tsqr_peak_mfma.argtypes = [dp, c_int, c_int, d, d, dp]
    lib.tsqr_peak_grid.argtypes = [c_int, i64]
    for f in EXPORTED:
        getattr(lib, f).restype = c_int
    _lib = lib
    return lib


def _stream(stream) -> int:
    return int((stream if stream is not None else torch.cuda.current_stream()).cuda_stream)


def _check(name: str, rc: int) -> None:
    if rc != 0:
        raise RuntimeError(f"{name} returned {rc}")


def _need(cond: bool, what: str) -> None:
    if not cond:
        raise ValueError(what)


def default_grid(kind: int, nbytes: int = 0) -> int:
    """tsqr_peak_grid: the default grid of a copy (0) or a read (1) of nbytes
    bytes, or of the loops (2)."""
    g = load().tsqr_peak_grid(kind, nbytes)
    if g <= 0:
        raise RuntimeError(f"tsqr_peak_grid({kind}) returned {g}")
    return g


def copy(src: torch.Tensor, dst: torch.Tensor, grid: int = 0, stream=None) -> None:
    """tsqr_peak_copy over the bytes of two contiguous device tensors of equal size."""
    _need(src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous(),
          "copy: contiguous device tensors")
    nb = src.numel() * src.element_size()
    _need(dst.numel() * dst.element_size() == nb, "copy: tensors of equal size")
    _check("tsqr_peak_copy", load().tsqr_peak_copy(src.data_ptr(), dst.data_ptr(), nb, grid, _stream(stream)))


def read(src: torch.Tensor, partial: torch.Tensor, grid: int = 0, stream=None) -> None:
    """tsqr_peak_read: per-workgroup sums of src into partial (FP64, >= grid entries)."""
    _need(src.is_cuda and src.is_contiguous() and partial.is_cuda and partial.dtype == torch.float64,
          "read: a contiguous device tensor and an FP64 device tensor")
    nb = src.numel() * src.element_size()
    g = grid if grid > 0 else default_grid(1, nb)
    _need(partial.is_contiguous() and partial.numel() >= g, f"read: partial needs {g} doubles")
    _check("tsqr_peak_read", load().tsqr_peak_read(src.data_ptr(), nb, partial.data_ptr(), grid, _stream(stream)))


def copy_leaf(src: torch.Tensor, dst: torch.Tensor, leaf_rows: int, tile_rows: int, stream=None) -> None:
    """tsqr_peak_copy_leaf between two column-major FP64 device matrices of one shape."""
    _need(src.is_cuda and dst.is_cuda and src.dtype == torch.float64 and dst.dtype == torch.float64
          and src.dim() == 2 and src.shape == dst.shape, "copy_leaf: two FP64 device matrices of one shape")
    m, n = src.shape
    for X in (src, dst):
        _need(X.stride(0) == 1 and (n == 1 or X.stride(1) >= m), "copy_leaf: column-major matrices")
    lds = src.stride(1) if n > 1 else m
    ldd = dst.stride(1) if n > 1 else m
    _check("tsqr_peak_copy_leaf", load().tsqr_peak_copy_leaf(src.data_ptr(), lds, dst.data_ptr(), ldd, m, n,
                                                             leaf_rows, tile_rows, _stream(stream)))


def fma(out: torch.Tensor, iters: int, c: float = 1.0, d: float = 1.0, grid: int = 0, stream=None) -> None:
    """tsqr_peak_fma; out holds grid * 256 doubles."""
    g = grid if grid > 0 else default_grid(2)
    _need(out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= g * 256,
          f"fma: out needs {g * 256} contiguous device doubles")
    _check("tsqr_peak_fma", load().tsqr_peak_fma(out.data_ptr(), grid, iters, c, d, _stream(stream)))


def mfma(out: torch.Tensor, iters: int, a: float = 0.5, b: float = 0.5, grid: int = 0, stream=None) -> None:
    """tsqr_peak_mfma; out holds grid * 256 doubles."""
    g = grid if grid > 0 else default_grid(2)
    _need(out.is_cuda and out.dtype == torch.float64 and out.is_contiguous() and out.numel() >= g * 256,
          f"mfma: out needs {g * 256} contiguous device doubles")
    _check("tsqr_peak_mfma", load().tsqr_peak_mfma(out.data_ptr(), grid, iters, a, b, _stream(stream)))
