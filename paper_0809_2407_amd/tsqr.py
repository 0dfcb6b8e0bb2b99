"""Python binding of libtsqr with the C ABI's names.  torch supplies device
memory and the current HIP stream; the binding only marshals pointers, leading
dimensions and options.

Matrices are column-major: an m x n matrix with leading dimension ld is a torch
tensor of shape (m, n) and strides (1, ld), e.g. ``colmajor(m, n)`` or
``T.t()`` for a contiguous (n, ld) tensor T.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import (PHASES, TSQR_FP64, TSQR_MIXED, TSQR_TREE_AUTO, TSQR_TREE_BINARY, TSQR_TREE_FLAT,
                   TSQR_TREE_HYBRID, TsqrInfo, TsqrOpts, TsqrTimings, check)

_LEAF_KINDS = {"auto": 0, "compact_wy": 1, "recursive": 2}
_LEAF_KIND_NAMES = {v: k for k, v in _LEAF_KINDS.items()}
_TREES = {"auto": TSQR_TREE_AUTO, "binary": TSQR_TREE_BINARY, "flat": TSQR_TREE_FLAT,
          "hybrid": TSQR_TREE_HYBRID}
_PREC = {"fp64": TSQR_FP64, "mixed": TSQR_MIXED}


def colmajor(m: int, n: int, device="cuda", ld: Optional[int] = None, dtype=torch.float64) -> torch.Tensor:
    """An uninitialised m x n column-major tensor with leading dimension ld."""
    ld = m if ld is None else ld
    return torch.empty((n, ld), dtype=dtype, device=device).t()[:m]


def to_colmajor(X: torch.Tensor, device="cuda") -> torch.Tensor:
    Y = colmajor(X.shape[0], X.shape[1], device=device, dtype=torch.float64)
    Y.copy_(X)
    return Y


def _ld(X: torch.Tensor, rows: int, name: str, dtype=torch.float64) -> int:
    if X.dim() != 2 or X.dtype != dtype:
        raise ValueError(f"{name}: a 2-D {dtype} tensor is required")
    if X.shape[0] != rows:
        raise ValueError(f"{name}: expected {rows} rows, got {X.shape[0]}")
    if X.stride(0) != 1 and X.shape[0] > 1:
        raise ValueError(f"{name}: must be column-major (stride (1, ld))")
    cols = X.shape[1]
    if cols > 1 and X.stride(1) < rows:
        # an expanded or overlapping view: the kernels would run past its storage
        raise ValueError(f"{name}: column stride {X.stride(1)} is below the row count {rows}")
    ld = X.stride(1) if cols > 1 else max(rows, 1)
    need = X.storage_offset() + (cols - 1) * ld + rows if cols > 0 and rows > 0 else 0
    if X.untyped_storage().nbytes() // X.element_size() < need:
        raise ValueError(f"{name}: its storage holds fewer than (n-1)*ld + m elements")
    if not X.is_cuda:
        raise ValueError(f"{name}: a device tensor is required")
    return ld


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _opts_or_null(tree, leaf_rows, tile_rows, flat_len, waves, want_q, leaf_kind="auto"):
    """Options for the C ABI; NULL when every field is at its default, so that
    the library may take the autotuned choice of the problem's class."""
    if tree == "auto" and not (leaf_rows or tile_rows or flat_len or waves) and want_q and leaf_kind == "auto":
        return None
    return ctypes.byref(TsqrOpts(_TREES[tree], int(leaf_rows), int(tile_rows), int(flat_len), int(waves),
                                 1 if want_q else 0, _LEAF_KINDS[leaf_kind]))


def plan_query(m: int, n: int, precision: str = "fp64", tree: str = "auto", leaf_rows: int = 0,
               tile_rows: int = 0, flat_len: int = 0, waves: int = 0, want_q: bool = True,
               leaf_kind: str = "auto") -> dict:
    """tsqr_plan_query: what a plan would choose (no device needed)."""
    lib = _lib.load()
    opts = _opts_or_null(tree, leaf_rows, tile_rows, flat_len, waves, want_q, leaf_kind)
    out = TsqrInfo()
    check("tsqr_plan_query", lib.tsqr_plan_query(int(m), int(n), _PREC[precision], opts, ctypes.byref(out)))
    d = {f: getattr(out, f) for f, _ in TsqrInfo._fields_}
    d["leaf_kind"] = _LEAF_KIND_NAMES[d["leaf_kind"]]
    return d


class Plan:
    """tsqr_plan_create / tsqr_factor / tsqr_form_q / tsqr_apply_qt /
    tsqr_plan_info / tsqr_plan_destroy."""

    def __init__(self, m: int, n: int, precision: str = "fp64", tree: str = "auto", leaf_rows: int = 0,
                 tile_rows: int = 0, flat_len: int = 0, waves: int = 0, want_q: bool = True, stream=None,
                 leaf_kind: str = "auto"):
        self._lib = _lib.load()
        self.m, self.n = int(m), int(n)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opts = _opts_or_null(tree, leaf_rows, tile_rows, flat_len, waves, want_q, leaf_kind)
        h = ctypes.c_void_p()
        check("tsqr_plan_create", self._lib.tsqr_plan_create(ctypes.byref(h), self.m, self.n, _PREC[precision],
                                                              opts, _stream_handle(self.stream)))
        self._h = h

    def close(self) -> None:
        # the library frees the plan even when it reports an error (say, a
        # fault of earlier work seen at the final synchronisation): forget the
        # handle first so that __del__ never destroys it a second time
        h = getattr(self, "_h", None)
        self._h = None
        if h is not None and h.value:
            check("tsqr_plan_destroy", self._lib.tsqr_plan_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def info(self) -> dict:
        out = TsqrInfo()
        check("tsqr_plan_info", self._lib.tsqr_plan_info(self._h, ctypes.byref(out)))
        d = {f: getattr(out, f) for f, _ in TsqrInfo._fields_}
        d["leaf_kind"] = _LEAF_KIND_NAMES[d["leaf_kind"]]
        return d

    def factor(self, A: torch.Tensor, R: Optional[torch.Tensor] = None) -> torch.Tensor:
        lda = _ld(A, self.m, "A")
        if R is None:
            R = colmajor(self.n, self.n, device=A.device)
        ldr = _ld(R, self.n, "R")
        check("tsqr_factor", self._lib.tsqr_factor(self._h, A.data_ptr(), lda, R.data_ptr(), ldr))
        return R

    def factor_into(self, A: torch.Tensor, V: Optional[torch.Tensor], R: Optional[torch.Tensor] = None) -> torch.Tensor:
        """tsqr_factor_into: A is only read; the reflectors go to V."""
        lda = _ld(A, self.m, "A")
        if R is None:
            R = colmajor(self.n, self.n, device=A.device)
        ldr = _ld(R, self.n, "R")
        vptr, ldv = (V.data_ptr(), _ld(V, self.m, "V")) if V is not None else (0, self.m)
        check("tsqr_factor_into", self._lib.tsqr_factor_into(self._h, A.data_ptr(), lda, vptr, ldv,
                                                             R.data_ptr(), ldr))
        return R

    def profile(self, enable: bool = True) -> None:
        check("tsqr_plan_profile", self._lib.tsqr_plan_profile(self._h, 1 if enable else 0))

    def timings(self) -> dict:
        """Summed device milliseconds and call counts per phase since profile()."""
        out = TsqrTimings()
        check("tsqr_plan_timings", self._lib.tsqr_plan_timings(self._h, ctypes.byref(out)))
        return {name: (out.ms[i], out.calls[i]) for i, name in enumerate(PHASES)}

    def form_q(self, A: Optional[torch.Tensor], Q: Optional[torch.Tensor] = None) -> torch.Tensor:
        """tsqr_form_q.  A is the factored matrix (FP64 plans); a MIXED plan keeps
        its reflectors itself and takes A = None."""
        aptr, lda = (A.data_ptr(), _ld(A, self.m, "A")) if A is not None else (0, self.m)
        if Q is None:
            Q = colmajor(self.m, self.n, device=A.device if A is not None else "cuda")
        ldq = _ld(Q, self.m, "Q")
        check("tsqr_form_q", self._lib.tsqr_form_q(self._h, aptr, lda, Q.data_ptr(), ldq))
        return Q

    def mixed_q1(self) -> torch.Tensor:
        """tsqr_mixed_q1: the FP32 first-pass Q1 of a MIXED plan (m x n, column-major)."""
        Q1 = colmajor(self.m, self.n, dtype=torch.float32)
        check("tsqr_mixed_q1", self._lib.tsqr_mixed_q1(self._h, Q1.data_ptr(), _ld(Q1, self.m, "Q1", torch.float32)))
        return Q1

    def apply_qt(self, A: Optional[torch.Tensor], B: torch.Tensor) -> torch.Tensor:
        """tsqr_apply_qt, B in place.  A is the factored matrix (FP64 plans); a
        MIXED plan takes A = None and writes Q^T B into the top n rows of B."""
        aptr, lda = (A.data_ptr(), _ld(A, self.m, "A")) if A is not None else (0, self.m)
        ldb = _ld(B, self.m, "B")
        check("tsqr_apply_qt", self._lib.tsqr_apply_qt(self._h, aptr, lda, B.shape[1], B.data_ptr(), ldb))
        return B


class BatchedPlan:
    """tsqr_batched_plan_create / tsqr_batched_factor / tsqr_batched_form_q /
    tsqr_batched_problem_info / tsqr_batched_plan_destroy for a list of
    problem sizes."""

    def __init__(self, ms, ns, precision: str = "fp64", tree: str = "auto", leaf_rows: int = 0,
                 flat_len: int = 0, waves: int = 0, want_q: bool = True, stream=None):
        self._lib = _lib.load()
        self.ms = [int(x) for x in ms]
        self.ns = [int(x) for x in ns]
        if len(self.ms) != len(self.ns):
            raise ValueError("ms and ns differ in length")
        self.count = len(self.ms)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opts = _opts_or_null(tree, leaf_rows, 0, flat_len, waves, want_q)
        I64 = ctypes.c_int64 * self.count
        h = ctypes.c_void_p()
        check("tsqr_batched_plan_create",
              self._lib.tsqr_batched_plan_create(ctypes.byref(h), self.count, I64(*self.ms), I64(*self.ns),
                                                 _PREC[precision], opts, _stream_handle(self.stream)))
        self._h = h

    def _arrays(self, mats, rows, name):
        if len(mats) != self.count:
            raise ValueError(f"{name}: {self.count} matrices expected")
        ptrs = (ctypes.c_void_p * self.count)(*[X.data_ptr() for X in mats])
        lds = (ctypes.c_int64 * self.count)(*[_ld(X, r, name) for X, r in zip(mats, rows)])
        return ptrs, lds

    def factor(self, As, Rs=None):
        """Factor every A (column-major, overwritten by the reflectors); returns the R's."""
        if Rs is None:
            Rs = [colmajor(n, n, device=A.device) for A, n in zip(As, self.ns)]
        ap, al = self._arrays(As, self.ms, "A")
        rp, rl = self._arrays(Rs, self.ns, "R")
        check("tsqr_batched_factor", self._lib.tsqr_batched_factor(self._h, ap, al, rp, rl))
        return Rs

    def form_q(self, As, Qs=None):
        if Qs is None:
            Qs = [colmajor(m, n, device=A.device) for A, m, n in zip(As, self.ms, self.ns)]
        ap, al = self._arrays(As, self.ms, "A")
        qp, ql = self._arrays(Qs, self.ms, "Q")
        check("tsqr_batched_form_q", self._lib.tsqr_batched_form_q(self._h, ap, al, qp, ql))
        return Qs

    def problem_info(self, i: int) -> dict:
        out = TsqrInfo()
        check("tsqr_batched_problem_info", self._lib.tsqr_batched_problem_info(self._h, int(i), ctypes.byref(out)))
        d = {f: getattr(out, f) for f, _ in TsqrInfo._fields_}
        d["leaf_kind"] = _LEAF_KIND_NAMES[d["leaf_kind"]]
        return d

    def close(self) -> None:
        # the library frees the plan even when it reports an error (say, a
        # fault of earlier work seen at the final synchronisation): forget the
        # handle first so that __del__ never destroys it a second time
        h = getattr(self, "_h", None)
        self._h = None
        if h is not None and h.value:
            check("tsqr_batched_plan_destroy", self._lib.tsqr_batched_plan_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_TREE_NAMES = {0: "auto", 1: "binary", 2: "flat", 3: "hybrid"}


def _opts_dict(o: TsqrOpts) -> dict:
    return {"tree": _TREE_NAMES[o.tree], "leaf_rows": o.leaf_rows, "tile_rows": o.tile_rows,
            "flat_len": o.flat_len, "waves": o.waves, "want_q": bool(o.want_q),
            "leaf_kind": _LEAF_KIND_NAMES[o.leaf_kind]}


def autotune(m: int, n: int, precision: str = "fp64", want_q: bool = True, A: Optional[torch.Tensor] = None,
             cache: Optional[str] = None, reps: int = 3, stream=None) -> dict:
    """tsqr_autotune: the fastest geometry for the class of (m, n); A (if given)
    is a representative column-major device matrix, only read.  The returned
    'opts' are Plan keyword arguments."""
    lib = _lib.load()
    stream = stream if stream is not None else torch.cuda.current_stream()
    aptr, lda = (A.data_ptr(), _ld(A, m, "A")) if A is not None else (None, int(m))
    out = _lib.TsqrTuneResult()
    check("tsqr_autotune", lib.tsqr_autotune(int(m), int(n), _PREC[precision], 1 if want_q else 0, aptr, lda,
                                             _stream_handle(stream), cache.encode() if cache else None, int(reps),
                                             ctypes.byref(out)))
    return {"opts": _opts_dict(out.opts), "ms": out.ms, "candidates": out.candidates,
            "from_cache": bool(out.from_cache)}


def tune_cache_lookup(path: str, m: int, n: int, precision: str = "fp64", want_q: bool = True) -> Optional[dict]:
    """tsqr_tune_cache_lookup: the cached options of a class, or None."""
    lib = _lib.load()
    o = TsqrOpts()
    ms = ctypes.c_double()
    st = lib.tsqr_tune_cache_lookup(path.encode(), int(m), int(n), _PREC[precision], 1 if want_q else 0,
                                    ctypes.byref(o), ctypes.byref(ms))
    if st == 5:
        return None
    check("tsqr_tune_cache_lookup", st)
    return {"opts": _opts_dict(o), "ms": ms.value}


def tune_cache_store(path: str, m: int, n: int, opts: dict, ms: float, precision: str = "fp64") -> None:
    """tsqr_tune_cache_store."""
    lib = _lib.load()
    o = TsqrOpts(_TREES[opts.get("tree", "auto")], int(opts.get("leaf_rows", 0)), int(opts.get("tile_rows", 0)),
                 int(opts.get("flat_len", 0)), int(opts.get("waves", 0)), 1 if opts.get("want_q", True) else 0,
                 _LEAF_KINDS[opts.get("leaf_kind", "auto")])
    check("tsqr_tune_cache_store", lib.tsqr_tune_cache_store(path.encode(), int(m), int(n), _PREC[precision],
                                                             ctypes.byref(o), float(ms)))


class StreamPlan:
    """tsqr_stream_plan_create / tsqr_stream_factor / tsqr_stream_plan_info /
    tsqr_stream_plan_destroy: the R of an m x n matrix held in host memory,
    streamed through the GPU in blocks (the out-of-DRAM flat tree of Sec. 7.1)."""

    def __init__(self, m: int, n: int, block_rows: int = 0, stream=None):
        self._lib = _lib.load()
        self.m, self.n = int(m), int(n)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check("tsqr_stream_plan_create", self._lib.tsqr_stream_plan_create(ctypes.byref(h), self.m, self.n,
                                                                           int(block_rows),
                                                                           _stream_handle(self.stream)))
        self._h = h

    def info(self) -> dict:
        b, k = ctypes.c_int64(0), ctypes.c_int64(0)
        check("tsqr_stream_plan_info", self._lib.tsqr_stream_plan_info(self._h, ctypes.byref(b), ctypes.byref(k)))
        return {"block_rows": int(b.value), "num_blocks": int(k.value)}

    def factor(self, A: torch.Tensor, R: Optional[torch.Tensor] = None) -> torch.Tensor:
        """R (on the device) of A, a column-major float64 tensor in host memory."""
        if A.is_cuda or A.dim() != 2 or A.dtype != torch.float64 or A.shape[0] != self.m or A.shape[1] != self.n:
            raise ValueError("A: an m x n float64 host tensor is required")
        if A.stride(0) != 1 and self.m > 1:
            raise ValueError("A: must be column-major (stride (1, ld))")
        lda = A.stride(1) if self.n > 1 else self.m
        if self.n > 1 and lda < self.m:
            raise ValueError("A: column stride below the row count")
        if R is None:
            R = colmajor(self.n, self.n)
        ldr = _ld(R, self.n, "R")
        check("tsqr_stream_factor", self._lib.tsqr_stream_factor(self._h, A.data_ptr(), lda, R.data_ptr(), ldr))
        return R

    def close(self) -> None:
        h = getattr(self, "_h", None)
        self._h = None
        if h is not None and h.value:
            check("tsqr_stream_plan_destroy", self._lib.tsqr_stream_plan_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class CaqrPlan:
    """tsqr_caqr_plan_create / tsqr_caqr_factor / tsqr_caqr_factor_rhs / tsqr_caqr_apply_qt /
    tsqr_caqr_plan_info / tsqr_caqr_plan_destroy: CAQR of an m x n matrix
    (Sec. 6) with TSQR panels of `panel` columns."""

    def __init__(self, m: int, n: int, panel: int = 0, stream=None):
        self._lib = _lib.load()
        self.m, self.n = int(m), int(n)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check("tsqr_caqr_plan_create", self._lib.tsqr_caqr_plan_create(ctypes.byref(h), self.m, self.n, int(panel),
                                                                       _stream_handle(self.stream)))
        self._h = h

    def info(self) -> dict:
        b, k = ctypes.c_int64(0), ctypes.c_int64(0)
        check("tsqr_caqr_plan_info", self._lib.tsqr_caqr_plan_info(self._h, ctypes.byref(b), ctypes.byref(k)))
        return {"panel": int(b.value), "num_panels": int(k.value)}

    def factor(self, A: torch.Tensor, R: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Factor A in place (reflectors and R's row blocks); returns R."""
        lda = _ld(A, self.m, "A")
        if R is None:
            R = colmajor(self.n, self.n, device=A.device)
        ldr = _ld(R, self.n, "R")
        check("tsqr_caqr_factor", self._lib.tsqr_caqr_factor(self._h, A.data_ptr(), lda, R.data_ptr(), ldr))
        return R

    def factor_rhs(self, AB: torch.Tensor, R: Optional[torch.Tensor] = None) -> torch.Tensor:
        """tsqr_caqr_factor_rhs on AB = [A B] (m x (n + k), column-major): A is
        factored in place and B becomes Q^T B; returns R."""
        if AB.dim() != 2 or AB.shape[1] < self.n:
            raise ValueError(f"AB: expected at least {self.n} columns")
        k = AB.shape[1] - self.n
        lda = _ld(AB, self.m, "AB")
        if R is None:
            R = colmajor(self.n, self.n, device=AB.device)
        ldr = _ld(R, self.n, "R")
        check("tsqr_caqr_factor_rhs", self._lib.tsqr_caqr_factor_rhs(self._h, AB.data_ptr(), lda, R.data_ptr(), ldr,
                                                                     k))
        return R

    def apply_qt(self, A: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
        lda = _ld(A, self.m, "A")
        ldb = _ld(B, self.m, "B")
        check("tsqr_caqr_apply_qt", self._lib.tsqr_caqr_apply_qt(self._h, A.data_ptr(), lda, B.shape[1],
                                                                 B.data_ptr(), ldb))
        return B

    def close(self) -> None:
        h = getattr(self, "_h", None)
        self._h = None
        if h is not None and h.value:
            check("tsqr_caqr_plan_destroy", self._lib.tsqr_caqr_plan_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


_CMP = {"cholqr": 0, "cholqr2": 1, "cgs": 2, "mgs": 3}


class CmpPlan:
    """tsqr_cmp_plan_create / tsqr_cmp_factor / tsqr_cmp_breakdown /
    tsqr_cmp_plan_destroy: one of TSQR's competitors of Sec. 5 (method
    "cholqr", "cholqr2", "cgs" or "mgs") for m x n problems."""

    def __init__(self, m: int, n: int, method: str, stream=None):
        self._lib = _lib.load()
        self.m, self.n, self.method = int(m), int(n), method
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        check("tsqr_cmp_plan_create", self._lib.tsqr_cmp_plan_create(ctypes.byref(h), self.m, self.n, _CMP[method],
                                                                     _stream_handle(self.stream)))
        self._h = h

    def factor(self, A: torch.Tensor, Q: Optional[torch.Tensor] = None, R: Optional[torch.Tensor] = None):
        """Q (may be A itself) and R of A; returns (Q, R)."""
        lda = _ld(A, self.m, "A")
        if Q is None:
            Q = colmajor(self.m, self.n, device=A.device)
        if R is None:
            R = colmajor(self.n, self.n, device=A.device)
        ldq, ldr = _ld(Q, self.m, "Q"), _ld(R, self.n, "R")
        check("tsqr_cmp_factor", self._lib.tsqr_cmp_factor(self._h, A.data_ptr(), lda, Q.data_ptr(), ldq,
                                                           R.data_ptr(), ldr))
        return Q, R

    def breakdown(self) -> int:
        """0, or j + 1 for the first column j where the method broke down."""
        c = ctypes.c_int(0)
        check("tsqr_cmp_breakdown", self._lib.tsqr_cmp_breakdown(self._h, ctypes.byref(c)))
        return int(c.value)

    def close(self) -> None:
        h = getattr(self, "_h", None)
        self._h = None
        if h is not None and h.value:
            check("tsqr_cmp_plan_destroy", self._lib.tsqr_cmp_plan_destroy(h))

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def factor_r_noalloc(A: torch.Tensor, R: Optional[torch.Tensor] = None, stream=None):
    """tsqr_factor_r_noalloc: the FP64 R of A (only read) with no device
    allocation by the library (its workspace is a fixed per-GPU array).
    Returns (R, geometry dict)."""
    lib = _lib.load()
    m, n = A.shape
    lda = _ld(A, m, "A")
    if R is None:
        R = colmajor(n, n, device=A.device)
    ldr = _ld(R, n, "R")
    out = TsqrInfo()
    h = _stream_handle(stream)
    check("tsqr_factor_r_noalloc", lib.tsqr_factor_r_noalloc(m, n, A.data_ptr(), lda, R.data_ptr(), ldr, h,
                                                             ctypes.byref(out)))
    return R, {f: getattr(out, f) for f, _ in TsqrInfo._fields_}


def qr(A: torch.Tensor, **plan_kw):
    """Thin QR of a column-major device matrix: returns (Q, R); A is overwritten
    by the reflectors."""
    m, n = A.shape
    with Plan(m, n, **plan_kw) as p:
        R = p.factor(A)
        Q = p.form_q(A)
        torch.cuda.current_stream().synchronize()
    return Q, R
