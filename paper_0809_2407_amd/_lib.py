"""ctypes declarations of libtsqr's C ABI (include/tsqr.h).  Argument
marshalling only: every step of the computation runs in the library's HIP
kernels.  Loading fails loudly when the library has not been built."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TSQR_LIBRARY names another build of the same library (the host-sanitized
# libtsqr_checked.so of the sanitizer tests)
LIB_PATH = os.environ.get("TSQR_LIBRARY") or os.path.join(HERE, "libtsqr.so")

TSQR_FP64, TSQR_MIXED = 0, 1
TSQR_CMP_CHOLQR, TSQR_CMP_CHOLQR2, TSQR_CMP_CGS, TSQR_CMP_MGS = 0, 1, 2, 3
TSQR_TREE_AUTO, TSQR_TREE_BINARY, TSQR_TREE_FLAT, TSQR_TREE_HYBRID = 0, 1, 2, 3

i64 = ctypes.c_int64
dp = ctypes.c_void_p  # device pointers travel as plain addresses


class TsqrOpts(ctypes.Structure):
    _fields_ = [("tree", ctypes.c_int), ("leaf_rows", i64), ("tile_rows", i64),
                ("flat_len", ctypes.c_int), ("waves", ctypes.c_int), ("want_q", ctypes.c_int),
                ("leaf_kind", ctypes.c_int)]


class TsqrInfo(ctypes.Structure):
    _fields_ = [("m", i64), ("n", i64), ("n_padded", i64), ("tile_rows", i64), ("leaf_rows", i64),
                ("num_leaves", i64), ("num_tiles", i64), ("tree_levels", ctypes.c_int),
                ("tree", ctypes.c_int), ("waves", ctypes.c_int), ("precision", ctypes.c_int),
                ("workspace_bytes", i64), ("reorth_applied", ctypes.c_int),
                ("orth_estimate", ctypes.c_double), ("leaf_kind", ctypes.c_int)]


PHASES = ["leaf", "tree", "root", "seeds", "form_q", "apply_qt", "q1", "reorth", "leaf_t"]


class TsqrTimings(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(PHASES)), ("calls", i64 * len(PHASES))]


class TsqrTuneResult(ctypes.Structure):
    _fields_ = [("opts", TsqrOpts), ("ms", ctypes.c_double), ("candidates", ctypes.c_int),
                ("from_cache", ctypes.c_int)]



EXPORTED = [
    "tsqr_plan_create", "tsqr_plan_query", "tsqr_factor", "tsqr_factor_into", "tsqr_form_q", "tsqr_apply_qt",
    "tsqr_plan_info", "tsqr_plan_profile", "tsqr_plan_timings", "tsqr_plan_destroy", "tsqr_status_string",
    "tsqr_version", "tsqr_mixed_q1",
    "tsqr_batched_plan_create", "tsqr_batched_factor", "tsqr_batched_form_q", "tsqr_batched_problem_info",
    "tsqr_batched_plan_destroy", "tsqr_autotune", "tsqr_tune_cache_lookup", "tsqr_tune_cache_store",
    "tsqr_factor_r_noalloc",
    "tsqr_cmp_plan_create", "tsqr_cmp_factor", "tsqr_cmp_breakdown", "tsqr_cmp_plan_destroy",
    "tsqr_stream_plan_create", "tsqr_stream_factor", "tsqr_stream_plan_info", "tsqr_stream_plan_destroy",
    "tsqr_caqr_plan_create", "tsqr_caqr_factor", "tsqr_caqr_factor_rhs", "tsqr_caqr_apply_qt", "tsqr_caqr_plan_info",
    "tsqr_caqr_plan_destroy",
]

_lib = None


class TsqrError(RuntimeError):
    def __init__(self, fn: str, status: int):
        self.status = status
        text = load().tsqr_status_string(status).decode()
        super().__init__(f"{fn} failed with status {status}: {text}")


def load(path: str = LIB_PATH):
    """Load libtsqr.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libtsqr.so not found at {path}; build it with "
                           f"`python -m paper_0809_2407_amd.build`")
    # torch carries its own HIP runtime: loading it first makes the library bind
    # to that one (same soname) instead of bringing a second runtime into the process
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.tsqr_plan_create.argtypes = [ctypes.POINTER(P), i64, i64, ctypes.c_int, ctypes.POINTER(TsqrOpts), P]
    lib.tsqr_plan_create.restype = ctypes.c_int
    lib.tsqr_plan_query.argtypes = [i64, i64, ctypes.c_int, ctypes.POINTER(TsqrOpts), ctypes.POINTER(TsqrInfo)]
    lib.tsqr_plan_query.restype = ctypes.c_int
    lib.tsqr_factor.argtypes = [P, dp, i64, dp, i64]
    lib.tsqr_factor.restype = ctypes.c_int
    lib.tsqr_factor_into.argtypes = [P, dp, i64, dp, i64, dp, i64]
    lib.tsqr_factor_into.restype = ctypes.c_int
    lib.tsqr_plan_profile.argtypes = [P, ctypes.c_int]
    lib.tsqr_plan_profile.restype = ctypes.c_int
    lib.tsqr_plan_timings.argtypes = [P, ctypes.POINTER(TsqrTimings)]
    lib.tsqr_plan_timings.restype = ctypes.c_int
    lib.tsqr_form_q.argtypes = [P, dp, i64, dp, i64]
    lib.tsqr_form_q.restype = ctypes.c_int
    lib.tsqr_apply_qt.argtypes = [P, dp, i64, i64, dp, i64]
    lib.tsqr_apply_qt.restype = ctypes.c_int
    lib.tsqr_plan_info.argtypes = [P, ctypes.POINTER(TsqrInfo)]
    lib.tsqr_plan_info.restype = ctypes.c_int
    lib.tsqr_plan_destroy.argtypes = [P]
    lib.tsqr_plan_destroy.restype = ctypes.c_int
    lib.tsqr_status_string.argtypes = [ctypes.c_int]
    lib.tsqr_status_string.restype = ctypes.c_char_p
    lib.tsqr_version.argtypes = []
    lib.tsqr_version.restype = ctypes.c_int
    lib.tsqr_mixed_q1.argtypes = [P, ctypes.c_void_p, i64]
    lib.tsqr_mixed_q1.restype = ctypes.c_int
    i64p = ctypes.POINTER(ctypes.c_int64)
    vpp = ctypes.POINTER(ctypes.c_void_p)
    lib.tsqr_batched_plan_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, i64p, i64p, ctypes.c_int,
                                             ctypes.POINTER(TsqrOpts), P]
    lib.tsqr_batched_plan_create.restype = ctypes.c_int
    lib.tsqr_batched_factor.argtypes = [P, vpp, i64p, vpp, i64p]
    lib.tsqr_batched_factor.restype = ctypes.c_int
    lib.tsqr_batched_form_q.argtypes = [P, vpp, i64p, vpp, i64p]
    lib.tsqr_batched_form_q.restype = ctypes.c_int
    lib.tsqr_batched_problem_info.argtypes = [P, ctypes.c_int, ctypes.POINTER(TsqrInfo)]
    lib.tsqr_batched_problem_info.restype = ctypes.c_int
    lib.tsqr_batched_plan_destroy.argtypes = [P]
    lib.tsqr_batched_plan_destroy.restype = ctypes.c_int
    lib.tsqr_autotune.argtypes = [i64, i64, ctypes.c_int, ctypes.c_int, dp, i64, P, ctypes.c_char_p, ctypes.c_int,
                                  ctypes.POINTER(TsqrTuneResult)]
    lib.tsqr_autotune.restype = ctypes.c_int
    lib.tsqr_tune_cache_lookup.argtypes = [ctypes.c_char_p, i64, i64, ctypes.c_int, ctypes.c_int,
                                           ctypes.POINTER(TsqrOpts), ctypes.POINTER(ctypes.c_double)]
    lib.tsqr_tune_cache_lookup.restype = ctypes.c_int
    lib.tsqr_tune_cache_store.argtypes = [ctypes.c_char_p, i64, i64, ctypes.c_int, ctypes.POINTER(TsqrOpts),
                                          ctypes.c_double]
    lib.tsqr_tune_cache_store.restype = ctypes.c_int
    lib.tsqr_cmp_plan_create.argtypes = [ctypes.POINTER(P), i64, i64, ctypes.c_int, P]
    lib.tsqr_cmp_plan_create.restype = ctypes.c_int
    lib.tsqr_cmp_factor.argtypes = [P, dp, i64, dp, i64, dp, i64]
    lib.tsqr_cmp_factor.restype = ctypes.c_int
    lib.tsqr_cmp_breakdown.argtypes = [P, ctypes.POINTER(ctypes.c_int)]
    lib.tsqr_cmp_breakdown.restype = ctypes.c_int
    lib.tsqr_cmp_plan_destroy.argtypes = [P]
    lib.tsqr_cmp_plan_destroy.restype = ctypes.c_int
    lib.tsqr_stream_plan_create.argtypes = [ctypes.POINTER(P), i64, i64, i64, P]
    lib.tsqr_stream_plan_create.restype = ctypes.c_int
    lib.tsqr_stream_factor.argtypes = [P, dp, i64, dp, i64]
    lib.tsqr_stream_factor.restype = ctypes.c_int
    lib.tsqr_stream_plan_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.tsqr_stream_plan_info.restype = ctypes.c_int
    lib.tsqr_stream_plan_destroy.argtypes = [P]
    lib.tsqr_stream_plan_destroy.restype = ctypes.c_int
    lib.tsqr_caqr_plan_create.argtypes = [ctypes.POINTER(P), i64, i64, i64, P]
    lib.tsqr_caqr_plan_create.restype = ctypes.c_int
    lib.tsqr_caqr_factor.argtypes = [P, dp, i64, dp, i64]
    lib.tsqr_caqr_factor.restype = ctypes.c_int
    lib.tsqr_caqr_factor_rhs.argtypes = [P, dp, i64, dp, i64, i64]
    lib.tsqr_caqr_factor_rhs.restype = ctypes.c_int
    lib.tsqr_caqr_apply_qt.argtypes = [P, dp, i64, i64, dp, i64]
    lib.tsqr_caqr_apply_qt.restype = ctypes.c_int
    lib.tsqr_caqr_plan_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.tsqr_caqr_plan_info.restype = ctypes.c_int
    lib.tsqr_caqr_plan_destroy.argtypes = [P]
    lib.tsqr_caqr_plan_destroy.restype = ctypes.c_int
    lib.tsqr_factor_r_noalloc.argtypes = [i64, i64, dp, i64, dp, i64, P, ctypes.POINTER(TsqrInfo)]
    lib.tsqr_factor_r_noalloc.restype = ctypes.c_int
    _lib = lib
    return lib


def check(fn: str, status: int) -> None:
    if status != 0:
        raise TsqrError(fn, status)
