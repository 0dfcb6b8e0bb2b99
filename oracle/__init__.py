"""FP64 CPU oracle for TSQR -- test infrastructure only.

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it and shares
no code with it.  The arithmetic lives in ``tsqr_oracle.c`` (plain loops, no
BLAS); this module only builds it and marshals numpy arrays through ctypes.

Functions follow the paper (Demmel, Grigori, Hoemmen, Langou, arXiv 0809.2407):
  * ``householder_qr`` / ``apply_q`` / ``apply_qt``: the local Householder QR of
    one block and the application of its Q or Q^T (Sec. 4.2, Alg. 1 step 1).
  * ``qr_reference``: the sign-normalised thin QR of the whole matrix by one
    plain Householder QR -- the unique result TSQR must reproduce (Sec. 2).
  * ``TSQR``: the hybrid tree of Alg. 2 (flat chain inside a leaf) under Alg. 1
    (binary tree over leaves), with explicit Q and Q^T B (Sec. 2, Sec. 4.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsqr_oracle.c")
# the comparison methods of Sec. 5 (CholeskyQR, CGS, MGS) live beside it
_SRCS = [_SRC, os.path.join(_HERE, "cmp_oracle.c")]
_LIB = os.path.join(_HERE, "libtsqr_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(f) for f in _SRCS):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
               *_SRCS, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    i64, dp, vp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p
    lib.orc_householder_qr.argtypes = [i64, i64, dp, i64, dp]
    lib.orc_apply_q.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
    lib.orc_apply_qt.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
    lib.orc_qr_reference.argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
    lib.orc_qr_reference.restype = ctypes.c_int
    lib.orc_tsqr_factor.argtypes = [i64, i64, dp, i64, i64, i64]
    lib.orc_tsqr_factor.restype = vp
    lib.orc_tsqr_free.argtypes = [vp]
    lib.orc_tsqr_R.argtypes = [vp, dp, i64]
    lib.orc_tsqr_signs.argtypes = [vp, dp]
    lib.orc_tsqr_form_q.argtypes = [vp, dp, i64]
    lib.orc_tsqr_apply_qt.argtypes = [vp, i64, dp, i64]
    lib.orc_tsqr_node.argtypes = [vp, ctypes.c_int, i64, ctypes.POINTER(dp), ctypes.POINTER(dp)]
    lib.orc_tsqr_node.restype = i64
    lib.orc_tsqr_leaf_stage.argtypes = [vp, i64, i64, ctypes.POINTER(dp), ctypes.POINTER(dp)]
    lib.orc_tsqr_leaf_stage.restype = i64
    lib.orc_tsqr_node_homes.argtypes = [vp, ctypes.c_int, i64, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.orc_tsqr_node_homes.restype = ctypes.c_int
    lib.orc_tsqr_num_leaves.argtypes = [vp]
    lib.orc_tsqr_num_leaves.restype = i64
    lib.orc_tsqr_num_levels.argtypes = [vp]
    lib.orc_tsqr_num_levels.restype = ctypes.c_int
    lib.orc_num_leaves.argtypes = [i64, i64]
    lib.orc_num_leaves.restype = i64
    lib.orc_tree_levels.argtypes = [i64, ctypes.POINTER(i64), ctypes.c_int]
    lib.orc_tree_levels.restype = ctypes.c_int
    lib.orc_set_mutation.argtypes = [ctypes.c_int]
    for f in ("orc_cholqr", "orc_cholqr2", "orc_cgs", "orc_mgs"):
        getattr(lib, f).argtypes = [i64, i64, dp, i64, dp, i64, dp, i64]
        getattr(lib, f).restype = ctypes.c_int
    lib.orc_num_threads.restype = ctypes.c_int
    lib.orc_set_num_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _f64(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    return np.asfortranarray(a)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ld(a: np.ndarray) -> int:
    return max(1, a.strides[1] // 8) if a.ndim == 2 else max(1, a.shape[0])


def set_mutation(code: int) -> None:
    """Test-only: plant a known mistake in the oracle (0 restores it)."""
    _load().orc_set_mutation(int(code))


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(t: int) -> None:
    _load().orc_set_num_threads(int(t))


def householder_qr(A: np.ndarray):
    """Plain Householder QR of one block; returns (VR, tau) in LAPACK layout."""
    W = _f64(A).copy(order="F")
    m, n = W.shape
    tau = np.zeros(min(m, n), dtype=np.float64)
    if tau.size == 0:
        tau = np.zeros(1)
    _load().orc_householder_qr(m, n, _p(W), _ld(W), _p(tau))
    return W, tau[: min(m, n)]


def apply_q(VR: np.ndarray, tau: np.ndarray, X: np.ndarray) -> np.ndarray:
    VR = _f64(VR); tau = np.ascontiguousarray(tau, dtype=np.float64)
    X = _f64(X).copy(order="F")
    m, n = VR.shape
    k = X.shape[1]
    _load().orc_apply_q(m, n, _p(VR), _ld(VR), _p(tau), k, _p(X), _ld(X))
    return X


def apply_qt(VR: np.ndarray, tau: np.ndarray, X: np.ndarray) -> np.ndarray:
    VR = _f64(VR); tau = np.ascontiguousarray(tau, dtype=np.float64)
    X = _f64(X).copy(order="F")
    m, n = VR.shape
    k = X.shape[1]
    _load().orc_apply_qt(m, n, _p(VR), _ld(VR), _p(tau), k, _p(X), _ld(X))
    return X


def qr_reference(A: np.ndarray, want_q: bool = True):
    """Sign-normalised thin QR of A by one plain Householder QR."""
    A = _f64(A)
    m, n = A.shape
    R = np.zeros((n, n), dtype=np.float64, order="F")
    Q = np.zeros((m, n), dtype=np.float64, order="F") if want_q else None
    rc = _load().orc_qr_reference(m, n, _p(A), _ld(A), _p(R), n,
                                  _p(Q) if want_q else None, m if want_q else 1)
    if rc != 0:
        raise ValueError("qr_reference: bad arguments (need m >= n >= 1)")
    return (R, Q) if want_q else R


def num_leaves(m: int, leaf_rows: int) -> int:
    return int(_load().orc_num_leaves(m, leaf_rows))


def tree_level_counts(P: int):
    cnt = (ctypes.c_int64 * 64)()
    L = _load().orc_tree_levels(P, cnt, 64)
    return [int(cnt[i]) for i in range(L)]


class TSQR:
    """TSQR of A on the hybrid tree: leaves of ``leaf_rows`` rows (the last leaf
    absorbs the remainder), each reduced by a flat chain over tiles of
    ``tile_rows`` rows, then a binary tree over the leaf R factors."""

    def __init__(self, A: np.ndarray, leaf_rows: int, tile_rows: Optional[int] = None):
        A = _f64(A)
        self.m, self.n = A.shape
        if tile_rows is None:
            tile_rows = leaf_rows
        self.leaf_rows, self.tile_rows = int(leaf_rows), int(tile_rows)
        self._lib = _load()
        self._st = self._lib.orc_tsqr_factor(self.m, self.n, _p(A), _ld(A), self.leaf_rows, self.tile_rows)
        if not self._st:
            raise ValueError("TSQR oracle: bad arguments")

    def __del__(self):
        st = getattr(self, "_st", None)
        if st:
            self._lib.orc_tsqr_free(st)
            self._st = None

    @property
    def num_leaves(self) -> int:
        return int(self._lib.orc_tsqr_num_leaves(self._st))

    @property
    def num_levels(self) -> int:
        return int(self._lib.orc_tsqr_num_levels(self._st))

    def R(self) -> np.ndarray:
        R = np.zeros((self.n, self.n), dtype=np.float64, order="F")
        self._lib.orc_tsqr_R(self._st, _p(R), self.n)
        return R

    def signs(self) -> np.ndarray:
        d = np.zeros(self.n, dtype=np.float64)
        self._lib.orc_tsqr_signs(self._st, _p(d))
        return d

    def form_q(self) -> np.ndarray:
        Q = np.zeros((self.m, self.n), dtype=np.float64, order="F")
        self._lib.orc_tsqr_form_q(self._st, _p(Q), self.m)
        return Q

    def apply_qt(self, B: np.ndarray) -> np.ndarray:
        B = _f64(B).copy(order="F")
        if B.shape[0] != self.m:
            raise ValueError("apply_qt: B must have m rows")
        self._lib.orc_tsqr_apply_qt(self._st, B.shape[1], _p(B), _ld(B))
        return B

    def node(self, level: int, q: int):
        """(V, tau) of tree node q at level ``level`` (rows = 2n); None for a
        pass-through node."""
        V = ctypes.POINTER(ctypes.c_double)()
        t = ctypes.POINTER(ctypes.c_double)()
        rows = self._lib.orc_tsqr_node(self._st, level, q, ctypes.byref(V), ctypes.byref(t))
        if rows < 0:
            raise IndexError("no such node")
        if rows == 0:
            return None
        Va = np.ctypeslib.as_array(V, shape=(self.n * rows,)).reshape((self.n, rows)).T.copy()
        ta = np.ctypeslib.as_array(t, shape=(self.n,)).copy()
        return Va, ta

    def node_homes(self, level: int, q: int):
        """(first leaf of the left subtree, first leaf of the right subtree or -1)."""
        a = ctypes.c_int64(); b = ctypes.c_int64()
        if self._lib.orc_tsqr_node_homes(self._st, level, q, ctypes.byref(a), ctypes.byref(b)) != 0:
            raise IndexError("no such node")
        return int(a.value), int(b.value)

    def leaf_stage(self, leaf: int, k: int):
        V = ctypes.POINTER(ctypes.c_double)()
        t = ctypes.POINTER(ctypes.c_double)()
        rows = self._lib.orc_tsqr_leaf_stage(self._st, leaf, k, ctypes.byref(V), ctypes.byref(t))
        if rows < 0:
            raise IndexError("no such stage")
        Va = np.ctypeslib.as_array(V, shape=(self.n * rows,)).reshape((self.n, rows)).T.copy()
        ta = np.ctypeslib.as_array(t, shape=(self.n,)).copy()
        return Va, ta


# ---------------------------------------------------------------- Sec. 5 competitors
def _cmp(fn: str, A: np.ndarray):
    A = _f64(A)
    m, n = A.shape
    Q = np.zeros((m, n), order="F")
    R = np.zeros((n, n), order="F")
    info = getattr(_load(), fn)(m, n, _p(A), _ld(A), _p(Q), m, _p(R), n)
    return Q, R, int(info)


def cholqr(A: np.ndarray):
    """CholeskyQR (Sec. 5): G = A^T A = R^T R, Q = A R^{-1}.  Returns (Q, R,
    info); info = j + 1 when the j-th Cholesky pivot is not positive."""
    return _cmp("orc_cholqr", A)


def cholqr2(A: np.ndarray):
    """CholeskyQR applied to A, then to its Q; R = R2 R1.  (Q, R, info)."""
    return _cmp("orc_cholqr2", A)


def cgs(A: np.ndarray):
    """Classical Gram-Schmidt (Sec. 5).  (Q, R, info); info = j + 1 on a zero norm."""
    return _cmp("orc_cgs", A)


def mgs(A: np.ndarray):
    """Modified Gram-Schmidt (Sec. 5).  (Q, R, info); info = j + 1 on a zero norm."""
    return _cmp("orc_mgs", A)
