"""Exact-rational QR of small integer matrices -- an independent pin for the oracle.

For full-column-rank integer A, A^T A = L D L^T (unit lower L, diagonal D > 0) is
computed in exact rational arithmetic.  The unique QR with diag(R) > 0 is then
R = D^{1/2} L^T and Q = A L^{-T} D^{-1/2}; the only inexact step is the square
root of each d_i, taken with 50 significant digits before rounding to float64.
None of this uses Householder reflections, so it shares no mistake with the oracle.
"""
from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction
from typing import List, Optional, Tuple

import numpy as np

getcontext().prec = 50


def _fr_matrix(A: np.ndarray) -> List[List[Fraction]]:
    m, n = A.shape
    out = []
    for i in range(m):
        row = []
        for j in range(n):
            v = A[i, j]
            assert float(v).is_integer(), "exact pins take integer matrices"
            row.append(Fraction(int(v)))
        out.append(row)
    return out


def _sqrt_dec(q: Fraction) -> Decimal:
    return (Decimal(q.numerator) / Decimal(q.denominator)).sqrt()


def ldl_of_gram(A: np.ndarray) -> Optional[Tuple[List[List[Fraction]], List[Fraction]]]:
    """L, d with A^T A = L diag(d) L^T, or None when some d_i == 0 (rank deficient)."""
    F = _fr_matrix(A)
    m, n = A.shape
    G = [[sum((F[k][i] * F[k][j] for k in range(m)), Fraction(0)) for j in range(n)] for i in range(n)]
    L = [[Fraction(1) if i == j else Fraction(0) for j in range(n)] for i in range(n)]
    d = [Fraction(0)] * n
    for j in range(n):
        d[j] = G[j][j] - sum((L[j][k] * L[j][k] * d[k] for k in range(j)), Fraction(0))
        if d[j] == 0:
            return None
        for i in range(j + 1, n):
            L[i][j] = (G[i][j] - sum((L[i][k] * L[j][k] * d[k] for k in range(j)), Fraction(0))) / d[j]
    return L, d


def exact_qr(A: np.ndarray):
    """(R, Q) as float64 from exact arithmetic, or None if A is rank deficient."""
    res = ldl_of_gram(A)
    if res is None:
        return None
    L, d = res
    m, n = A.shape
    F = _fr_matrix(A)
    sd = [_sqrt_dec(x) for x in d]
    R = np.zeros((n, n))
    for i in range(n):
        for j in range(i, n):
            R[i, j] = float(sd[i] * (Decimal(L[j][i].numerator) / Decimal(L[j][i].denominator)))
    # M = A L^{-T}: M[:, j] = A[:, j] - sum_{k<j} M[:, k] L[j][k]
    M = [[Fraction(0)] * n for _ in range(m)]
    for j in range(n):
        for r in range(m):
            v = F[r][j]
            for k in range(j):
                v -= M[r][k] * L[j][k]
            M[r][j] = v
    Q = np.zeros((m, n))
    for r in range(m):
        for j in range(n):
            q = M[r][j]
            Q[r, j] = float((Decimal(q.numerator) / Decimal(q.denominator)) / sd[j])
    return R, Q


def exact_lstsq(A: np.ndarray, b: np.ndarray) -> List[Fraction]:
    """x solving the normal equations A^T A x = A^T b exactly."""
    F = _fr_matrix(A)
    m, n = A.shape
    bb = [Fraction(int(v)) for v in b]
    G = [[sum((F[k][i] * F[k][j] for k in range(m)), Fraction(0)) for j in range(n)] for i in range(n)]
    h = [sum((F[k][i] * bb[k] for k in range(m)), Fraction(0)) for i in range(n)]
    # Gaussian elimination (G is SPD, no pivoting needed in exact arithmetic)
    for c in range(n):
        for r in range(c + 1, n):
            f = G[r][c] / G[c][c]
            for k in range(c, n):
                G[r][k] -= f * G[c][k]
            h[r] -= f * h[c]
    x = [Fraction(0)] * n
    for r in range(n - 1, -1, -1):
        x[r] = (h[r] - sum((G[r][k] * x[k] for k in range(r + 1, n)), Fraction(0))) / G[r][r]
    return x
