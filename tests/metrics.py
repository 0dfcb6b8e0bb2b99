"""Error measures shared by the tests (Frobenius norms throughout)."""
from __future__ import annotations

import numpy as np

EPS = 2.0 ** -53


def fp64_bound(n: int) -> float:
    """20 * n * 2^-53: the FP64 bound on backward error and orthogonality."""
    return 20.0 * n * EPS


def backward_error(A, Q, R) -> float:
    return float(np.linalg.norm(A - Q @ R) / np.linalg.norm(A))


def orthogonality(Q) -> float:
    n = Q.shape[1]
    return float(np.linalg.norm(Q.T @ Q - np.eye(n)))


def rel_diff(X, Xref) -> float:
    d = np.linalg.norm(Xref)
    return float(np.linalg.norm(X - Xref) / (d if d > 0 else 1.0))


def is_upper(R, tol=0.0) -> bool:
    return bool(np.all(np.abs(np.tril(R, -1)) <= tol))
