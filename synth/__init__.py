"""Seeded synthetic inputs shaped like the TSQR workloads.

This module serves both the oracle-side tests and the GPU path.  It holds none
of TSQR's arithmetic: it only draws random numbers and builds matrices with a
prescribed spectrum (Haar factors come from a library QR of a Gaussian matrix --
input generation only) or a Krylov-type basis.  All matrices are float64 and
column-major (numpy Fortran order, or a torch tensor whose transpose is
contiguous).

Recipes
-------
* ``gaussian``: entries iid N(0, 1) from numpy PCG64 ``default_rng(seed)``.
* ``prescribed_sigma``: A = U diag(sigma) V^T, U Haar m x n, V Haar n x n, both the
  Q of a Gaussian matrix with the signs fixed so that diag(R) > 0, and
  sigma_i = 10**(-decades * i / (n - 1)).
* ``krylov_basis``: the s-step monomial basis of the 2-D 5-point Laplacian
  (4 on the diagonal, -1 for the N/S/E/W neighbours, zero Dirichlet boundary,
  row-major grid ordering i*g + j): v_0 = b/||b||, v_{k+1} = L v_k/||L v_k||,
  b iid N(0, 1).
* ``batched_shapes``: m_i uniform on [m_lo, m_hi] (numpy ``integers``), n_i
  uniform on ``n_choices``.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np


def gaussian(m: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((n, m)).T)


def _haar(rng: np.random.Generator, m: int, n: int) -> np.ndarray:
    G = rng.standard_normal((n, m)).T  # Fortran-ordered m x n
    Q, R = np.linalg.qr(G, mode="reduced")
    s = np.where(np.diag(R) < 0, -1.0, 1.0)
    return Q * s[None, :]


def log_sigma(n: int, decades: float) -> np.ndarray:
    if n == 1:
        return np.ones(1)
    return 10.0 ** (-decades * np.arange(n) / (n - 1))


def prescribed_sigma(m: int, n: int, seed: int, decades: float = 12.0) -> Tuple[np.ndarray, np.ndarray]:
    """A = U diag(sigma) V^T with sigma log-spaced from 1 to 10**-decades.
    Returns (A, sigma)."""
    rng = np.random.default_rng(seed)
    U = _haar(rng, m, n)
    V = _haar(rng, n, n)
    sig = log_sigma(n, decades)
    A = np.asfortranarray((U * sig[None, :]) @ V.T)
    return A, sig


def prescribed_sigma_torch(m: int, n: int, seed: int, decades: float, device: str = "cuda"):
    """The same recipe drawn with torch's generator on ``device`` (for sizes
    where host generation would dominate the run).  Returns a (n, m) row-major
    tensor T; A = T.t() is the m x n column-major matrix.  sigma is returned on
    the host.  The draws differ from the numpy recipe of the same seed."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    G = torch.randn((n, m), generator=g, device=device, dtype=torch.float64)
    # Q of G^T through the Q of its transpose: G^T = U R
    U, R = torch.linalg.qr(G.t(), mode="reduced")
    s = torch.where(torch.diagonal(R) < 0, -1.0, 1.0).to(torch.float64)
    U = U * s[None, :]
    H = torch.randn((n, n), generator=g, device=device, dtype=torch.float64)
    V, RV = torch.linalg.qr(H, mode="reduced")
    V = V * torch.where(torch.diagonal(RV) < 0, -1.0, 1.0)[None, :]
    sig = torch.tensor(log_sigma(n, decades), dtype=torch.float64, device=device)
    A = (U * sig[None, :]) @ V.t().contiguous()
    T = A.t().contiguous()
    del G, U, R, H, V, RV, A
    return T, log_sigma(n, decades)


def laplacian_2d_apply(v: np.ndarray, g: int) -> np.ndarray:
    """y = L v for the g x g 5-point Laplacian with zero Dirichlet boundary."""
    X = v.reshape(g, g)
    Y = 4.0 * X
    Y[1:, :] -= X[:-1, :]
    Y[:-1, :] -= X[1:, :]
    Y[:, 1:] -= X[:, :-1]
    Y[:, :-1] -= X[:, 1:]
    return Y.reshape(-1)


def krylov_basis(g: int, s: int, seed: int) -> np.ndarray:
    """m = g*g rows, n = s + 1 columns: [v_0, ..., v_s], each column normalised."""
    rng = np.random.default_rng(seed)
    m = g * g
    B = np.empty((m, s + 1), dtype=np.float64, order="F")
    v = rng.standard_normal(m)
    v /= np.linalg.norm(v)
    B[:, 0] = v
    for k in range(s):
        v = laplacian_2d_apply(v, g)
        v /= np.linalg.norm(v)
        B[:, k + 1] = v
    return B


def batched_shapes(count: int, seed: int, m_lo: int = 1000, m_hi: int = 200000,
                   n_choices: Sequence[int] = (8, 16, 32, 64)) -> List[Tuple[int, int]]:
    rng = np.random.default_rng(seed)
    ms = rng.integers(m_lo, m_hi + 1, size=count)
    ns = rng.choice(np.asarray(n_choices), size=count)
    return [(int(a), int(b)) for a, b in zip(ms, ns)]


def small_int_matrix(m: int, n: int, seed: int, lo: int = -5, hi: int = 5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.integers(lo, hi + 1, size=(m, n)).astype(np.float64))
