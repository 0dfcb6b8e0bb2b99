"""Helpers for the GPU tests: run the HIP path through the C ABI on host
numpy inputs and bring the results back."""
from __future__ import annotations

import sys

import numpy as np
import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU in this environment")
    return torch


def announce(msg: str) -> None:
    """Name the case before a GPU step, flushed, so a crash log points at it."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def run_tsqr(A: np.ndarray, want_q: bool = True, lda: int | None = None, ldq: int | None = None,
             alias: bool = False, **plan_kw):
    """Factor A on the GPU (and form Q).  Returns (R, Q or None, A_after, info)."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = A.shape
    Ad = T.colmajor(m, n, ld=lda or m)
    Ad.copy_(torch.from_numpy(np.ascontiguousarray(A)))
    with T.Plan(m, n, want_q=want_q, **plan_kw) as p:
        info = p.info()
        R = p.factor(Ad)
        Q = None
        if want_q:
            if alias:
                Q = p.form_q(Ad, Ad)
            else:
                Q = p.form_q(Ad, T.colmajor(m, n, ld=ldq or m))
        torch.cuda.synchronize()
    Rh = R.cpu().numpy()
    Qh = Q.cpu().numpy() if Q is not None else None
    return Rh, Qh, Ad.cpu().numpy(), info
