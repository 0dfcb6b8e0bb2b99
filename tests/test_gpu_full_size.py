"""Parity at the full sizes of the measured workloads, with the geometry a plan
chooses by itself (the launch configuration bench.py times).

- m = 2^24, n = 32 and 64, Gaussian entries: the whole R and the whole Q
  against the oracle run on the same tree, element by element.
- The measured matrices themselves (sigma log-spaced, kappa = 1e12 at n = 32
  and 1e6 at n = 64, the seed bench.py uses): R normwise against the oracle
  (R is unique up to signs, Sec. 2) and Q through backward error and
  orthogonality.  Q's columns of the small singular values are determined only
  to about kappa eps, so they are not compared element by element.
- The mixed path on the n = 64 matrix: its stated bounds, and R within 1e-5
  of the FP64 oracle's.
- Q^T B at the Krylov workload's shape (m = 2^22, n = 17, 32 columns): every
  row against the oracle's on Gaussian inputs; on the Krylov basis itself, the
  column norms Q^T keeps and the top n rows against the plan's explicit Q.

The oracle runs on the host's cores; each case takes some seconds."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import announce, need_gpu
from metrics import fp64_bound

pytestmark = pytest.mark.gpu

M = 1 << 24
SEED = 2024  # the seed of the measured workloads


def _device_errors(torch, A, Q, R):
    """Backward error and orthogonality in FP64 on the device (Q^T Q summed over
    row blocks, so the sum itself stays below the orthogonality measured)."""
    m, n = A.shape
    with torch.no_grad():
        bwd = float(torch.linalg.norm(torch.addmm(A, Q, R, alpha=-1.0)) / torch.linalg.norm(A))
        nb = 4096
        Qb = Q.t().reshape(n, m // nb, nb)
        G = torch.zeros((n, n), dtype=torch.float64, device=Q.device)
        for c in range(0, m // nb, 256):
            blk = Qb[:, c:c + 256, :].permute(1, 0, 2).contiguous()
            G += torch.bmm(blk, blk.transpose(1, 2).contiguous()).sum(dim=0)
        orth = float(torch.linalg.norm(G - torch.eye(n, dtype=torch.float64, device=Q.device)))
    return bwd, orth


def _factor(torch, T, A, precision="fp64"):
    m, n = A.shape
    with T.Plan(m, n, precision=precision) as p:
        info = p.info()
        V = T.colmajor(m, n) if precision == "fp64" else None
        R, Q = T.colmajor(n, n), T.colmajor(m, n)
        p.factor_into(A, V, R)
        p.form_q(V, Q)
        torch.cuda.synchronize()
        info = p.info()
    del V
    return R, Q, info


@pytest.mark.parametrize("n", [32, 64])
def test_gaussian_r_and_q_element_by_element(n):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    announce(f"full size Gaussian {M} x {n}")
    g = torch.Generator(device="cuda")
    g.manual_seed(3000 + n)
    A = torch.randn((n, M), generator=g, device="cuda", dtype=torch.float64).t()
    R, Q, info = _factor(torch, T, A)
    bwd, orth = _device_errors(torch, A, Q, R)
    assert bwd <= fp64_bound(n) and orth <= fp64_bound(n), (bwd, orth)
    Ah = np.asfortranarray(A.cpu().numpy())
    del A
    Rh = R.cpu().numpy()
    Qh = Q.cpu().numpy()
    del Q
    torch.cuda.empty_cache()
    announce(f"oracle on the same tree: {info['num_leaves']} leaves of {info['leaf_rows']} rows")
    t = oracle.TSQR(Ah, info["leaf_rows"], info["tile_rows"])
    Ro = t.R()
    assert np.abs(Rh - Ro).max() <= 1e-13 * np.linalg.norm(Ro)
    Qo = t.form_q()
    del t, Ah
    assert np.abs(Qh - Qo).max() <= 1e-13


@pytest.mark.parametrize("n,decades", [(32, 12.0), (64, 6.0)])
def test_measured_matrices(n, decades):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    announce(f"full size kappa 1e{decades:g} {M} x {n}")
    At, _ = synth.prescribed_sigma_torch(M, n, SEED, decades, device="cuda")
    A = At.t()
    R, Q, info = _factor(torch, T, A)
    bwd, orth = _device_errors(torch, A, Q, R)
    assert bwd <= fp64_bound(n) and orth <= fp64_bound(n), (bwd, orth)
    del Q
    Ah = np.asfortranarray(A.cpu().numpy())
    del A, At
    torch.cuda.empty_cache()
    Rh = R.cpu().numpy()
    assert np.all(np.diag(Rh) >= 0) and np.all(np.tril(Rh, -1) == 0)
    Ro = oracle.TSQR(Ah, info["leaf_rows"], info["tile_rows"]).R()
    assert np.linalg.norm(Rh - Ro) <= 1e-13 * np.linalg.norm(Ro)


def test_mixed_on_the_n64_matrix():
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    n = 64
    announce(f"full size mixed {M} x {n}")
    At, _ = synth.prescribed_sigma_torch(M, n, SEED, 6.0, device="cuda")
    A = At.t()
    R, Q, info = _factor(torch, T, A, precision="mixed")
    assert info["reorth_applied"] == 1
    bwd, orth = _device_errors(torch, A, Q, R)
    assert bwd <= 1e-6 and orth <= 1e-13, (bwd, orth)
    del Q
    Ah = np.asfortranarray(A.cpu().numpy())
    del A, At
    torch.cuda.empty_cache()
    Rh = R.cpu().numpy()
    pf = T.plan_query(M, n)
    Ro = oracle.TSQR(Ah, pf["leaf_rows"], pf["tile_rows"]).R()
    assert np.linalg.norm(Rh - Ro) <= 1e-5 * np.linalg.norm(Ro)


def test_qtb_at_the_krylov_shape():
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n, k = 2048 * 2048, 17, 32
    g = torch.Generator(device="cuda")
    g.manual_seed(SEED + 1)
    B0 = torch.randn((k, m), generator=g, device="cuda", dtype=torch.float64).t()
    Bh = np.asfortranarray(B0.cpu().numpy())
    # Gaussian inputs: every row of Q^T B against the oracle on the same tree
    announce(f"Q^T B at {m} x {n}, {k} columns, Gaussian")
    A = torch.randn((n, m), generator=g, device="cuda", dtype=torch.float64).t()
    Ah = np.asfortranarray(A.cpu().numpy())
    with T.Plan(m, n) as p:
        info = p.info()
        V, R = T.colmajor(m, n), T.colmajor(n, n)
        B = T.colmajor(m, k)
        B.copy_(B0)
        p.factor_into(A, V, R)
        p.apply_qt(V, B)
        torch.cuda.synchronize()
        X = B.cpu().numpy()
    del V, B, A
    t = oracle.TSQR(Ah, info["leaf_rows"], info["tile_rows"])
    Xo = t.apply_qt(Bh)
    assert np.abs(X - Xo).max() <= 1e-13 * np.linalg.norm(Bh)
    del t, Xo, X, Ah
    # the Krylov basis itself (ill-conditioned): properties that hold at any kappa
    announce(f"Q^T B on the Krylov basis {m} x {n}")
    Kh = synth.krylov_basis(2048, 16, SEED)
    K = T.to_colmajor(torch.from_numpy(Kh))
    with T.Plan(m, n) as p:
        V, R, Q = T.colmajor(m, n), T.colmajor(n, n), T.colmajor(m, n)
        B = T.colmajor(m, k)
        B.copy_(B0)
        p.factor_into(K, V, R)
        p.form_q(V, Q)
        p.apply_qt(V, B)
        torch.cuda.synchronize()
        with torch.no_grad():
            keep = float(((torch.linalg.norm(B, dim=0) - torch.linalg.norm(B0, dim=0)).abs()
                          / torch.linalg.norm(B0, dim=0)).max())
            top = float((B[:n] - Q.t().matmul(B0)).abs().max() / torch.linalg.norm(B0))
    assert keep <= 1e-13, keep
    assert top <= 1e-15, top


def test_more_elements_than_a_32_bit_index_reaches():
    """m = 2^27 + 4321, n = 20: 2.7e9 elements (21.5 GB per matrix), so element
    offsets pass 2^31 and byte offsets 2^34, in the geometry a plan picks by
    itself and with a ragged last tile.  R and Q element by element against the
    oracle on the same tree; backward error and orthogonality on the device."""
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = (1 << 27) + 4321, 20
    announce(f"beyond 32-bit element offsets: {m} x {n}")
    g = torch.Generator(device="cuda")
    g.manual_seed(SEED + 7)
    A = torch.randn((n, m), generator=g, device="cuda", dtype=torch.float64).t()
    with T.Plan(m, n) as p:
        V, R, Q = T.colmajor(m, n), T.colmajor(n, n), T.colmajor(m, n)
        p.factor_into(A, V, R)
        p.form_q(V, Q)
        torch.cuda.synchronize()
        info = p.info()
    del V
    torch.cuda.empty_cache()
    assert (m - 1) * n >= 1 << 31 and m % info["tile_rows"] != 0
    with torch.no_grad():
        # by row chunks, each copied to compact storage first: a device GEMM on
        # the column-major views themselves (leading dimension m, so the operand
        # spans (n - 1) m + rows > 2^31 elements) returned wrong products here,
        # for a Q and R that match the oracle's
        e2, a2, bad = 0.0, 0.0, []
        for r in range(0, m, 1 << 22):
            Ac = A[r:r + (1 << 22)].contiguous()
            Ec = torch.addmm(Ac, Q[r:r + (1 << 22)].contiguous(), R.contiguous(), alpha=-1.0)
            ec, ac = float(torch.linalg.norm(Ec)) ** 2, float(torch.linalg.norm(Ac)) ** 2
            e2, a2 = e2 + ec, a2 + ac
            if ec > 1e-24 * ac:
                bad.append(r)
            del Ec, Ac
        bwd = (e2 / a2) ** 0.5
        if bad:
            announce(f"row chunks of 2^22 with a large residual start at rows {bad[:8]} ({len(bad)} chunks)")
        G = torch.zeros((n, n), dtype=torch.float64, device="cuda")
        for r in range(0, m, 1 << 22):
            blk = Q[r:r + (1 << 22)]
            nb = blk.shape[0] // 4096 * 4096
            if nb:
                Qb = blk[:nb].t().reshape(n, nb // 4096, 4096).permute(1, 0, 2).contiguous()
                G += torch.bmm(Qb, Qb.transpose(1, 2).contiguous()).sum(dim=0)
                del Qb
            if nb < blk.shape[0]:
                G += blk[nb:].t().matmul(blk[nb:])
        orth = float(torch.linalg.norm(G - torch.eye(n, dtype=torch.float64, device="cuda")))
    announce(f"device: backward {bwd:.2e}, orthogonality {orth:.2e}; oracle on {info['num_leaves']} leaves")
    Ah = np.asfortranarray(A.cpu().numpy())
    del A
    Rh = R.cpu().numpy()
    Qh = Q.cpu().numpy()
    del Q
    torch.cuda.empty_cache()
    t = oracle.TSQR(Ah, info["leaf_rows"], info["tile_rows"])
    del Ah
    Ro = t.R()
    Qo = t.form_q()
    del t
    dr = np.abs(Rh - Ro).max() / np.linalg.norm(Ro)
    dq = np.abs(Qh - Qo).max(axis=1)
    rows = np.nonzero(dq > 1e-13)[0]
    announce(f"oracle: |R - R_oracle| / |R| {dr:.2e}, max |Q - Q_oracle| {dq.max():.2e}, "
             f"{rows.size} rows of Q off" + (f" (first {rows[:4]}, last {rows[-1]})" if rows.size else ""))
    assert dr <= 1e-13 and rows.size == 0
    assert bwd <= fp64_bound(n) and orth <= fp64_bound(n), (bwd, orth)
