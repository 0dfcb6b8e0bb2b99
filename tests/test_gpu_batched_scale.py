"""Batched plans at the scale of the many-problem workload: the persistent
grids hold at most 2048 wavefronts, and here every width class has more leaf
items than that, so each wavefront walks several (problem, leaf) items and
reuses its LDS between them.  Every problem is checked bit for bit against a
single-problem plan of the same geometry, against the oracle's R (uniqueness
of R up to signs, Sec. 2) and against the bounds of its path."""
import concurrent.futures as cf

import numpy as np
import pytest

import oracle
from gpu_util import announce, need_gpu
from metrics import backward_error, fp64_bound, is_upper, orthogonality, rel_diff

pytestmark = pytest.mark.gpu

GRID_WAVES = 2048  # the persistent launches' wavefront cap


def _shapes(count, m_lo, m_hi, seed):
    rng = np.random.default_rng(seed)
    ms = [int(x) for x in rng.integers(m_lo, m_hi + 1, size=count)]
    ns = [int(x) for x in rng.choice([8, 16, 32, 64], size=count)]
    return ms, ns


def _matrices(ms, ns, seed):
    rng = np.random.default_rng(seed)
    return [np.asfortranarray(rng.standard_normal((m, n))) for m, n in zip(ms, ns)]


def _oracle_rs(mats):
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        return list(ex.map(lambda A: oracle.qr_reference(A, want_q=False), mats))


def _leaf_items_per_class(bp, count):
    items = {}
    for i in range(count):
        info = bp.problem_info(i)
        items[info["n_padded"]] = items.get(info["n_padded"], 0) + info["num_leaves"]
    return items


def _run_batched(T, torch, bp, mats):
    As = [T.to_colmajor(torch.from_numpy(A)) for A in mats]
    Rs = bp.factor(As)
    Qs = bp.form_q(As, [T.colmajor(A.shape[0], A.shape[1]) for A in mats])
    torch.cuda.synchronize()
    Rh = [R.cpu().numpy() for R in Rs]
    Qh = [Q.cpu().numpy() for Q in Qs]
    del As, Rs, Qs
    return Rh, Qh


def _single(T, torch, A, precision, **kw):
    m, n = A.shape
    Ad = T.to_colmajor(torch.from_numpy(A))
    with T.Plan(m, n, precision=precision, **kw) as p:
        R = p.factor(Ad)
        Q = p.form_q(Ad, T.colmajor(m, n))
        torch.cuda.synchronize()
    return R.cpu().numpy(), Q.cpu().numpy()


def _check_scale(precision, count, m_lo, m_hi, seed, tree="auto", min_items=GRID_WAVES + 1):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    ms, ns = _shapes(count, m_lo, m_hi, seed)
    announce(f"batched {precision} at scale: {count} problems, m in [{m_lo}, {m_hi}], tree {tree}")
    mats = _matrices(ms, ns, seed + 1)
    kw = {} if tree == "auto" else {"tree": tree}
    with T.BatchedPlan(ms, ns, precision=precision, **kw) as bp:
        items = _leaf_items_per_class(bp, count)
        announce(f"leaf items per width class {items}")
        assert len(items) == 4 and min(items.values()) >= min_items
        lrs = [bp.problem_info(i)["leaf_rows"] for i in range(count)]
        Rb, Qb = _run_batched(T, torch, bp, mats)
    announce("oracle R of every problem")
    Ro = _oracle_rs(mats)
    mixed = precision == "mixed"
    worst = {"R": 0.0, "bwd": 0.0, "orth": 0.0}
    for i, A in enumerate(mats):
        if i % 500 == 0:
            announce(f"batched {precision} problem {i} {A.shape}")
        n = A.shape[1]
        R1, Q1 = _single(T, torch, A, precision, leaf_rows=lrs[i], **kw)
        assert np.array_equal(Rb[i], R1) and np.array_equal(Qb[i], Q1), f"problem {i} {A.shape}"
        assert is_upper(Rb[i]) and np.all(np.diag(Rb[i]) >= 0)
        dr = rel_diff(Rb[i], Ro[i])
        bwd = backward_error(A, Qb[i], Rb[i])
        orth = orthogonality(Qb[i])
        rb, bb, ob = (1e-5, 1e-6, 1e-13) if mixed else (1e-13, fp64_bound(n), fp64_bound(n))
        assert dr <= rb and bwd <= bb and orth <= ob, f"problem {i} {A.shape}: {dr:.2e} {bwd:.2e} {orth:.2e}"
        worst["R"] = max(worst["R"], dr / rb)
        worst["bwd"] = max(worst["bwd"], bwd / bb)
        worst["orth"] = max(worst["orth"], orth / ob)
    announce(f"worst fraction of each bound over {count} problems: {worst}")


def test_batched_fp64_every_wave_walks_several_leaves():
    # automatic geometry: more than 2048 leaf items in every width class
    # (2156 at 64 columns, up to 10322 at 16)
    _check_scale("fp64", 3600, 1000, 5000, seed=31)


def test_batched_fp64_binary_tree_deep_levels():
    # every tile a leaf: over 7000 leaf items and five to six tree levels of
    # hundreds of nodes at 64 columns
    _check_scale("fp64", 1200, 1000, 2000, seed=37, tree="binary", min_items=1000)


def test_batched_mixed_every_wave_walks_several_leaves():
    # the FP32 tiles are twice as tall: m from 2000 keeps every class past 2048
    _check_scale("mixed", 3600, 2000, 6000, seed=41)
