"""The autotuner through the C ABI: it times the candidates of a class, keeps
the fastest in the JSON cache, answers the same class from the cache, and the
geometry it picks gives a correct factorisation; plans created without
options take the cached geometry when TSQR_TUNE_CACHE names the cache."""
import numpy as np
import pytest

import synth
from gpu_util import announce, need_gpu
from metrics import backward_error, fp64_bound, orthogonality

pytestmark = pytest.mark.gpu


def test_autotune_fp64_then_cache_then_plans(tmp_path, monkeypatch):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    m, n = 200000, 16
    A = synth.gaussian(m, n, seed=31)
    Ad = T.to_colmajor(torch.from_numpy(A))
    A0 = Ad.clone()
    cache = str(tmp_path / "tune.json")
    announce("autotune 200000x16")
    r = T.autotune(m, n, A=Ad, cache=cache, reps=2)
    print("autotune:", r)
    assert not r["from_cache"] and r["candidates"] >= 6 and r["ms"] > 0
    assert torch.equal(Ad, A0)  # the scratch matrix is only read
    r2 = T.autotune(m, n, cache=cache)
    assert r2["from_cache"] and r2["opts"] == r["opts"] and r2["candidates"] == 0
    o = r["opts"]
    kw = dict(tree=o["tree"], leaf_rows=o["leaf_rows"], flat_len=o["flat_len"], waves=o["waves"])
    with T.Plan(m, n, **kw) as p:
        R = p.factor(Ad)
        Q = p.form_q(Ad)
        torch.cuda.synchronize()
        info_tuned = p.info()
    R, Q = R.cpu().numpy(), Q.cpu().numpy()
    assert backward_error(A, Q, R) <= fp64_bound(n)
    assert orthogonality(Q) <= fp64_bound(n)
    monkeypatch.setenv("TSQR_TUNE_CACHE", cache)
    with T.Plan(m, n) as p:
        info = p.info()
    assert info["leaf_rows"] == info_tuned["leaf_rows"] and info["waves"] == info_tuned["waves"]


def test_autotune_mixed_and_r_only_classes(tmp_path):
    torch = need_gpu()
    from paper_0809_2407_amd import tsqr as T

    cache = str(tmp_path / "tune.json")
    announce("autotune mixed 50000x32")
    rm = T.autotune(50000, 32, precision="mixed", cache=cache, reps=1)
    announce("autotune R only 50000x32")
    rr = T.autotune(50000, 32, want_q=False, cache=cache, reps=1)
    assert rm["candidates"] >= 3 and rr["candidates"] >= 3
    assert T.tune_cache_lookup(cache, 50000, 32, precision="mixed")["opts"] == rm["opts"]
    assert T.tune_cache_lookup(cache, 50000, 32, want_q=False)["opts"] == rr["opts"]
    assert T.tune_cache_lookup(cache, 50000, 32) is None  # FP64 R+Q not tuned
    torch.cuda.synchronize()
