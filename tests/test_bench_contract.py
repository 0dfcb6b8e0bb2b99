"""bench.py without a GPU: the flop and byte conventions, the refusal of more
than one GPU, and that the committed byte-counter summaries under profiles/
were taken from the current kernel sources (bench.py reports their traffic
only then)."""
import io
import json
import os
import sys
from contextlib import redirect_stdout

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_flop_conventions():
    # Sec. 4.2: 2mn^2 - 2n^3/3 for R (Householder QR); twice that with the explicit Q
    m, n = 1 << 24, 32
    assert bench.flops_r(m, n) == 2.0 * m * n * n - 2.0 * n ** 3 / 3.0
    assert bench.flops_rq(m, n) == 2.0 * bench.flops_r(m, n)
    assert bench.flops_r(n, n) > 0


def test_more_than_one_gpu_is_refused():
    out = io.StringIO()
    with redirect_stdout(out):
        rc = bench.main(["--gpus", "2"])
    assert rc == 2
    msg = json.loads(out.getvalue().strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_bad_step_counts_are_refused():
    for argv in (["--steps", "0"], ["--warmup", "-1"]):
        out = io.StringIO()
        with redirect_stdout(out):
            rc = bench.main(argv)
        assert rc == 2 and "steps" in json.loads(out.getvalue())["error"]


def test_workloads_are_well_formed():
    for name, w in bench.WORKLOADS.items():
        assert w["mode"] in ("r", "rq"), name
        assert w["m"] >= w["n"] >= 1, name
        assert w.get("precision", "fp64") in ("fp64", "mixed"), name
        assert ("mixed" in name) == (w.get("precision") == "mixed"), name
        assert f"_n{w['n']}" in name and f"m{w['m']}" in name, name
    assert bench.DEFAULT in bench.WORKLOADS
    for name, w in bench.BATCHED.items():
        assert w["count"] >= 1 and w["m_lo"] <= w["m_hi"], name
    # the paper-shaped sweep: TSQR plans exist for every width up to 64 (wider ones go through CAQR)
    from paper_0809_2407_amd import tsqr as T
    for m, n in bench.PAPER_SHAPES:
        assert m >= n >= 1, (m, n)
        if n <= 64:
            assert T.plan_query(m, n)["num_leaves"] >= 1


def test_profiles_match_the_kernel_sources():
    # the default workload's dominant kernel and the Q kernel have byte counters
    # taken from the kernel sources as they are now, at the geometry a plan
    # chooses for it
    from paper_0809_2407_amd import tsqr as T

    m, n = bench.WORKLOADS[bench.DEFAULT]["m"], bench.WORKLOADS[bench.DEFAULT]["n"]
    info = T.plan_query(m, n)
    for kernel in ("leaf", "form_q"):
        t = bench.measured_traffic(m, n, kernel, info["leaf_rows"], info["tile_rows"])
        assert t is not None, f"no byte counters for {kernel} at the current kernel sources"
        # within 15% of the algorithmic 16mn bytes (counters include T slots and re-reads)
        assert 16.0 * m * n <= t <= 1.15 * 16.0 * m * n, (kernel, t)
