#!/usr/bin/env python3
"""TSQR benchmark on one MI355X: FP64 R + explicit Q of a tall-skinny matrix.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

One step is one pass of the whole hot path over the resident input: the leaf
chains (local Householder QRs of every tile), the binary tree over the leaf R
factors, the root sign normalisation, the top-down seed descent and the Q
expansion (tsqr_factor_into + tsqr_form_q; A is only read, so every step sees
the same input).  Prints ONE JSON line.

Flop convention (nominal): R + Q = 4mn^2 - 4n^3/3, R only = 2mn^2 - 2n^3/3.
Byte convention (algorithmic HBM traffic): factor with reflectors 16mn (read A,
write V), Q expansion 16mn (read V, write Q).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 (vector and matrix)

WORKLOADS = {
    # m = 2^24, n = 32, A = U diag(sigma) V^T, sigma log-spaced 1 .. 1e-12
    "tsqr_fp64_rq_m16777216_n32_kappa1e12": dict(m=1 << 24, n=32, decades=12.0, mode="rq"),
    "tsqr_fp64_r_m16777216_n32_kappa1e12": dict(m=1 << 24, n=32, decades=12.0, mode="r"),
    # m = 4096, n = 16, A iid N(0,1), 8 leaves of 512 rows, binary tree over them
    "tsqr_fp64_rq_m4096_n16_gaussian": dict(m=4096, n=16, decades=None, mode="rq", leaf_rows=512),
    # m = 2^24, n = 64, sigma log-spaced 1 .. 1e-6 (the matrix of the mixed-precision comparison)
    "tsqr_fp64_rq_m16777216_n64_kappa1e6": dict(m=1 << 24, n=64, decades=6.0, mode="rq"),
    "tsqr_fp64_r_m16777216_n64_kappa1e6": dict(m=1 << 24, n=64, decades=6.0, mode="r"),
    # the same matrix on the mixed-precision path (FP32 first pass, FP64 second pass)
    "tsqr_mixed_rq_m16777216_n64_kappa1e6": dict(m=1 << 24, n=64, decades=6.0, mode="rq", precision="mixed"),
    "tsqr_mixed_rq_m16777216_n32_kappa1e12": dict(m=1 << 24, n=32, decades=12.0, mode="rq", precision="mixed"),
    # s-step monomial basis of the 2-D 5-point Laplacian on a 2048 x 2048 grid (n = 17), R + Q,
    # then Q^T applied to 32 iid N(0,1) right-hand sides
    "tsqr_fp64_rq_qtb_krylov_m4194304_n17_k32": dict(m=2048 * 2048, n=17, decades=None, mode="rq",
                                                     krylov=(2048, 16), rhs=32),
    # the same basis, R + Q only: the FP64 path and the mixed path with its second pass
    "tsqr_fp64_rq_krylov_m4194304_n17": dict(m=2048 * 2048, n=17, decades=None, mode="rq", krylov=(2048, 16)),
    "tsqr_mixed_rq_krylov_m4194304_n17": dict(m=2048 * 2048, n=17, decades=None, mode="rq", krylov=(2048, 16),
                                              precision="mixed"),
}
DEFAULT = "tsqr_fp64_rq_m16777216_n32_kappa1e12"

# Many independent problems: m_i uniform on 1000..200000, n_i uniform on
# {8, 16, 32, 64}, entries iid N(0,1); one batched plan (captured graph) against
# a loop of single-problem calls on the same stream.
BATCHED = {
    "tsqr_batched_fp64_rq_p2048_m1000_200000_n8_64": dict(count=2048, m_lo=1000, m_hi=200000, ns=(8, 16, 32, 64)),
    "tsqr_batched_fp64_rq_p256_m1000_200000_n8_64": dict(count=256, m_lo=1000, m_hi=200000, ns=(8, 16, 32, 64)),
    # the same 256 problems on the mixed path (FP32 first pass, FP64 second pass per problem)
    "tsqr_batched_mixed_rq_p256_m1000_200000_n8_64": dict(count=256, m_lo=1000, m_hi=200000, ns=(8, 16, 32, 64),
                                                          precision="mixed"),
}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def flops_rq(m: int, n: int) -> float:
    return 4.0 * m * n * n - 4.0 * n ** 3 / 3.0


def flops_r(m: int, n: int) -> float:
    return 2.0 * m * n * n - 2.0 * n ** 3 / 3.0


def make_input(w: dict, seed: int):
    import numpy as np
    import torch

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import synth
    from paper_0809_2407_amd import tsqr as T

    m, n = w["m"], w["n"]
    if "krylov" in w:
        g, s_ = w["krylov"]
        A = T.to_colmajor(torch.from_numpy(synth.krylov_basis(g, s_, seed)))
        sig = None
    elif w["decades"] is None:
        A = T.to_colmajor(torch.from_numpy(synth.gaussian(m, n, seed)))
        sig = None
    else:
        At, sig = synth.prescribed_sigma_torch(m, n, seed, w["decades"], device="cuda")
        A = At.t()  # column-major view, ld = m
    torch.cuda.synchronize()
    return A, sig


def sources_sha256() -> str:
    import glob
    import hashlib

    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in sorted(glob.glob(os.path.join(here, "paper_0809_2407_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(m: int, n: int, kernel: str):
    """HBM bytes (read + write) of one launch of `kernel` from the committed
    rocprofv3 byte-counter summary under profiles/, or None when no summary
    matches this workload and the current kernel sources."""
    import glob
    import re

    here = os.path.dirname(os.path.abspath(__file__))
    sha = sources_sha256()
    for f in sorted(glob.glob(os.path.join(here, "profiles", "*.md"))):
        text = open(f).read()
        for blk in re.findall(r"```json\n(.*?)\n```", text, flags=re.S):
            try:
                d = json.loads(blk)
            except ValueError:
                continue
            if d.get("workload_m") == m and d.get("workload_n") == n and d.get("sources_sha256") == sha:
                k = d.get("kernels", {}).get(kernel)
                if k:
                    return k["read_bytes"] + k["write_bytes"]
    return None


def cpu_baseline(A_dev, info: dict, sample_rows: int, mode: str):
    """The oracle as it stands, on the first sample_rows rows of the same input,
    on the host cores (tree of the same shape: same leaf and tile rows)."""
    import numpy as np

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import oracle

    m, n = A_dev.shape
    ms = min(m, sample_rows)
    As = np.asfortranarray(A_dev[:ms].cpu().numpy())
    threads = oracle.num_threads()
    t0 = time.perf_counter()
    t = oracle.TSQR(As, info["leaf_rows"], info["tile_rows"])
    if mode == "rq":
        t.form_q()
    t.R()
    dt = time.perf_counter() - t0
    fl = flops_rq(ms, n) if mode == "rq" else flops_r(ms, n)
    return {"value": fl / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"first {ms} of {m} rows (x{n}), same leaf/tile rows, "
                      f"{'R + explicit Q' if mode == 'rq' else 'R only'}, {dt:.2f} s"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) + sorted(BATCHED))
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=1 << 24)
    ap.add_argument("--no-check", action="store_true", help="skip the accuracy check after timing")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="before warm-up, run one plain device copy of m x n doubles (8mn bytes read, "
                         "8mn written) so that hardware byte counters can be scaled against it")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "this TSQR build runs on one GPU; the multi-GPU path (one all-gather "
                                   "of the R factors) is a design, not a build: use --gpus 1"}))
        return 2

    import torch
    from paper_0809_2407_amd import tsqr as T

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        return 1
    if args.workload in BATCHED:
        return run_batched(args)
    w = dict(WORKLOADS[args.workload])
    m, n, mode = w["m"], w["n"], w["mode"]
    log(f"workload {args.workload}: generating input")
    A, sig = make_input(w, args.seed)
    mixed = w.get("precision", "fp64") == "mixed"
    plan = T.Plan(m, n, precision="mixed" if mixed else "fp64", leaf_rows=w.get("leaf_rows", 0),
                  want_q=(mode == "rq"))
    info = plan.info()
    log(f"plan: {info}")
    V = T.colmajor(m, n) if mode == "rq" and not mixed else None
    Q = T.colmajor(m, n) if mode == "rq" else None
    R = T.colmajor(n, n)
    k_rhs = w.get("rhs", 0)
    if k_rhs:
        g = torch.Generator(device="cuda")
        g.manual_seed(args.seed + 1)
        B0 = torch.randn((k_rhs, m), generator=g, device="cuda", dtype=torch.float64).t()
        B = T.colmajor(m, k_rhs)

    def step():
        plan.factor_into(A, V, R)  # a MIXED plan keeps its reflectors itself (V is None)
        if mode == "rq":
            plan.form_q(V, Q)
        if k_rhs:
            B.copy_(B0)
            plan.apply_qt(V, B)

    if args.calibrate_copy:
        Cdst = T.colmajor(m, n)
        Cdst.copy_(A)
        torch.cuda.synchronize()
        del Cdst
        log(f"calibration copy: {8 * m * n} bytes read, {8 * m * n} bytes written")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    plan.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ph = plan.timings()
    plan.profile(False)
    ms_step = (t1 - t0) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_step:.4f} ms/step; phases {ph}")

    fl = flops_rq(m, n) if mode == "rq" else flops_r(m, n)
    if k_rhs:
        fl += 4.0 * m * n * k_rhs  # Q^T B on k columns
    value = fl / (ms_step * 1e-3) / 1e9
    # dominant kernel: the phase with the largest device time
    if mixed:
        # A read (FP64) + V32 written; V32 read + Q1 written; Q1 read (Gram); Q1 read + Q written (FP64)
        phase_bytes = {"leaf": (12.0 if mode == "rq" else 8.0) * m * n, "q1": 8.0 * m * n,
                       "reorth": 4.0 * m * n, "form_q": 12.0 * m * n}
    else:
        phase_bytes = {"leaf": (16.0 if mode == "rq" else 8.0) * m * n, "form_q": 16.0 * m * n}
    dom = max(phase_bytes, key=lambda k: ph[k][0] / max(1, ph[k][1]) if ph[k][1] else 0.0)
    dom_ms = ph[dom][0] / max(1, ph[dom][1])
    achieved = phase_bytes[dom] / (dom_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(m, n, dom) if mode == "rq" and not mixed else None,
                "kernel": dom,
                "kernel_ms": dom_ms, "bytes_per_launch": phase_bytes[dom]}
    path_bytes = (32.0 if mode == "rq" else 8.0) * m * n + (8.0 * m * n + 16.0 * m * k_rhs if k_rhs else 0.0)
    if mixed and mode == "rq":
        path_bytes = 36.0 * m * n  # the byte model of the mixed path with its Gram pass unfused
    t_roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), path_bytes / (HBM_PEAK_GBS * 1e9))

    result = {
        "metric": "TSQR R+Q GFLOP/s & % roofline; mixed/batched vs FP64 at stated backward error",
        "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "m": m, "n": n, "mode": mode,
                   "sigma": None if sig is None else f"logspace(0,-{w['decades']:g},{n})",
                   "seed": args.seed, "tree": {1: "binary", 2: "flat", 3: "hybrid"}.get(info["tree"], "auto"),
                   "tile_rows": info["tile_rows"], "leaf_rows": info["leaf_rows"],
                   "num_leaves": info["num_leaves"], "tree_levels": info["tree_levels"],
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "path_roofline": {"t_roof_ms": t_roof * 1e3, "frac": t_roof * 1e3 / ms_step,
                          "bytes": path_bytes, "flops": fl},
        "phases_ms": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in ph.items()},
    }

    if not args.no_check and mode == "rq":
        with torch.no_grad():
            nA = torch.linalg.norm(A)
            E = torch.addmm(A, Q, R, alpha=-1.0)
            bwd = float(torch.linalg.norm(E) / nA)
            del E
            # Q^T Q as a sum over row blocks: one GEMM with k = m accumulates
            # an error near sqrt(m) eps, above the orthogonality being measured
            nb = 4096
            while m % nb:
                nb //= 2
            Qb = Q.t().reshape(n, nb, m // nb).permute(1, 0, 2).contiguous()
            G = torch.bmm(Qb, Qb.transpose(1, 2).contiguous()).sum(dim=0)
            del Qb
            orth = float(torch.linalg.norm(G - torch.eye(n, dtype=G.dtype, device=G.device)))
        result["accuracy"] = {"backward_error": bwd, "orthogonality": orth, "bound": 20 * n * 2.0 ** -53}
        log(f"accuracy {result['accuracy']}")

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on host cores)")
        result["cpu_baseline"] = cpu_baseline(A, info, args.cpu_sample_rows, mode)
    else:
        result["cpu_baseline"] = None

    plan.close()
    print(json.dumps(result), flush=True)
    return 0


def run_batched(args) -> int:
    """One step = R and explicit Q of every problem of the batch: one replay of
    the batched plan's factor graph and one of its Q graph.  The loop of single
    calls does the same problems one plan at a time.  A is regenerated before
    every step (outside the timed events: the factorisation overwrites it)."""
    import numpy as np
    import torch
    from paper_0809_2407_amd import tsqr as T

    w = BATCHED[args.workload]
    rng = np.random.default_rng(args.seed)
    ms = [int(x) for x in rng.integers(w["m_lo"], w["m_hi"] + 1, size=w["count"])]
    ns = [int(x) for x in rng.choice(w["ns"], size=w["count"])]
    fl = sum(flops_rq(m, n) for m, n in zip(ms, ns))
    entries = sum(m * n for m, n in zip(ms, ns))
    log(f"batched workload {args.workload}: {w['count']} problems, {entries * 8 / 1e9:.1f} GB per matrix set")
    g = torch.Generator(device="cuda")
    As = [T.colmajor(m, n) for m, n in zip(ms, ns)]
    Qs = [T.colmajor(m, n) for m, n in zip(ms, ns)]

    def fill(A, step, i):
        g.manual_seed((args.seed * 1000 + step) * 8192 + i)
        A.normal_(generator=g)

    def regenerate(step):
        for i, A in enumerate(As):
            fill(A, step, i)

    prec = w.get("precision", "fp64")
    mixed = prec == "mixed"
    bp = T.BatchedPlan(ms, ns, precision=prec)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]

    def batched_step():
        bp.factor(As)
        bp.form_q(As, Qs)

    for i in range(args.warmup):
        regenerate(i)
        batched_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        regenerate(100 + i)
        ev[i][0].record()
        batched_step()
        ev[i][1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b_ms = sum(a.elapsed_time(b) for a, b in ev) / args.steps
    log(f"batched: {b_ms:.3f} ms/step (events), wall {wall * 1e3 / args.steps:.1f} ms/step with regeneration")

    # accuracy on a sample of problems of the last step (against the regenerated input)
    regen_check = {}
    sample = list(range(0, w["count"], max(1, w["count"] // 16)))
    worst_b = worst_o = 0.0
    if not args.no_check:
        # the sampled problems' inputs again, into fresh buffers, for the residuals
        last = 100 + args.steps - 1
        A0 = {}
        for i in sample:
            A0[i] = torch.empty_like(As[i])
            fill(A0[i], last, i)
        regenerate(last)
        Rs = bp.factor(As)
        bp.form_q(As, Qs)
        torch.cuda.synchronize()
        for i in sample:
            A, Q, R = A0[i], Qs[i], Rs[i]
            bwd = float(torch.linalg.norm(torch.addmm(A, Q, R, alpha=-1.0)) / torch.linalg.norm(A))
            G = sum(Q[r:r + 4096].t() @ Q[r:r + 4096] for r in range(0, ms[i], 4096))  # blocked Gram
            orth = float(torch.linalg.norm(G - torch.eye(ns[i], dtype=G.dtype, device=G.device)))
            bb = 1e-6 if mixed else 20 * ns[i] * 2.0 ** -53  # the stated bounds of each path
            ob = 1e-13 if mixed else 20 * ns[i] * 2.0 ** -53
            worst_b, worst_o = max(worst_b, bwd / bb), max(worst_o, orth / ob)
        regen_check = {"sampled_problems": len(sample), "max_backward_over_bound": worst_b,
                       "max_orthogonality_over_bound": worst_o}
        log(f"accuracy {regen_check}")
        del A0

    # the loop of single calls on the same problems
    plans = [T.Plan(m, n, precision=prec) for m, n in zip(ms, ns)]

    def loop_step():
        for p, A, Q in zip(plans, As, Qs):
            p.factor(A)
            p.form_q(A, Q)

    regenerate(0)
    loop_step()
    torch.cuda.synchronize()
    lev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for i in range(args.steps):
        regenerate(100 + i)
        lev[i][0].record()
        loop_step()
        lev[i][1].record()
    torch.cuda.synchronize()
    l_ms = sum(a.elapsed_time(b) for a, b in lev) / args.steps
    log(f"loop of single calls: {l_ms:.3f} ms/step")
    for p in plans:
        p.close()

    result = {
        "metric": "TSQR R+Q GFLOP/s & % roofline; mixed/batched vs FP64 at stated backward error",
        "value": fl / (b_ms * 1e-3) / 1e9, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": b_ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "problems": w["count"], "precision": prec, "m_range": [w["m_lo"], w["m_hi"]],
                   "n_choices": list(w["ns"]), "seed": args.seed, "sum_mn": entries, "flops": fl,
                   "parallelism": "single GPU"},
        "loop_of_single_calls": {"ms_per_step": l_ms, "value": fl / (l_ms * 1e-3) / 1e9,
                                 "batched_speedup": l_ms / b_ms},
        "path_roofline": {"t_roof_ms": max(fl / (FP64_PEAK_TFLOPS * 1e12),
                                           (36.0 if mixed else 32.0) * entries / (HBM_PEAK_GBS * 1e9)) * 1e3,
                          "bytes": (36.0 if mixed else 32.0) * entries, "flops": fl},
        "accuracy": regen_check or None,
        "roofline": None,
        "cpu_baseline": None,
    }
    result["path_roofline"]["frac"] = result["path_roofline"]["t_roof_ms"] / b_ms
    bp.close()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
