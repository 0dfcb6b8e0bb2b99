#!/usr/bin/env python3
"""TSQR benchmark on one MI355X: FP64 R + explicit Q of a tall-skinny matrix.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]

One step is one pass of the whole hot path over the resident input: the leaf
chains (local Householder QRs of every tile), the binary tree over the leaf R
factors, the root sign normalisation, the top-down seed descent and the Q
expansion (tsqr_factor_into + tsqr_form_q; A is only read, so every step sees
the same input).  Prints ONE JSON line.

The default line also carries, unless --no-extras:
  accuracy.R_vs_oracle   ||R - R_oracle||_F / ||R_oracle||_F on the whole matrix
                         (the oracle of the cpu_baseline leg, signs normalised);
  mixed_vs_fp64          m = 2^24, n = 64, sigma 1 .. 1e-6: the FP64 path and
                         the mixed path on the same matrix, both times, each
                         path's accuracy against its own stated bounds and the
                         R of each against the FP64 oracle;
  krylov_mixed_vs_fp64   the s-step Krylov basis (m = 2^22, n = 17): R, Q and
                         Q^T B on 32 right-hand sides, FP64 against mixed;
  batched                2048 problems (m_i uniform on 1000..200000, n_i on
                         {8, 16, 32, 64}): one batched plan per call against the
                         loop of single calls on the same stream (FP64), and
                         the mixed batched plan on the same problems;
  beyond_tsqr            CAQR, the out-of-HBM flat tree, the competitors of
                         Sec. 5 and the paper-shaped sweep (10^5 x {50, 200,
                         400}, 10^6 x 50, 6.4e6 x 50, m n = 2^24 at n = 4 ..
                         64), three timed steps each (their full lines:
                         --workload caqr_... / stream_... / competitors_... /
                         paper_shapes_fp64).
Unless --no-peaks, every single-problem line also carries the part's measured
ceilings (measured_peaks: streaming copy and read, FP64 FMA and MFMA loops, and
a copy in the Q kernel's access pattern at the workload's geometry) and the
fractions against them (roofline.frac_of_measured_copy, q_kernel,
path_roofline.measured_peaks).  step_ms holds the median, minimum and maximum
of the timed steps (events between steps).

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
    # the mixed path with Q^T B on the 32 right-hand sides (its Q = Q1 R2^-1 has no complement:
    # only the top n rows of B are written, 8mk bytes read instead of 16mk moved)
    "tsqr_mixed_rq_qtb_krylov_m4194304_n17_k32": dict(m=2048 * 2048, n=17, decades=None, mode="rq",
                                                      krylov=(2048, 16), rhs=32, precision="mixed"),
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


# The rows beyond the TSQR path, each measured on its own line (--workload):
# CAQR of a general tall matrix with Q^T B (Sec. 6), the out-of-HBM flat tree
# over host-resident blocks (Sec. 7.1), and TSQR's competitors of Sec. 5 on
# the headline matrix and on a well-conditioned one.
NEXT_ROWS = {
    "caqr_fp64_rqtb_m131072_n256_b32_k32": dict(m=1 << 17, n=256, panel=32, rhs=32, decades=6.0),
    "stream_fp64_r_m16777216_n32_kappa1e12": dict(m=1 << 24, n=32, decades=12.0),
    "competitors_fp64_rq_m16777216_n32": dict(m=1 << 24, n=32, decades=(3.0, 12.0)),
    "paper_shapes_fp64": dict(),
}

# The shapes of the paper's experiments (context, not a target): the matrices
# of its local-QR tables (10^5 x {50, 200, 400}, 10^6 x 50, 6.4e6 x 50) and
# its out-of-DRAM sweep at m n = 2^24, n = 4 .. 64.  Widths above 64 go
# through CAQR with TSQR panels (R only).
PAPER_SHAPES = [(100_000, 50), (100_000, 200), (100_000, 400), (1_000_000, 50), (6_400_000, 50),
                (1 << 22, 4), (1 << 21, 8), (1 << 20, 16), (1 << 19, 32), (1 << 18, 64)]


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


# The files the kernels' code comes from: a byte-counter summary stays valid
# while these are unchanged and the launch geometry (leaf and tile rows) is
# the one it was taken at; host code (argument checks, plans) does not enter.
KERNEL_SOURCES = ("tsqr_kernels.h", "tsqr_internal.h", "tsqr_dispatch.hip", "tsqr_np_0.hip", "tsqr_np_1.hip",
                  "tsqr_np_2.hip", "tsqr_np_3.hip")


def sources_sha256() -> str:
    import hashlib

    h = hashlib.sha256()
    here = os.path.dirname(os.path.abspath(__file__))
    for f in KERNEL_SOURCES:
        with open(os.path.join(here, "paper_0809_2407_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(m: int, n: int, kernel: str, leaf_rows: int, tile_rows: int):
    """HBM bytes (read + write) of one launch of `kernel` from the committed
    rocprofv3 byte-counter summary under profiles/, or None when no summary
    matches this workload, its geometry and the current kernel sources."""
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
            if (d.get("workload_m") == m and d.get("workload_n") == n and d.get("sources_sha256") == sha
                    and d.get("leaf_rows") == leaf_rows and d.get("tile_rows") == tile_rows):
                k = d.get("kernels", {}).get(kernel)
                if k:
                    return k["read_bytes"] + k["write_bytes"]
    return None


def cpu_model() -> str:
    """The host CPU's model string, as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess

    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(A_dev, info: dict, sample_rows: int, mode: str, one_thread_rows: int = 1 << 20,
                 k_rhs: int = 32, seed: int = 0):
    """The oracle as it stands, on the first sample_rows rows of the same input,
    on the host cores (tree of the same shape: same leaf and tile rows), and
    on one core over the first one_thread_rows rows.  Three legs on the same
    input: the factorisation with R (R only), then the explicit Q (factor +
    form_q), then Q^T B on k_rhs host-generated columns.  Returns the record
    and the oracle's R of the sample."""
    import numpy as np

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import oracle

    m, n = A_dev.shape
    ms = min(m, sample_rows)
    As = np.asfortranarray(A_dev[:ms].cpu().numpy())
    threads = oracle.num_threads()

    def legs(X):
        rows = X.shape[0]
        t0 = time.perf_counter()
        t = oracle.TSQR(X, info["leaf_rows"], info["tile_rows"])
        R = t.R()
        t1 = time.perf_counter()
        t.form_q()
        t2 = time.perf_counter()
        B = np.asfortranarray(np.random.default_rng(seed).standard_normal((rows, k_rhs)))
        t3 = time.perf_counter()
        t.apply_qt(B)
        t4 = time.perf_counter()
        rec = {"r_only": {"gflops": flops_r(rows, n) / (t1 - t0) / 1e9, "s": t1 - t0},
               "factor_form_q": {"gflops": flops_rq(rows, n) / (t2 - t0) / 1e9, "s": t2 - t0},
               f"apply_qt_k{k_rhs}": {"gflops": 4.0 * rows * n * k_rhs / (t4 - t3) / 1e9, "s": t4 - t3}}
        return R, rec

    Ro, lg = legs(As)
    m1 = min(ms, one_thread_rows)
    oracle.set_num_threads(1)
    try:
        _, lg1 = legs(np.asfortranarray(As[:m1]))
    finally:
        oracle.set_num_threads(threads)
    key = "factor_form_q" if mode == "rq" else "r_only"
    what = "R + explicit Q" if mode == "rq" else "R only"
    rec = {"value": lg[key]["gflops"], "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"first {ms} of {m} rows (x{n}), same leaf/tile rows, {what}, {lg[key]['s']:.2f} s",
           "legs": lg,
           "one_thread": {"value": lg1[key]["gflops"], "unit": "GFLOP/s", "cores": 1,
                          "sample": f"first {m1} rows, {what}, {lg1[key]['s']:.2f} s", "legs": lg1},
           "host": {"nproc": os.cpu_count(), "model": cpu_model()}}
    return rec, Ro


def r_vs_oracle(R_dev, Ro) -> float:
    """||R - R_oracle||_F / ||R_oracle||_F; both are sign-normalised (diag >= 0)."""
    import numpy as np

    R = R_dev.cpu().numpy()
    return float(np.linalg.norm(R - Ro) / np.linalg.norm(Ro))


def fp64_bounds(n: int) -> dict:
    b = 20 * n * 2.0 ** -53
    return {"backward_error": b, "orthogonality": b, "R_vs_oracle": 1e-13}


# the mixed path's stated bounds: backward error and orthogonality after the
# second pass; its R against the FP64 oracle is reported (the FP32 first pass
# limits it to about 1e-7)
MIXED_BOUNDS = {"backward_error": 1e-6, "orthogonality": 1e-13, "R_vs_oracle": 1e-5}


def accuracy_of(A, Q, R) -> dict:
    """Backward error and orthogonality on the device, in FP64."""
    import torch

    m, n = A.shape
    with torch.no_grad():
        if m * n < 1 << 31:
            nA = torch.linalg.norm(A)
            E = torch.addmm(A, Q, R, alpha=-1.0)
            bwd = float(torch.linalg.norm(E) / nA)
            del E
        else:
            # a device GEMM on column-major views spanning more than 2^31
            # elements returned wrong products: compact row chunks instead
            e2 = a2 = 0.0
            for r in range(0, m, 1 << 22):
                Ac = A[r:r + (1 << 22)].contiguous()
                e2 += float(torch.linalg.norm(torch.addmm(Ac, Q[r:r + (1 << 22)].contiguous(), R.contiguous(),
                                                          alpha=-1.0))) ** 2
                a2 += float(torch.linalg.norm(Ac)) ** 2
            bwd = (e2 / a2) ** 0.5
        # Q^T Q as a sum over row blocks: one GEMM with k = m accumulates
        # an error near sqrt(m) eps, above the orthogonality being measured
        nb = 4096
        while m % nb:
            nb //= 2
        Qb = Q.t().reshape(n, nb, m // nb).permute(1, 0, 2).contiguous()
        G = torch.bmm(Qb, Qb.transpose(1, 2).contiguous()).sum(dim=0)
        del Qb
        orth = float(torch.linalg.norm(G - torch.eye(n, dtype=G.dtype, device=G.device)))
    return {"backward_error": bwd, "orthogonality": orth}


def oracle_r_only(A_dev, leaf_rows: int, tile_rows: int):
    """The FP64 oracle's R of the whole matrix (host cores)."""
    import numpy as np

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import oracle

    As = np.asfortranarray(A_dev.cpu().numpy())
    t0 = time.perf_counter()
    R = oracle.TSQR(As, leaf_rows, tile_rows).R()
    return R, time.perf_counter() - t0


def time_steps(step, plan, steps: int, warmup: int):
    """W untimed steps, then K timed ones bracketed by device synchronisation;
    per-phase device times from the plan's HIP events over the timed steps,
    and each step's device time from events on the plan's stream between the
    steps."""
    import torch

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    plan.profile(True)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(plan.stream)
    for i in range(steps):
        step()
        ev[i + 1].record(plan.stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ph = plan.timings()
    plan.profile(False)
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    stats = {"median": per[len(per) // 2] if len(per) % 2 else 0.5 * (per[len(per) // 2 - 1] + per[len(per) // 2]),
             "min": per[0], "max": per[-1], "timing": "HIP events on the plan's stream between steps"}
    return (t1 - t0) * 1e3 / steps, ph, stats


def phase_means(ph: dict) -> dict:
    return {k: (v[0] / v[1] if v[1] else 0.0) for k, v in ph.items()}


def run_single(args, wname: str, cpu: bool, check: bool):
    """One workload of WORKLOADS: the result record (the JSON line's fields)."""
    import torch
    from paper_0809_2407_amd import tsqr as T

    w = dict(WORKLOADS[wname])
    m, n, mode = w["m"], w["n"], w["mode"]
    log(f"workload {wname}: generating input")
    A, sig = make_input(w, args.seed)
    mixed = w.get("precision", "fp64") == "mixed"
    plan = T.Plan(m, n, precision="mixed" if mixed else "fp64", leaf_rows=w.get("leaf_rows", 0),
                  want_q=(mode == "rq"), leaf_kind=args.leaf_kind)
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
    ms_step, ph, step_stats = time_steps(step, plan, args.steps, args.warmup)
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
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": (measured_traffic(m, n, dom, info["leaf_rows"], info["tile_rows"])
                            if mode == "rq" and not mixed else None),
                "kernel": dom, "kernel_ms": dom_ms, "bytes_per_launch": phase_bytes[dom],
                "timing": "HIP events on the plan's stream around each launch of the kernel, "
                          "mean over the timed steps"}
    path_bytes = (32.0 if mode == "rq" else 8.0) * m * n + (8.0 * m * n + 16.0 * m * k_rhs if k_rhs else 0.0)
    if mixed and mode == "rq":
        path_bytes = 36.0 * m * n  # the byte model of the mixed path with its Gram pass unfused
        if k_rhs:
            path_bytes += 4.0 * m * n + 8.0 * m * k_rhs  # Q1 and B read; n rows of B written
    t_roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), path_bytes / (HBM_PEAK_GBS * 1e9))

    result = {
        "metric": "TSQR R+Q GFLOP/s & % roofline; mixed/batched vs FP64 at stated backward error",
        "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64", "data": "synthetic",
        "config": {"workload": wname, "m": m, "n": n, "mode": mode,
                   "sigma": None if sig is None else f"logspace(0,-{w['decades']:g},{n})",
                   "seed": args.seed, "tree": {1: "binary", 2: "flat", 3: "hybrid"}.get(info["tree"], "auto"),
                   "tile_rows": info["tile_rows"], "leaf_rows": info["leaf_rows"],
                   "num_leaves": info["num_leaves"], "tree_levels": info["tree_levels"],
                   "leaf_kind": info["leaf_kind"], "parallelism": "single GPU"},
        "roofline": roofline,
        "step_ms": step_stats,
        "path_roofline": {"t_roof_ms": t_roof * 1e3, "frac": t_roof * 1e3 / ms_step,
                          "frac_median": t_roof * 1e3 / step_stats["median"],
                          "frac_min": t_roof * 1e3 / step_stats["min"],
                          "bytes": path_bytes, "flops": fl},
        "phases_ms": phase_means(ph),
    }
    if check and mode == "rq":
        acc = accuracy_of(A, Q, R)
        acc["bounds"] = MIXED_BOUNDS if mixed else fp64_bounds(n)
        result["accuracy"] = acc
        log(f"accuracy {acc}")
    result["cpu_baseline"] = None
    if cpu:
        log("cpu baseline (oracle on host cores)")
        rec, Ro = cpu_baseline(A, info, args.cpu_sample_rows, mode, seed=args.seed + 2)
        result["cpu_baseline"] = rec
        if Ro.shape[0] == n and args.cpu_sample_rows >= m:
            result.setdefault("accuracy", {})["R_vs_oracle"] = r_vs_oracle(R, Ro)
            log(f"R vs oracle {result['accuracy']['R_vs_oracle']:.3e}")
    plan.close()
    del A, V, Q, R
    torch.cuda.empty_cache()
    return result


def measured_peaks(reps: int = 10, geom=None) -> dict:
    """The part's own ceilings from libtsqr_peaks: a streaming copy and a
    streaming read with 16-byte accesses over 1 GiB buffers (far beyond the
    caches), and FP64 FMA and FP64 MFMA loops; best and median of `reps`
    launches timed with HIP events on the current stream, each launch's output
    checked against its exact value.  With geom = (m, n, leaf_rows, tile_rows),
    also a copy of an m x n matrix in the access pattern of the Q kernel at that
    geometry (16mn bytes)."""
    import torch
    from paper_0809_2407_amd import peaks as PK

    st = torch.cuda.current_stream()
    nb = 1 << 30
    src = torch.empty(nb // 8, dtype=torch.float64, device="cuda").uniform_(-1.0, 1.0)
    dst = torch.empty_like(src)
    g0, g1 = PK.default_grid(1, nb), PK.default_grid(2)
    partial = torch.empty(g0, dtype=torch.float64, device="cuda")
    out = torch.empty(g1 * 256, dtype=torch.float64, device="cuda")

    def timed(fn):
        fn()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record(st)
            fn()
            b.record(st)
        torch.cuda.synchronize()
        t = sorted(a.elapsed_time(b) for a, b in ev)
        return t[0], t[len(t) // 2]

    def rate(amount, ms_pair, scale):
        return {"best": amount / (ms_pair[0] * 1e-3) / scale, "median": amount / (ms_pair[1] * 1e-3) / scale,
                "ms_best": ms_pair[0], "ms_median": ms_pair[1]}

    res = {}
    t = timed(lambda: PK.copy(src, dst))
    res["copy"] = dict(rate(2.0 * nb, t, 1e9), unit="GB/s", bytes=2 * nb, ok=bool(torch.equal(src, dst)))
    del dst
    t = timed(lambda: PK.read(src, partial))
    total = float(src.sum())
    res["read"] = dict(rate(1.0 * nb, t, 1e9), unit="GB/s", bytes=nb,
                       ok=abs(float(partial.sum()) - total) <= 1e-9 * float(src.abs().sum()))
    del src
    it_fma = 100000
    t = timed(lambda: PK.fma(out, it_fma))
    res["fp64_fma"] = dict(rate(16.0 * it_fma * g1 * 256, t, 1e12), unit="TFLOP/s", iters=it_fma,
                           ok=bool((out == 28.0 + 8.0 * it_fma).all()))
    it_mfma = 1000
    t = timed(lambda: PK.mfma(out, it_mfma))
    res["fp64_mfma"] = dict(rate(131072.0 * it_mfma * g1 * 4, t, 1e12), unit="TFLOP/s", iters=it_mfma,
                            ok=bool((out == 256.0 * it_mfma).all()))
    if geom is not None:
        from paper_0809_2407_amd import tsqr as T

        m, n, leaf_rows, tile_rows = geom
        X = T.colmajor(m, n)
        X.copy_(torch.rand((n, m), device="cuda", dtype=torch.float64).t())
        Y = T.colmajor(m, n)
        t = timed(lambda: PK.copy_leaf(X, Y, leaf_rows, tile_rows))
        res["copy_in_q_pattern"] = dict(rate(16.0 * m * n, t, 1e9), unit="GB/s", bytes=16 * m * n,
                                        m=m, n=n, leaf_rows=leaf_rows, tile_rows=tile_rows,
                                        ok=bool(torch.equal(X, Y)))
        del X, Y
    res["grids"] = {"copy": PK.default_grid(0, nb), "read": g0, "loops": g1, "block": 256}
    res["datasheet"] = {"hbm_GBps": HBM_PEAK_GBS, "fp64_TFLOPs": FP64_PEAK_TFLOPS}
    del partial, out
    torch.cuda.empty_cache()
    return res


def against_measured(result: dict, pk: dict) -> None:
    """Roofline fractions against the measured ceilings (copy rate for bytes,
    the faster FP64 loop for flops), beside the datasheet ones."""
    if not (pk["copy"]["ok"] and pk["fp64_mfma"]["ok"] and pk["fp64_fma"]["ok"]):
        return
    bw = pk["copy"]["best"]
    fl_rate = max(pk["fp64_mfma"]["best"], pk["fp64_fma"]["best"]) * 1e12
    rf = result.get("roofline")
    if rf and rf.get("unit") == "GB/s":
        rf["frac_of_measured_copy"] = rf["achieved"] / bw
    cq = pk.get("copy_in_q_pattern")
    ph = result.get("phases_ms", {})
    cfg = result.get("config", {})
    if cq and cq["ok"] and ph.get("form_q") and result.get("dtype") == "f64" and cfg.get("mode") == "rq":
        q_rate = 16.0 * cfg["m"] * cfg["n"] / (ph["form_q"] * 1e-3) / 1e9
        result["q_kernel"] = {"ms": ph["form_q"], "GBps": q_rate, "bytes": 16.0 * cfg["m"] * cfg["n"],
                              "frac_of_copy_in_its_pattern": q_rate / cq["best"],
                              "frac_of_measured_copy": q_rate / bw}
    pr = result.get("path_roofline")
    if pr and "flops" in pr:
        t = max(pr["flops"] / fl_rate, pr["bytes"] / (bw * 1e9)) * 1e3
        pr["measured_peaks"] = {"t_roof_ms": t, "frac": t / result["ms_per_step"],
                                "frac_median": t / result["step_ms"]["median"] if "step_ms" in result else None}


def mixed_vs_fp64(args, steps: int, warmup: int) -> dict:
    """The FP64 path and the mixed path (FP32 first pass, FP64 second pass) on
    the same m = 2^24, n = 64 matrix (sigma 1 .. 1e-6): both times, each path's
    accuracy against its stated bounds and R against the FP64 oracle."""
    import torch
    from paper_0809_2407_amd import tsqr as T

    m, n, dec = 1 << 24, 64, 6.0
    log(f"mixed vs FP64: m = {m}, n = {n}, generating input")
    A, _ = make_input(dict(m=m, n=n, decades=dec), args.seed)
    Q = T.colmajor(m, n)
    out = {"workload": f"tsqr_rq_m{m}_n{n}_kappa1e6", "m": m, "n": n, "sigma": f"logspace(0,-{dec:g},{n})",
           "seed": args.seed, "steps": steps, "warmup": warmup, "flops_credited": flops_rq(m, n)}
    Rs = {}
    fp64_geom = None
    for prec in ("fp64", "mixed"):
        plan = T.Plan(m, n, precision=prec)
        info = plan.info()
        V = T.colmajor(m, n) if prec == "fp64" else None
        R = T.colmajor(n, n)

        def step():
            plan.factor_into(A, V, R)
            plan.form_q(V, Q)

        ms_step, ph, step_stats = time_steps(step, plan, steps, warmup)
        acc = accuracy_of(A, Q, R)
        rec = {"ms_per_step": ms_step, "step_ms": step_stats,
               "value": flops_rq(m, n) / (ms_step * 1e-3) / 1e9, "unit": "GFLOP/s",
               "phases_ms": phase_means(ph), "accuracy": acc,
               "bounds": MIXED_BOUNDS if prec == "mixed" else fp64_bounds(n),
               "leaf_rows": info["leaf_rows"], "tile_rows": info["tile_rows"]}
        if prec == "mixed":
            i2 = plan.info()
            rec["second_pass"] = {"orth_estimate": i2["orth_estimate"], "applied": bool(i2["reorth_applied"])}
        log(f"{prec}: {ms_step:.3f} ms/step, accuracy {acc}")
        out[prec] = rec
        Rs[prec] = R
        if prec == "fp64":
            fp64_geom = (info["leaf_rows"], info["tile_rows"])
        plan.close()
        del V
    if args.no_cpu_baseline:
        out["oracle"] = None
    else:
        log("mixed vs FP64: the FP64 oracle's R of the whole matrix (host cores)")
        Ro, dt = oracle_r_only(A, *fp64_geom)
        for prec in ("fp64", "mixed"):
            out[prec]["accuracy"]["R_vs_oracle"] = r_vs_oracle(Rs[prec], Ro)
        out["oracle"] = {"seconds": dt, "what": "R of the whole matrix, FP64 oracle (same leaf and tile rows "
                                                "as the FP64 plan)"}
    out["mixed_speedup"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    for prec in ("fp64", "mixed"):
        a, b = out[prec]["accuracy"], out[prec]["bounds"]
        out[prec]["within_bounds"] = all(a[k] <= b[k] for k in b if k in a)
    del A, Q, Rs
    torch.cuda.empty_cache()
    return out


def krylov_mixed_vs_fp64(args, steps: int, warmup: int) -> dict:
    """The s-step Krylov basis (2-D Laplacian on a 2048 x 2048 grid, n = 17):
    R, the explicit Q and Q^T B on 32 right-hand sides, FP64 path against the
    mixed path, each with its accuracy against its stated bounds and the top n
    rows of Q^T B against Q^T B formed from the plan's own explicit Q."""
    import torch
    from paper_0809_2407_amd import tsqr as T

    w = dict(WORKLOADS["tsqr_fp64_rq_qtb_krylov_m4194304_n17_k32"])
    m, n, k = w["m"], w["n"], w["rhs"]
    log(f"Krylov mixed vs FP64: m = {m}, n = {n}, {k} right-hand sides, generating input")
    A, _ = make_input(w, args.seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed + 1)
    B0 = torch.randn((k, m), generator=g, device="cuda", dtype=torch.float64).t()
    B = T.colmajor(m, k)
    Q = T.colmajor(m, n)
    fl = flops_rq(m, n) + 4.0 * m * n * k
    out = {"workload": "krylov_rq_qtb_m4194304_n17_k32", "m": m, "n": n, "rhs": k, "seed": args.seed,
           "steps": steps, "warmup": warmup, "flops_credited": fl,
           "note": "FP64 Q^T B transforms all m rows (the tree's full orthogonal factor); the mixed Q = Q1 R2^-1 "
                   "has no complement, so only its top n rows are written"}
    for prec in ("fp64", "mixed"):
        plan = T.Plan(m, n, precision=prec)
        V = T.colmajor(m, n) if prec == "fp64" else None
        R = T.colmajor(n, n)

        def step():
            plan.factor_into(A, V, R)
            plan.form_q(V, Q)
            B.copy_(B0)
            plan.apply_qt(V, B)

        ms_step, ph, step_stats = time_steps(step, plan, steps, warmup)
        acc = accuracy_of(A, Q, R)
        with torch.no_grad():
            acc["qtb_vs_explicit_q"] = float((B[:n] - Q.t().matmul(B0)).abs().max() / torch.linalg.norm(B0))
        rec = {"ms_per_step": ms_step, "step_ms": step_stats, "value": fl / (ms_step * 1e-3) / 1e9,
               "unit": "GFLOP/s", "phases_ms": phase_means(ph), "accuracy": acc,
               "bounds": MIXED_BOUNDS if prec == "mixed" else fp64_bounds(n)}
        log(f"Krylov {prec}: {ms_step:.3f} ms/step, accuracy {acc}")
        out[prec] = rec
        plan.close()
        del V, R
    out["mixed_speedup"] = out["fp64"]["ms_per_step"] / out["mixed"]["ms_per_step"]
    for prec in ("fp64", "mixed"):
        a, b = out[prec]["accuracy"], out[prec]["bounds"]
        out[prec]["within_bounds"] = all(a[kk] <= b[kk] for kk in b if kk in a)
    del A, B, B0, Q
    torch.cuda.empty_cache()
    return out


def batched_record(args, count: int, m_lo: int, m_hi: int, ns, precision: str, steps: int, warmup: int,
                   loop_steps: int, sample_oracle: bool, state=None) -> dict:
    """One batched plan (captured graph) over `count` problems, R and explicit
    Q per step, against a loop of single calls on the same stream (loop_steps
    > 0).  A is regenerated before every step, outside the timed events (the
    factorisation overwrites it).  `state` carries the problems' buffers from
    one call to the next (same problems, another precision)."""
    import numpy as np
    import torch
    from paper_0809_2407_amd import tsqr as T

    if state is None:
        rng = np.random.default_rng(args.seed)
        ms = [int(x) for x in rng.integers(m_lo, m_hi + 1, size=count)]
        nn = [int(x) for x in rng.choice(ns, size=count)]
        state = {"ms": ms, "ns": nn, "As": [T.colmajor(m, n) for m, n in zip(ms, nn)],
                 "Qs": [T.colmajor(m, n) for m, n in zip(ms, nn)], "g": torch.Generator(device="cuda")}
    ms, nn, As, Qs, g = state["ms"], state["ns"], state["As"], state["Qs"], state["g"]
    fl = sum(flops_rq(m, n) for m, n in zip(ms, nn))
    entries = sum(m * n for m, n in zip(ms, nn))
    mixed = precision == "mixed"
    log(f"batched {precision}: {count} problems, {entries * 8 / 1e9:.1f} GB per matrix set")

    def fill(A, step, i):
        g.manual_seed((args.seed * 1000 + step) * 8192 + i)
        A.normal_(generator=g)

    def regenerate(step):
        for i, A in enumerate(As):
            fill(A, step, i)

    bp = T.BatchedPlan(ms, nn, precision=precision)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]

    def batched_step():
        bp.factor(As)
        bp.form_q(As, Qs)

    for i in range(warmup):
        regenerate(i)
        batched_step()
    torch.cuda.synchronize()
    for i in range(steps):
        regenerate(100 + i)
        ev[i][0].record()
        batched_step()
        ev[i][1].record()
    torch.cuda.synchronize()
    b_ms = sum(a.elapsed_time(b) for a, b in ev) / steps
    log(f"batched {precision}: {b_ms:.3f} ms/step (events)")

    # accuracy on a sample of problems: regenerate the last step's input, keep
    # copies of the sampled ones, factor again and check the residuals
    sample = list(range(0, count, max(1, count // 16)))
    last = 100 + steps - 1
    A0 = {}
    for i in sample:
        A0[i] = torch.empty_like(As[i])
        fill(A0[i], last, i)
    regenerate(last)
    Rs = bp.factor(As)
    bp.form_q(As, Qs)
    torch.cuda.synchronize()
    worst = {"backward_error": 0.0, "orthogonality": 0.0, "R_vs_oracle": 0.0}
    for i in sample:
        A, Q, R = A0[i], Qs[i], Rs[i]
        bwd = float(torch.linalg.norm(torch.addmm(A, Q, R, alpha=-1.0)) / torch.linalg.norm(A))
        G = sum(Q[r:r + 4096].t() @ Q[r:r + 4096] for r in range(0, ms[i], 4096))  # blocked Gram
        orth = float(torch.linalg.norm(G - torch.eye(nn[i], dtype=G.dtype, device=G.device)))
        b = MIXED_BOUNDS if mixed else fp64_bounds(nn[i])
        worst["backward_error"] = max(worst["backward_error"], bwd / b["backward_error"])
        worst["orthogonality"] = max(worst["orthogonality"], orth / b["orthogonality"])
        if sample_oracle:
            sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
            import oracle

            Ro = oracle.qr_reference(np.asfortranarray(A.cpu().numpy()), want_q=False)
            worst["R_vs_oracle"] = max(worst["R_vs_oracle"], r_vs_oracle(R, Ro) / b["R_vs_oracle"])
    del A0, Rs
    acc = {"sampled_problems": len(sample), "max_over_bound": worst,
           "bounds": MIXED_BOUNDS if mixed else {"backward_error": "20 n 2^-53", "orthogonality": "20 n 2^-53",
                                                 "R_vs_oracle": 1e-13}}
    log(f"batched {precision} accuracy {acc}")
    bp.close()

    rec = {"problems": count, "precision": precision, "m_range": [m_lo, m_hi], "n_choices": list(ns),
           "seed": args.seed, "sum_mn": entries, "flops": fl, "steps": steps, "warmup": warmup,
           "ms_per_step": b_ms, "value": fl / (b_ms * 1e-3) / 1e9, "unit": "GFLOP/s", "accuracy": acc}
    bytes_ = (36.0 if mixed else 32.0) * entries
    t_roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), bytes_ / (HBM_PEAK_GBS * 1e9))
    rec["path_roofline"] = {"t_roof_ms": t_roof * 1e3, "frac": t_roof * 1e3 / b_ms, "bytes": bytes_, "flops": fl}

    if loop_steps > 0:
        plans = [T.Plan(m, n, precision=precision) for m, n in zip(ms, nn)]

        def loop_step():
            for p, A, Q in zip(plans, As, Qs):
                p.factor(A)
                p.form_q(A, Q)

        regenerate(0)
        loop_step()
        torch.cuda.synchronize()
        lev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(loop_steps)]
        for i in range(loop_steps):
            regenerate(100 + i)
            lev[i][0].record()
            loop_step()
            lev[i][1].record()
        torch.cuda.synchronize()
        l_ms = sum(a.elapsed_time(b) for a, b in lev) / loop_steps
        log(f"loop of single {precision} calls: {l_ms:.3f} ms/step")
        for p in plans:
            p.close()
        del plans
        rec["loop_of_single_calls"] = {"ms_per_step": l_ms, "value": fl / (l_ms * 1e-3) / 1e9,
                                       "steps": loop_steps, "batched_speedup": l_ms / b_ms}
    torch.cuda.empty_cache()
    return rec, state


def events_time(work, steps: int, warmup: int, prepare=None):
    """Per-step device times (ms) of work() from events on the current stream;
    prepare() runs before each step outside the events."""
    import torch

    st = torch.cuda.current_stream()
    for _ in range(warmup):
        if prepare:
            prepare()
        work()
    torch.cuda.synchronize()
    ev = []
    for _ in range(steps):
        if prepare:
            prepare()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        work()
        b.record(st)
        ev.append((a, b))
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in ev)
    return {"mean": sum(t) / len(t), "median": t[len(t) // 2] if len(t) % 2 else 0.5 * (t[len(t) // 2 - 1] + t[len(t) // 2]),
            "min": t[0], "max": t[-1], "timing": "HIP events on the stream around each step"}


def line(metric: str, value: float, unit: str, steps: int, warmup: int, ms: float, dtype: str, config: dict) -> dict:
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
            "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
            "data": "synthetic", "config": config}


def caqr_line(args, name: str) -> dict:
    """CAQR (Sec. 6) of a tall general matrix with TSQR panels and Q^T B on k
    columns carried along (tsqr_caqr_factor_rhs on [A B]): per panel the
    panel's TSQR and one tree-structured update of the trailing columns and B
    together.  R against the oracle's plain Householder R of the whole matrix,
    Q^T B through the column norms it must keep.  The same results from
    tsqr_caqr_factor then tsqr_caqr_apply_qt (B in passes of its own) are
    timed beside it."""
    import numpy as np
    import torch
    from paper_0809_2407_amd import tsqr as T

    w = NEXT_ROWS[name]
    m, n, b, k = w["m"], w["n"], w["panel"], w["rhs"]
    log(f"CAQR m = {m}, n = {n}, panel {b}, {k} right-hand sides: generating input")
    A0, _ = make_input(dict(m=m, n=n, decades=w["decades"]), args.seed)
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed + 1)
    B0 = torch.randn((k, m), generator=g, device="cuda", dtype=torch.float64).t()
    AB, R = T.colmajor(m, n + k), T.colmajor(n, n)
    B = AB[:, n:]
    plan = T.CaqrPlan(m, n, b)
    info = plan.info()

    def prepare():
        AB[:, :n].copy_(A0)
        B.copy_(B0)

    t = events_time(lambda: plan.factor_rhs(AB, R), args.steps, args.warmup, prepare)
    t2 = same = None
    if not args.no_extras:
        # the same results with B in passes of its own
        A2, B2, R2 = T.colmajor(m, n), T.colmajor(m, k), T.colmajor(n, n)

        def prepare2():
            A2.copy_(A0)
            B2.copy_(B0)

        def separate():
            plan.factor(A2, R2)
            plan.apply_qt(A2, B2)

        t2 = events_time(separate, args.steps, args.warmup, prepare2)
        same = bool(torch.equal(R, R2) and torch.equal(B, B2))
        del A2, B2, R2
    fl = flops_r(m, n) + 4.0 * m * n * k - 2.0 * n * n * k
    by = 0.0
    for j in range(info["num_panels"]):
        mj, bj = m - j * b, min(b, n - j * b)
        cj = n - j * b - bj
        by += 16.0 * mj * bj + -(-(cj + k) // 32) * 8.0 * mj * bj + 16.0 * mj * (cj + k)
    t_roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), by / (HBM_PEAK_GBS * 1e9)) * 1e3
    with torch.no_grad():
        keep = float(((torch.linalg.norm(B, dim=0) - torch.linalg.norm(B0, dim=0)).abs()
                      / torch.linalg.norm(B0, dim=0)).max())
    res = line("CAQR R + Q^T B GFLOP/s & % roofline", fl / (t["median"] * 1e-3) / 1e9, "GFLOP/s", args.steps,
               args.warmup, t["mean"], "f64",
               {"workload": name, "m": m, "n": n, "panel": b, "num_panels": info["num_panels"], "rhs": k,
                "sigma": f"logspace(0,-{w['decades']:g},{n})", "seed": args.seed, "parallelism": "single GPU"})
    res["step_ms"] = t
    res["separate_rhs_passes"] = None if t2 is None else {
        "step_ms": t2, "speedup_median": t2["median"] / t["median"], "same_R_and_QtB_bitwise": same}
    res["roofline"] = None
    res["path_roofline"] = {"t_roof_ms": t_roof, "frac_median": t_roof / t["median"], "bytes": by, "flops": fl,
                            "bytes_model": "per panel: 16 m_j b (panel TSQR), 8 m_j b per 32 trailing and B "
                                           "columns (reflectors re-read) + 16 m_j per trailing or B column"}
    res["accuracy"] = {"qtb_column_norms_kept": keep}
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import oracle

        log("CAQR: the oracle's plain Householder R of the whole matrix (one thread)")
        Ah = np.asfortranarray(A0.cpu().numpy())
        t0 = time.perf_counter()
        Ro = oracle.qr_reference(Ah, want_q=False)
        dt = time.perf_counter() - t0
        res["accuracy"]["R_vs_oracle"] = r_vs_oracle(R, Ro)
        res["cpu_baseline"] = {"value": flops_r(m, n) / dt / 1e9, "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
                               "sample": f"plain Householder R of the whole {m} x {n} matrix, {dt:.2f} s",
                               "host": {"nproc": os.cpu_count(), "model": cpu_model()}}
    sep = f" ({t2['median']:.3f} with B in passes of its own)" if t2 else ""
    log(f"CAQR: {t['median']:.3f} ms median{sep}, accuracy {res['accuracy']}")
    plan.close()
    return res


def paper_shapes_line(args, name: str) -> dict:
    """The paper-shaped sweep: iid N(0,1) entries (the paper states no
    distribution), per shape R only and R + explicit Q (TSQR, n <= 64) or R
    (CAQR, panels of 32, wider), each against its path roofline (bytes 8mn for
    R, 32mn for R + Q; CAQR as in its own line), with the backward error and
    orthogonality of R + Q and ||R^T R - A^T A|| / ||A||^2 of the CAQR R."""
    import torch
    from paper_0809_2407_amd import tsqr as T

    recs = []
    for m, n in PAPER_SHAPES:
        g = torch.Generator(device="cuda")
        g.manual_seed(args.seed + m + n)
        A = torch.randn((n, m), generator=g, device="cuda", dtype=torch.float64).t()
        log(f"paper shapes: {m} x {n}")
        if n > 64:
            b = 32
            plan = T.CaqrPlan(m, n, b)
            W, R = T.colmajor(m, n), T.colmajor(n, n)
            t = events_time(lambda: plan.factor(W, R), args.steps, args.warmup, lambda: W.copy_(A))
            plan.close()
            fl = flops_r(m, n)
            by = 0.0
            for j in range(-(-n // b)):
                mj, bj = m - j * b, min(b, n - j * b)
                cj = n - j * b - bj
                by += 16.0 * mj * bj + -(-cj // 32) * 8.0 * mj * bj + 16.0 * mj * cj
            with torch.no_grad():
                gram = float(torch.linalg.norm(R.t().matmul(R) - A.t().matmul(A)) / torch.linalg.norm(A) ** 2)
            roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), by / (HBM_PEAK_GBS * 1e9)) * 1e3
            recs.append({"m": m, "n": n, "method": "caqr", "mode": "r", "ms_median": t["median"], "ms_min": t["min"],
                         "gflops": fl / (t["median"] * 1e-3) / 1e9, "bytes": by,
                         "path_roofline_frac": roof / t["median"], "gram_error": gram})
            del W, R, A
            continue
        with T.Plan(m, n, want_q=False) as p:
            R = T.colmajor(n, n)
            t = events_time(lambda: p.factor(A, R), args.steps, args.warmup)
        fl, by = flops_r(m, n), 8.0 * m * n
        roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), by / (HBM_PEAK_GBS * 1e9)) * 1e3
        recs.append({"m": m, "n": n, "method": "tsqr", "mode": "r", "ms_median": t["median"], "ms_min": t["min"],
                     "gflops": fl / (t["median"] * 1e-3) / 1e9, "bytes": by, "path_roofline_frac": roof / t["median"]})
        with T.Plan(m, n) as p:
            V, R, Q = T.colmajor(m, n), T.colmajor(n, n), T.colmajor(m, n)

            def rq():
                p.factor_into(A, V, R)
                p.form_q(V, Q)

            t = events_time(rq, args.steps, args.warmup)
            info = p.info()
        acc = accuracy_of(A, Q, R)  # Q^T Q summed over row blocks
        bwd, orth = acc["backward_error"], acc["orthogonality"]
        fl, by = flops_rq(m, n), 32.0 * m * n
        roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), by / (HBM_PEAK_GBS * 1e9)) * 1e3
        recs.append({"m": m, "n": n, "method": "tsqr", "mode": "rq", "ms_median": t["median"], "ms_min": t["min"],
                     "gflops": fl / (t["median"] * 1e-3) / 1e9, "bytes": by, "path_roofline_frac": roof / t["median"],
                     "backward_error": bwd, "orthogonality": orth, "leaf_rows": info["leaf_rows"],
                     "tile_rows": info["tile_rows"], "num_leaves": info["num_leaves"]})
        del V, R, Q, A
    torch.cuda.empty_cache()
    for r in recs:
        log(f"  {r['method']} {r['mode']} {r['m']} x {r['n']}: {r['ms_median']:.3f} ms, {r['gflops']:.0f} GFLOP/s, "
            f"{100 * r['path_roofline_frac']:.1f}% of its path roofline")
    return {"metric": "paper-shaped TSQR / CAQR GFLOP/s & % path roofline (context)", "workload": name,
            "steps": args.steps, "warmup": args.warmup, "dtype": "f64",
            "data": f"synthetic: iid N(0,1), torch generator on the device, seed {args.seed} + m + n",
            "records": recs}


def stream_line(args, name: str) -> dict:
    """The out-of-HBM flat tree (Sec. 7.1): A in pinned host memory, streamed
    to the GPU in row blocks while the previous block is factored.  Bound by
    the host link: the line reports the rate against a measured pinned
    host-to-device copy."""
    import numpy as np
    import torch
    from paper_0809_2407_amd import tsqr as T

    w = NEXT_ROWS[name]
    m, n = w["m"], w["n"]
    log(f"out-of-HBM m = {m}, n = {n}: generating input")
    A, _ = make_input(dict(m=m, n=n, decades=w["decades"]), args.seed)
    H = torch.empty((n, m), dtype=torch.float64, pin_memory=True).t()
    H.copy_(A)
    plan = T.StreamPlan(m, n)
    info = plan.info()
    R = T.colmajor(n, n)
    t = events_time(lambda: plan.factor(H, R), args.steps, args.warmup)
    by = 8.0 * m * n
    # the link's ceiling: a pinned host-to-device copy of 1 GiB
    nb = 1 << 30
    hsrc = torch.empty(nb // 8, dtype=torch.float64, pin_memory=True)
    dd = torch.empty(nb // 8, dtype=torch.float64, device="cuda")
    tc = events_time(lambda: dd.copy_(hsrc, non_blocking=True), 5, 1)
    h2d = nb / (tc["min"] * 1e-3) / 1e9
    del hsrc, dd
    with T.Plan(m, n, want_q=False) as p:
        Rh = p.factor(A)
    rate = by / (t["median"] * 1e-3) / 1e9
    res = line("out-of-HBM TSQR R: host GB/s streamed & % of the measured host link", rate, "GB/s", args.steps,
               args.warmup, t["mean"], "f64",
               {"workload": name, "m": m, "n": n, "block_rows": info["block_rows"], "num_blocks": info["num_blocks"],
                "sigma": f"logspace(0,-{w['decades']:g},{n})", "seed": args.seed, "host_memory": "pinned",
                "parallelism": "single GPU"})
    res["step_ms"] = t
    res["gflops"] = flops_r(m, n) / (t["median"] * 1e-3) / 1e9
    res["roofline"] = {"bound": "host link", "achieved": rate, "peak": h2d, "unit": "GB/s", "frac": rate / h2d,
                       "peak_source": "pinned host-to-device copy of 1 GiB, measured in the same run",
                       "traffic": None}
    res["accuracy"] = {"R_vs_in_hbm_tsqr": r_vs_oracle(R, Rh.cpu().numpy())}
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        log("out-of-HBM: the oracle's TSQR R of the whole matrix (host cores)")
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import oracle

        pi = T.plan_query(m, n, want_q=False)
        Ro, dt = oracle_r_only(A, pi["leaf_rows"], pi["tile_rows"])
        res["accuracy"]["R_vs_oracle"] = r_vs_oracle(R, Ro)
        res["cpu_baseline"] = {"value": flops_r(m, n) / dt / 1e9, "unit": "GFLOP/s", "cores": oracle.num_threads(),
                               "kind": "oracle", "sample": f"TSQR R of the whole matrix (in host memory), {dt:.2f} s",
                               "host": {"nproc": os.cpu_count(), "model": cpu_model()}}
    log(f"out-of-HBM: {t['median']:.2f} ms median, {rate:.1f} GB/s of {h2d:.1f}, accuracy {res['accuracy']}")
    plan.close()
    del H
    return res


CMP_FLOPS = {  # nominal flops of each method for R and Q (m x n): half of Householder's 4mn^2
    "cholqr": lambda m, n: 2.0 * m * n * n,        # Gram (symmetric) mn^2, Q = A R^-1 (triangular) mn^2
    "cholqr2": lambda m, n: 4.0 * m * n * n,
    "cgs": lambda m, n: 2.0 * m * n * n,
    "mgs": lambda m, n: 2.0 * m * n * n,
}
CMP_BYTES = {  # algorithmic HBM bytes: CholeskyQR reads A twice and writes Q; Gram-Schmidt passes over the columns
    "cholqr": lambda m, n: 24.0 * m * n,
    "cholqr2": lambda m, n: 48.0 * m * n,
    "cgs": lambda m, n: 8.0 * m * n * n,
    "mgs": lambda m, n: 8.0 * m * n * n,
}


def competitors_line(args, name: str) -> dict:
    """TSQR's competitors of Sec. 5 (CholeskyQR, CholeskyQR2, CGS, MGS) beside
    TSQR on the same matrices: a well-conditioned one (kappa = 1e3) and the
    headline one (kappa = 1e12), with times, roofline fractions, backward error,
    orthogonality and breakdowns (the stability contrast of Sec. 5)."""
    import numpy as np
    import torch
    from paper_0809_2407_amd import tsqr as T

    w = NEXT_ROWS[name]
    m, n = w["m"], w["n"]
    out = {}
    for dec in w["decades"]:
        key = f"kappa1e{int(dec)}"
        log(f"competitors m = {m}, n = {n}, kappa = 1e{int(dec)}: generating input")
        A, _ = make_input(dict(m=m, n=n, decades=dec), args.seed)
        Q, R = T.colmajor(m, n), T.colmajor(n, n)
        rec = {}
        with T.Plan(m, n) as p:
            V = T.colmajor(m, n)

            def tsqr_step():
                p.factor_into(A, V, R)
                p.form_q(V, Q)

            t = events_time(tsqr_step, args.steps, args.warmup)
            fl = flops_rq(m, n)
            t_roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), 32.0 * m * n / (HBM_PEAK_GBS * 1e9)) * 1e3
            rec["tsqr"] = {"ms_median": t["median"], "gflops": fl / (t["median"] * 1e-3) / 1e9,
                           "path_roofline_frac": t_roof / t["median"], "breakdown": 0, **accuracy_of(A, Q, R)}
            del V
        for meth in ("cholqr", "cholqr2", "cgs", "mgs"):
            with T.CmpPlan(m, n, meth) as p:
                t = events_time(lambda: p.factor(A, Q, R), args.steps, args.warmup)
                bd = p.breakdown()
            fl, by = CMP_FLOPS[meth](m, n), CMP_BYTES[meth](m, n)
            t_roof = max(fl / (FP64_PEAK_TFLOPS * 1e12), by / (HBM_PEAK_GBS * 1e9)) * 1e3
            r = {"ms_median": t["median"], "gflops": fl / (t["median"] * 1e-3) / 1e9,
                 "path_roofline_frac": t_roof / t["median"], "bytes": by, "breakdown": bd}
            if bd == 0:
                r.update(accuracy_of(A, Q, R))
            rec[meth] = r
            log(f"  {key} {meth}: {r}")
        out[key] = rec
        del A, Q, R
        torch.cuda.empty_cache()
    tk = out["kappa1e3"]["tsqr"]["ms_median"]
    res = line("TSQR against its competitors of Sec. 5: ms per R + Q, orthogonality", out["kappa1e3"]["tsqr"]["gflops"],
               "GFLOP/s", args.steps, args.warmup, tk, "f64",
               {"workload": name, "m": m, "n": n, "sigmas": [f"logspace(0,-{d:g},{n})" for d in w["decades"]],
                "seed": args.seed, "parallelism": "single GPU"})
    res["methods"] = out
    res["roofline"] = None
    res["cpu_baseline"] = None
    if not args.no_cpu_baseline:
        sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
        import oracle

        ms_ = 1 << 18
        As, _ = make_input(dict(m=ms_, n=n, decades=w["decades"][0]), args.seed)
        Ah = np.asfortranarray(As.cpu().numpy())
        legs = {}
        for meth, fn in (("cholqr", oracle.cholqr), ("cholqr2", oracle.cholqr2), ("cgs", oracle.cgs),
                         ("mgs", oracle.mgs)):
            t0 = time.perf_counter()
            fn(Ah)
            dt = time.perf_counter() - t0
            legs[meth] = {"gflops": CMP_FLOPS[meth](ms_, n) / dt / 1e9, "s": dt}
        res["cpu_baseline"] = {"value": legs["cholqr"]["gflops"], "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
                               "sample": f"{ms_} x {n}, kappa = 1e{int(w['decades'][0])}, each method once",
                               "legs": legs, "host": {"nproc": os.cpu_count(), "model": cpu_model()}}
    return res


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) + sorted(BATCHED) + sorted(NEXT_ROWS))
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=1 << 24)
    ap.add_argument("--no-check", action="store_true", help="skip the accuracy check after timing")
    ap.add_argument("--no-peaks", action="store_true",
                    help="skip measuring the part's copy, read, FMA and MFMA ceilings")
    ap.add_argument("--no-extras", action="store_true",
                    help="the default workload only (no mixed-vs-FP64, batched or beyond-TSQR records); "
                         "CAQR without the timing of B in passes of its own")
    ap.add_argument("--leaf-kind", default="auto", choices=["auto", "compact_wy", "recursive"],
                    help="local QR of the leaf tiles (single-problem workloads)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="before warm-up, run one plain device copy of m x n doubles (8mn bytes read, "
                         "8mn written) so that hardware byte counters can be scaled against it")
    args = ap.parse_args(argv)

    if args.steps < 1 or args.warmup < 0:
        print(json.dumps({"error": "--steps must be at least 1 and --warmup at least 0"}))
        return 2
    if args.gpus != 1:
        print(json.dumps({"error": "this TSQR build runs on one GPU; the multi-GPU path (one all-gather "
                                   "of the R factors) is a design, not a build: use --gpus 1"}))
        return 2

    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        return 1
    if args.workload in BATCHED:
        return run_batched(args)
    if args.workload in NEXT_ROWS:
        fn = {"caqr": caqr_line, "stream": stream_line, "competitors": competitors_line,
              "paper": paper_shapes_line}[args.workload.split("_")[0]]
        print(json.dumps(fn(args, args.workload)), flush=True)
        return 0
    result = run_single(args, args.workload, cpu=not args.no_cpu_baseline, check=not args.no_check)
    if not args.no_peaks:
        log("measured ceilings: copy, read, FP64 FMA and MFMA loops")
        c = result["config"]
        geom = (c["m"], c["n"], c["leaf_rows"], c["tile_rows"]) if c.get("mode") == "rq" else None
        pk = measured_peaks(geom=geom)
        log(f"measured ceilings {pk}")
        result["measured_peaks"] = pk
        against_measured(result, pk)
    if args.workload == DEFAULT and not args.no_extras:
        result["mixed_vs_fp64"] = mixed_vs_fp64(args, steps=min(args.steps, 10), warmup=2)
        result["krylov_mixed_vs_fp64"] = krylov_mixed_vs_fp64(args, steps=min(args.steps, 10), warmup=2)
        w = BATCHED["tsqr_batched_fp64_rq_p2048_m1000_200000_n8_64"]
        fp64, state = batched_record(args, w["count"], w["m_lo"], w["m_hi"], w["ns"], "fp64", steps=3, warmup=1,
                                     loop_steps=2, sample_oracle=not args.no_cpu_baseline)
        mx, state = batched_record(args, w["count"], w["m_lo"], w["m_hi"], w["ns"], "mixed", steps=3, warmup=1,
                                   loop_steps=0, sample_oracle=not args.no_cpu_baseline, state=state)
        del state
        result["batched"] = {"workload": "tsqr_batched_rq_p2048_m1000_200000_n8_64", "fp64": fp64, "mixed": mx,
                             "mixed_vs_fp64_batched": fp64["ms_per_step"] / mx["ms_per_step"]}
        # the rows beyond the TSQR path, three timed steps each (their own lines: --workload NAME)
        short = argparse.Namespace(**vars(args))
        short.steps, short.warmup = 3, 1
        result["beyond_tsqr"] = {name.split("_")[0]: fn(short, name) for name, fn in (
            ("caqr_fp64_rqtb_m131072_n256_b32_k32", caqr_line),
            ("stream_fp64_r_m16777216_n32_kappa1e12", stream_line),
            ("competitors_fp64_rq_m16777216_n32", competitors_line),
            ("paper_shapes_fp64", paper_shapes_line))}
    print(json.dumps(result), flush=True)
    return 0


def run_batched(args) -> int:
    """A batched workload alone: its record as the JSON line."""
    w = BATCHED[args.workload]
    prec = w.get("precision", "fp64")
    rec, _ = batched_record(args, w["count"], w["m_lo"], w["m_hi"], w["ns"], prec, steps=args.steps,
                            warmup=args.warmup, loop_steps=args.steps, sample_oracle=not args.no_cpu_baseline)
    result = {
        "metric": "TSQR R+Q GFLOP/s & % roofline; mixed/batched vs FP64 at stated backward error",
        "value": rec["value"], "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64" if prec == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": args.workload, "problems": w["count"], "precision": prec,
                   "m_range": [w["m_lo"], w["m_hi"]], "n_choices": list(w["ns"]), "seed": args.seed,
                   "sum_mn": rec["sum_mn"], "flops": rec["flops"], "parallelism": "single GPU"},
        "loop_of_single_calls": rec.get("loop_of_single_calls"),
        "path_roofline": rec["path_roofline"],
        "accuracy": rec["accuracy"],
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
