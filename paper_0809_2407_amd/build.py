"""Build libtsqr.so (HIP for gfx950) in-tree.

    python -m paper_0809_2407_amd.build            # full library
    python -m paper_0809_2407_amd.build --np 32    # one padded column count (fast experiments)

Every HIP unit is compiled with hipcc for gfx950 only; the kernel units are
compiled in parallel and linked into ``paper_0809_2407_amd/libtsqr.so``.  The
full build also makes ``paper_0809_2407_amd/libtsqr_peaks.so`` (calib/: the
copy, read, FMA and MFMA loops that measure the part's ceilings), which the
TSQR library does not link.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libtsqr.so")
PEAKS_SRC = os.path.join(HERE, "calib", "tsqr_peaks.hip")
PEAKS_LIB = os.path.join(HERE, "libtsqr_peaks.so")

UNITS = ["tsqr_np_0.hip", "tsqr_np_1.hip", "tsqr_np_2.hip", "tsqr_np_3.hip",
         "tsqr_dispatch.hip", "tsqr_noalloc.hip", "tsqr_cmp.hip", "tsqr_api.cpp", "tsqr_batched.cpp",
         "tsqr_tune.cpp", "tsqr_stream.cpp", "tsqr_caqr.hip"]

ARCH = "gfx950"
COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed-FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libtsqr")


CHECKED_LIB = os.path.join(HERE, "libtsqr_checked.so")
# host code under AddressSanitizer and UndefinedBehaviorSanitizer (the device
# code is compiled as usual); one padded width (32) keeps the build short
CHECKED_FLAGS = ["-O1", "-g", "-DTSQR_ONLY_NP=32",
                 "-Xarch_host", "-fsanitize=address",
                 "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]


def build_checked(out: str | None = None, jobs: int | None = None) -> str:
    """libtsqr_checked.so (at ``out``, by default beside libtsqr.so): the library
    with its host code under ASan and UBSan, for the sanitizer tests (loaded
    through TSQR_LIBRARY with the ASan runtime preloaded)."""
    out = out or CHECKED_LIB
    hipcc = _hipcc()
    tmp = tempfile.mkdtemp(prefix="tsqr_checked_")
    common = [c for c in COMMON if c != "-O3"]

    def compile_unit(u: str) -> str:
        obj = os.path.join(tmp, u + ".o")
        lang = ["-x", "hip"] if u.endswith(".hip") else []
        cmd = [hipcc] + common + CHECKED_FLAGS + lang + ["-c", os.path.join(CSRC, u), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {u}:\n{r.stderr[-4000:]}")
        return obj

    try:
        n = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
        with cf.ThreadPoolExecutor(max_workers=n) as ex:
            objs = list(ex.map(compile_unit, UNITS))
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC",
               "-Xarch_host", "-fsanitize=address",
               "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-shared-libsan", "-o", out + ".tmp"] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
        os.replace(out + ".tmp", out)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return out


def asan_runtime() -> str | None:
    """The shared AddressSanitizer runtime of the ROCm compiler (to preload)."""
    import glob

    root = os.path.dirname(os.path.dirname(os.path.realpath(_hipcc())))
    for base in (os.path.join(root, "llvm", "lib", "clang"), os.path.join(root, "lib", "llvm", "lib", "clang"),
                 "/opt/rocm/llvm/lib/clang"):
        hits = sorted(glob.glob(os.path.join(base, "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
        if hits:
            return hits[-1]
    return None


def build_peaks(verbose: bool = False) -> str:
    cmd = [_hipcc()] + COMMON + ["-shared", "-x", "hip", PEAKS_SRC, "-o", PEAKS_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {PEAKS_SRC}:\n{r.stderr[-4000:]}")
    os.replace(PEAKS_LIB + ".tmp", PEAKS_LIB)
    return PEAKS_LIB


def build(only_np: int | None = None, jobs: int | None = None, verbose: bool = False) -> str:
    hipcc = _hipcc()
    if not only_np:
        build_peaks(verbose)
    tmp = tempfile.mkdtemp(prefix="tsqr_build_")
    defs = [f"-DTSQR_ONLY_NP={only_np}"] if only_np else []
    objs = []

    def compile_unit(u: str) -> str:
        src = os.path.join(CSRC, u)
        obj = os.path.join(tmp, u + ".o")
        lang = ["-x", "hip"] if u.endswith(".hip") else []
        cmd = [hipcc] + COMMON + defs + lang + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {u}:\n{r.stderr[-4000:]}")
        return obj

    try:
        n = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
        with cf.ThreadPoolExecutor(max_workers=n) as ex:
            objs = list(ex.map(compile_unit, UNITS))
        out_tmp = LIB + ".tmp"
        cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp] + objs
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
        os.replace(out_tmp, LIB)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return LIB


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--np", type=int, default=None, help="build a single padded column count")
    ap.add_argument("-j", "--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--checked", action="store_true", help="the host-sanitized libtsqr_checked.so instead")
    a = ap.parse_args(argv)
    path = build_checked(jobs=a.jobs) if a.checked else build(a.np, a.jobs, a.verbose)
    print(path)
    return 0


if __name__ == "__main__":
    sys.exit(main())
