"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

libtsqr is built once more with its host code instrumented (the device code is
compiled as usual, for one padded width) and the C-ABI checks that need no GPU
(tests/test_abi.py: argument validation, layout queries, the tune cache, the
batched, comparison, streamed and CAQR argument checks) are run against it in a
child process with the ASan runtime preloaded.  Any invalid access, any
undefined behaviour (an out-of-range enumeration value, a float-to-integer
conversion that overflows) ends that process with an error report, and the
test with it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_clean_under_asan_and_ubsan(tmp_path_factory):
    from paper_0809_2407_amd import build as B

    try:
        B._hipcc()
    except RuntimeError:
        pytest.skip("no hipcc: the instrumented library cannot be built")
    rt = B.asan_runtime()
    if rt is None:
        pytest.skip("the compiler's shared ASan runtime was not found")
    lib = B.build_checked(out=str(tmp_path_factory.mktemp("checked") / "libtsqr_checked.so"))
    env = dict(os.environ)
    env.update({
        "TSQR_LIBRARY": lib,
        "LD_PRELOAD": rt,
        # Python's own allocations are not the library's: no leak report, and
        # no mismatch report for its allocator pairs
        "ASAN_OPTIONS": "detect_leaks=0:alloc_dealloc_mismatch=0:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1:exitcode=87",
    })
    env.pop("TSQR_TUNE_CACHE", None)
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_abi.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout[-6000:] + r.stderr[-6000:]
    assert r.returncode == 0, out
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out
