"""The host C++ of the library under AddressSanitizer and UBSan: the
sanitizer build (``make sanitize``) runs the front-end fuzz tests and the
C ABI tests (parser, code generation, compile cache, handle cache, argument
checks) in a child interpreter with the ASan runtime preloaded; any report
fails the run.  CPU only: no GPU code is instrumented."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1304_5553_amd", "csrc")
SAN = os.path.join(ROOT, "paper_1304_5553_amd", "libhipmr_san.so")


def _runtime(name):
    path = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True,
                          text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_host_code_under_address_and_ub_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("the compiler's sanitizer runtimes are not installed")
    subprocess.run(["make", "-C", CSRC, "-j", str(min(8, os.cpu_count() or 2)), "sanitize"],
                   check=True, capture_output=True)
    env = dict(os.environ, HIPMR_LIBRARY=SAN, LD_PRELOAD=f"{asan} {ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", "tests/test_frontend_fuzz.py", "tests/test_abi.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
