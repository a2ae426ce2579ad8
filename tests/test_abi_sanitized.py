"""The host code of the library (mesh validation and layout, workspace
carving, argument and error handling) under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/test_abi.py run against the host-sanitized
build, in a child process with the sanitizer runtime preloaded.  CPU only;
the build takes about a minute the first time."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_under_address_and_ub_sanitizers():
    sys.path.insert(0, ROOT)
    import glob
    from paper_2605_16082_amd import build as B
    sources = glob.glob(os.path.join(B.CSRC, "*")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    if not os.path.exists(B.ASAN_LIB) or os.path.getmtime(B.ASAN_LIB) < max(map(os.path.getmtime, sources)):
        B.build_sanitized()          # absent or older than a source
    env = dict(os.environ)
    env.update(LD_PRELOAD=B.asan_runtime(), SLIMDG_LIB=B.ASAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert "passed" in out
