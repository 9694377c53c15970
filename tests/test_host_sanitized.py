"""The C ABI's host-side argument handling under AddressSanitizer and
UndefinedBehaviorSanitizer.  The non-GPU ABI tests (tests/test_abi.py) run
in a child process against a copy of the library whose host code is
instrumented (device code unchanged), with the sanitizer runtime preloaded;
any sanitizer report stops the child with a failing status.  No GPU is
touched: every call in those tests fails its host checks before enqueueing
anything, or is a workspace query."""
import os
import subprocess
import sys

import pytest

from paper_2208_07731_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_checks_are_clean_under_asan_and_ubsan():
    rt = B.sanitizer_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime beside hipcc")
    lib = B.build_host_sanitized()
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    code = (
        "import sys\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import paper_2208_07731_amd._lib as L\n"
        f"L.LIB_PATH = {lib!r}\n"
        "import pytest\n"
        "sys.exit(pytest.main(['-q', '-s', '-p', 'no:cacheprovider', '-m', 'not gpu', 'tests/test_abi.py']))\n"
    )
    r = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out
