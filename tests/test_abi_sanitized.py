"""The C-ABI checks of test_abi.py against the sanitizer build of the library:
its host code compiled with AddressSanitizer and UndefinedBehaviorSanitizer
(`python -m paper_2004_02583_amd.build --sanitize`), run in a child process
with the sanitizer runtime preloaded.  No GPU: every call is validated or
sized on the host.  Skipped when that build is absent."""
import os
import subprocess
import sys

import pytest

from paper_2004_02583_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))


def test_abi_under_sanitizers():
    if not os.path.exists(B.LIB_SAN) or not os.path.exists(B.SANITIZER_RUNTIME):
        pytest.skip("sanitizer build absent (python -m paper_2004_02583_amd.build --sanitize)")
    env = dict(os.environ)
    env.update(LD_PRELOAD=B.SANITIZER_RUNTIME,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               TUCKER_ALS_LIBRARY=B.LIB_SAN)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_abi.py")],
                       env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-4000:], r.stderr[-4000:])
    assert "passed" in r.stdout
