"""Host-code sanitizer runs (CPU only): ThreadSanitizer, and AddressSanitizer
with UndefinedBehaviorSanitizer, on the request server's scheduler test mode
(tests/sanitize/server_stress.cpp, built by tests/sanitize/run.sh with the
library's host code instrumented).  Each build takes about a minute, so the
test runs only when SCFF_SANITIZE=1 is set."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.skipif(os.environ.get("SCFF_SANITIZE") != "1",
                                reason="sanitizer builds run on request (SCFF_SANITIZE=1)")


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["thread", "address"])
def test_server_under_sanitizer(kind, tmp_path):
    r = subprocess.run(["bash", os.path.join(ROOT, "tests", "sanitize", "run.sh"), kind, str(tmp_path)],
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ThreadSanitizer" not in out and "AddressSanitizer" not in out and "runtime error" not in out
    assert "inconsistent 0" in out
