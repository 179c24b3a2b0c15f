"""The serving loop under host-side AddressSanitizer and
UndefinedBehaviorSanitizer: tests/native/serve_stress (built by the package
build against a copy of the library whose host code carries both) runs
concurrent submitting and polling threads, checks every served result
against a plain ddks_distance call on the same inputs, and destroys a context
with requests still queued or in flight.  A sanitizer report, a mismatch or a
hang fails the test."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "native", "serve_stress")


def test_serving_under_host_sanitizers():
    assert os.path.exists(EXE), "tests/native/serve_stress is built by __graft_entry__.build()"
    env = dict(os.environ)
    # leak checking would report the HIP runtime's own process-lifetime allocations
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    print("  serve_stress 4 threads x 60 requests", flush=True)
    r = subprocess.run([EXE, "4", "60"], capture_output=True, text=True, timeout=240, env=env)
    print(r.stdout, flush=True)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert "240 checked against plain calls, 0 bad" in r.stdout
