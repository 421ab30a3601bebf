"""The serving scheduler (csrc/kstap_sched.h: HBM arena, admission in arrival
order, fair-share slicing, the two-step pipeline, failure handling) driven on
the CPU by a fake executor (tests/native/sched_fake.cpp), built with
AddressSanitizer and UndefinedBehaviorSanitizer.  The fake's two queue threads
stand in for the copy and compute streams; it fails a test if arena memory is
reused while work on it is still queued or running, or if any work position
of a completed frame is computed other than exactly once.  Scenarios: a
300-frame stream through a budget that admits a few frames at a time, BUSY
refusal of a frame larger than the budget, an injected launch failure, an
injected device error at a step's completion, an injected upload failure
(the failed frames report an error, the others complete, and the server keeps
serving), and shutdown with tickets never waited for."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sched_fake.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    out = str(tmp_path_factory.mktemp("sched") / "sched_fake")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-pthread", SRC, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def test_scheduler_scenarios_under_sanitizers(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    for name in ("slicing_policy", "mixed_stream", "busy_refusal", "launch_failure", "device_error",
                 "upload_failure", "destroy_with_open_tickets"):
        assert f"ok {name}" in r.stdout
    assert "all scenarios passed" in r.stdout
