"""Host-side memory and undefined-behaviour check of the C ABI: the
library's sources and tests/asan_driver.cpp built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code (device code unchanged), which
calls every entry point and host path on seeded inputs and checks the
returned statuses. Built by __graft_entry__.build(); a sanitizer report
fails the run."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2106_03508_amd", "agf2_asan_check")


def test_host_paths_under_sanitizers():
    if not os.path.exists(EXE):
        pytest.fail(f"{EXE} is missing: build it with __graft_entry__.build()")
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit: no leak report; the GPU
    # driver maps memory in the low shadow gap
    env["ASAN_OPTIONS"] = "detect_leaks=0:protect_shadow_gap=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=24"
    r = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    print(out[-4000:])
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out
    assert r.returncode == 0, out[-2000:]
    assert "PASSED: 0 failure(s)" in out
