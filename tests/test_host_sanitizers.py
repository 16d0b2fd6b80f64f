"""The host code of the plan and validation layer under AddressSanitizer and
UndefinedBehaviorSanitizer: tests/host_check.cpp drives every entry point
through its argument checks and error paths (no GPU needed; plan creations
stop at the device query and must unwind without leaks or undefined
behaviour)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.timeout(900)
def test_host_code_under_sanitizers():
    if not shutil.which("g++") or not (os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")):
        pytest.skip("hipcc and g++ are needed for the sanitizer build")
    from paper_2108_11871_amd import build as B

    exe = B.build_host_check()
    supp = os.path.join(HERE, "lsan_hip.supp")
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               LSAN_OPTIONS="suppressions=%s:print_suppressions=0" % supp,
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "host checks passed" in r.stdout
