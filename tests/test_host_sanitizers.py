"""The host analysis (sightline supports, nested dissection, multifrontal
layout, through ep_plan) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code, run on valid and invalid
inputs: no sanitizer report, and the expected return codes.  CPU only."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_09705_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_plan_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "plan_driver")
        cmd = ["hipcc", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
               "-Wno-unused-command-line-argument",
               os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "symbolic.cpp"),
               os.path.join(ROOT, "tests", "sanitize", "plan_driver.cpp"), "-o", exe, "-lpthread"]
        subprocess.run(cmd, check=True, capture_output=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        print(r.stdout[-2000:], r.stderr[-4000:])
        assert r.returncode == 0, r.stderr[-4000:]
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
        assert r.stdout.strip().endswith("OK")
