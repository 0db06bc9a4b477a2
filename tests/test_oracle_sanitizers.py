"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only) runs
every exported entry point on a small periodic box with many images (oracle/sanitize_check.c):
no memory or undefined-behaviour error, and the decomposed and halo results equal the whole."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-fopenmp", "-ffp-contract=off", "-o", str(exe),
                           os.path.join(ROOT, "oracle", "sanitize_check.c"),
                           os.path.join(ROOT, "oracle", "reann_oracle.c"), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
