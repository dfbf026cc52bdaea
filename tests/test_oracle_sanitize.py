"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code; gcc) and driven through every entry point on small inputs
(tests/oracle_sanitize_driver.c): all six families at n = 1, 2, 7, every
exchange scheme and variant, one and three threads, capture, replay,
Nelder-Mead, the network, its gradient and Adam, and the learned move in both
network precisions.  Any out-of-bounds access, use after free, leak or
undefined operation fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-std=c11", "-Wall",
           os.path.join(ROOT, "oracle", "sa_oracle.c"), os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
           "-o", str(exe), "-lm", "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "ok"
