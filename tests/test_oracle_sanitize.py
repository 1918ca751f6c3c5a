"""The oracle under the host's address and undefined-behaviour sanitizers: a
standalone C driver (oracle/sanitize_check.c) runs every entry point on seeded
synthetic sweeps, including the degenerate ones; any invalid access or undefined
operation aborts it."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no gcc")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "sanitize_check"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "lidar_oracle.c"),
           os.path.join(ROOT, "oracle", "sanitize_check.c"), "-lm", "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "sanitize check: 0 failures" in run.stdout
    assert "runtime error" not in run.stderr
