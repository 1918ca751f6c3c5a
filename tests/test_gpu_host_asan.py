"""The C ABI from a C++ driver whose host side runs under AddressSanitizer
(tests/native/host_api_check.cpp): every entry point, launch form, tuning,
workspace limit and argument error on device 0, with the forms checked against
each other.  An invalid host access aborts the driver."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "host_api_check")


def test_host_side_is_clean_under_asan():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(EXE):
        pytest.skip("driver not built (python tests/native/build.py)")
    # the HIP runtime keeps allocations until the process ends: leaks are not checked
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    print("running", EXE, flush=True)
    run = subprocess.run([EXE], capture_output=True, text=True, env=env, timeout=110)
    assert run.returncode == 0, run.stdout + run.stderr[-4000:]
    assert "host api check: 0 failures" in run.stdout
