"""The native served form's scheduler (csrc/serve_core.h) on the CPU: a C++
driver with a fake executor and a hand-advanced clock checks first come first
served admission, group size, the device-memory budget, buffer-set pools,
completion, the watchdog (a group that never finishes), launch failures and
releases; built with g++ under the address and undefined-behaviour sanitizers."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_scheduler_core(tmp_path):
    exe = tmp_path / "serve_core_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                    "-fno-sanitize-recover=all", "-pthread",
                    "-I", os.path.join(ROOT, "paper_2005_02704_amd", "csrc"),
                    os.path.join(HERE, "native", "serve_core_check.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "all checks passed" in out.stdout
