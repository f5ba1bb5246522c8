"""The host-ASan check executable (tests/native/host_asan_check.hip) is instrumented: a planted
heap overflow, taken before any HIP call so it runs on the CPU, is reported by
AddressSanitizer.  The run over the C ABI itself needs the GPU (tests/test_gpu_host_asan.py)."""
import os
import subprocess

import pytest

from paper_2507_19718_amd import build_lib


def test_host_asan_executable_reports_a_planted_overflow():
    exe = build_lib.ASAN_EXE
    if not os.path.exists(exe):
        pytest.skip("host ASan check not built (build_lib.build_host_asan_check())")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    r = subprocess.run([exe, "--planted-overflow"], capture_output=True, text=True, timeout=60,
                       env=env)
    assert r.returncode != 0
    assert "AddressSanitizer: heap-buffer-overflow" in r.stderr
    assert "planted overflow not reported" not in r.stdout
