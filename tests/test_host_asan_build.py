"""The checking builds on the CPU.  The host-ASan check executable
(tests/native/host_asan_check.hip) is instrumented: a planted heap overflow, taken before any HIP
call so it runs on the CPU, is reported by AddressSanitizer (the run over the C ABI itself needs
the GPU: tests/test_gpu_host_asan.py); its sanitizer flags reach host code only; and GSC_DEBUG=1
selects the debug library."""
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


def test_sanitizer_flags_apply_to_host_code_only():
    """Every -fsanitize= of the host-ASan build follows -Xarch_host, so the GPU code is built as
    in the library (no device sanitizer)."""
    for flags in (build_lib.ASAN_FLAGS,):
        for i, f in enumerate(flags):
            if f.startswith("-fsanitize="):
                assert i > 0 and flags[i - 1] == "-Xarch_host", flags
    src = open(build_lib.__file__).read()
    assert src.count('"-fsanitize=address"') == src.count('"-Xarch_host", "-fsanitize=address"')


def test_debug_library_is_selected_by_the_environment(monkeypatch):
    from paper_2507_19718_amd import _abi
    monkeypatch.delenv("GSC_DEBUG", raising=False)
    assert _abi.library_path() == _abi.LIB_PATH
    monkeypatch.setenv("GSC_DEBUG", "1")
    assert _abi.library_path() == _abi.DEBUG_LIB_PATH
    monkeypatch.setenv("GSC_DEBUG", "0")
    assert _abi.library_path() == _abi.LIB_PATH
