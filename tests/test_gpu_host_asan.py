"""The library's host code under AddressSanitizer, on the GPU.

tests/native/host_asan_check.hip drives the C ABI through its host paths: contexts with a
counting allocator hook, cache initialisation, scenes, frames under each tile size, the retry of
a frame that outgrows its lists, the deterministic adjoint, a batch of two scenes, the separate
hot-path calls, the tracer, checkpoints, an optics change and the argument checks.  It is linked
with the library's sources into one executable whose host code carries AddressSanitizer (the
device code is built as in the library), so a heap or stack overflow or a use after free in the
runtime's host code ends the run with a report.  It also checks that every block taken through
the allocator hook is returned."""
import os
import subprocess

import pytest

from paper_2507_19718_amd import build_lib

pytestmark = pytest.mark.gpu


def test_host_code_under_address_sanitizer():
    exe = build_lib.ASAN_EXE
    if not os.path.exists(exe):
        pytest.skip("host ASan check not built (build_lib.build_host_asan_check())")
    env = dict(os.environ)
    # The HIP runtime keeps allocations until the process ends: no leak report.
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    print(f"running {exe}", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=180, env=env)
    print(r.stdout[-2000:], r.stderr[-4000:], flush=True)
    assert "AddressSanitizer" not in r.stderr
    assert r.returncode == 0 and "host asan check ok" in r.stdout
