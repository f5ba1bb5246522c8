"""The debug build (libgsc_debug.so, -DGSC_DEBUG): its device bounds checks stay silent over
training frames and the separate binning and splat calls, and the check path itself reports
(gsc_debug_selftest sets a flag from a kernel; the call fails with the check's message, and the
context keeps working).  The release library compiles no check and answers the self-test with
GSC_E_UNSUPPORTED."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_release_library_has_no_debug_checks():
    import paper_2507_19718_amd as gsc
    from paper_2507_19718_amd import _abi
    assert _abi.library_path().endswith("libgsc.so")
    st, msg = gsc.Context(0).debug_selftest()
    assert st == _abi.GSC_E_UNSUPPORTED and "debug" in msg


def test_debug_build_checks_are_silent_and_report():
    from paper_2507_19718_amd import _abi
    if not os.path.exists(_abi.DEBUG_LIB_PATH):
        pytest.skip("libgsc_debug.so not built (build_lib.build(debug=True))")
    env = dict(os.environ, GSC_DEBUG="1")
    print("running tests/debug_build_check.py with GSC_DEBUG=1", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "debug_build_check.py")],
                       capture_output=True, text=True, timeout=240, env=env)
    print(r.stdout[-3000:], r.stderr[-3000:], flush=True)
    assert r.returncode == 0 and "debug build ok" in r.stdout
