"""The oracle's native code under AddressSanitizer and UndefinedBehaviorSanitizer.

liboracle.so is rebuilt with -fsanitize=address,undefined (host code, g++) into a temporary
directory and driven from a child Python process with the sanitizer runtimes preloaded: tracing
with point and area lights (both estimators, several samples per pixel), projection, binning,
brute-force forward splatting with lists, the transcendental helpers and ratio tracking, on small
seeded inputs.  Any out-of-bounds access or undefined behaviour aborts the child, which fails
the test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "gsc_oracle.cpp")

DRIVER = textwrap.dedent("""
    import sys
    import numpy as np
    import oracle, synth
    oracle._LIB_PATH = sys.argv[1]
    wl = synth.workload("tiny")
    cam = wl.camera().crop(40, 36, 24, 20)
    vol = wl.volume()
    for spp in (1, 3):
        out = oracle.trace(vol, cam, seed=5, frame=1, spp=spp, max_bounces=3, K=3, C=0.5,
                           second_moment=True, kinds=True)
        assert np.isfinite(out["targets"]).all()
    area = synth.Volume(vol.density, vol.density_max, vol.tf, vol.lights)
    area.spheres = synth.sphere_lights(2)
    for strategy in (oracle.STRATEGY_NEE, oracle.STRATEGY_UNIFORM):
        oracle.trace(area, cam, seed=7, frame=0, spp=2, max_bounces=3, K=3, C=float("inf"),
                     strategy=strategy)
    levels = [synth.random_gaussians(n, 11, index=i) for i, n in enumerate((600, 300))]
    projs = [oracle.project(g, cam) for g in levels]
    oracle.bin_levels(projs, cam)
    for g, pr in zip(levels, projs):
        oracle.forward(pr, g.rgb, cam, lists=True)
    x = np.linspace(-80.0, 80.0, 257, dtype=np.float32)
    oracle.expf(x)
    oracle.logf(np.abs(x) + 1e-3)
    oracle.sincosf(x)
    o = np.array([0.5, 0.5, -0.2], np.float32)
    w = np.array([0.0, 0.0, 1.0], np.float32)
    oracle.ratio_tracking_mean(vol, o, w, 1.4, seed=3, n=64)
    print("sanitized oracle ok", flush=True)
""")


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_native_code_is_clean_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("g++ sanitizer runtimes not installed")
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                           "-fno-fast-math", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                           "-shared", "-fPIC", SRC, "-o", lib])
    env = dict(os.environ)
    env.update(LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2",
               PYTHONPATH=ROOT + os.pathsep + env.get("PYTHONPATH", ""))
    r = subprocess.run([sys.executable, "-c", DRIVER, lib], capture_output=True, text=True,
                       env=env, cwd=ROOT, timeout=600)
    assert r.returncode == 0 and "sanitized oracle ok" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
