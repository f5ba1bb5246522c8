"""The allocation-free adjoint (gsc_splat_backward_noalloc) through the C ABI: the same gradients
as gsc_splat_backward on two calls in a row, the second with a smaller input, and a clear error
beyond its size limit."""
import math

import numpy as np
import pytest
import torch

import synth
from tests.gpu_common import grads_close, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


@pytest.fixture(scope="module")
def gctx(gsc):
    return gsc.Context(0)


def _forward(gsc, gctx, levels, cam):
    K = len(levels)
    b = gsc.gsc_project_bin(gctx, levels, cam)
    img = torch.empty((K, cam.h, cam.w, 3), device="cuda")
    T = torch.empty((K, cam.h, cam.w), device="cuda")
    last = torch.empty((K, cam.h, cam.w), dtype=torch.int32, device="cuda")
    gsc.gsc_splat_forward(gctx, b, img, T, last)
    return b, T, last


def test_noalloc_adjoint_matches_the_allocating_one(gsc, gctx):
    gctx.set_deterministic(False)
    cases = [
        (synth.orbit_camera(240, 180, azimuth_deg=40.0).crop(11, 7, 200, 150), (8000, 4000, 2000), 23),
        (synth.workload("tiny").camera(), (4096,), 5),
    ]
    for cam, sizes, seed in cases:
        print(f"noalloc adjoint: {cam.w}x{cam.h}, levels {sizes}", flush=True)
        lv_np = [synth.random_gaussians(n, seed, l, log_scale_mean=math.log(0.03), log_scale_std=0.2)
                 for l, n in enumerate(sizes)]
        levels = [gsc.level_to_device(g) for g in lv_np]
        b, T, last = _forward(gsc, gctx, levels, cam)
        rng = np.random.default_rng(seed)
        dL = torch.from_numpy(rng.normal(size=(len(sizes), cam.h, cam.w, 3)).astype(np.float32)).cuda()
        ref = [{k: torch.empty_like(lv[k]) for k in gsc.PARAM_NAMES} for lv in levels]
        got = [{k: torch.full_like(lv[k], float("nan")) for k in gsc.PARAM_NAMES} for lv in levels]
        gsc.gsc_splat_backward(gctx, b, levels, cam, T, last, dL, ref)
        gsc.gsc_splat_backward_noalloc(gctx, b, levels, cam, T, last, dL, got)
        torch.cuda.synchronize()
        for l in range(len(levels)):
            for k in gsc.PARAM_NAMES:
                # Both are the same fp32 adjoint; they differ only in float-atomic order.
                good, info = grads_close(to_np(got[l][k]), to_np(ref[l][k]))
                assert good, (cam.w, l, k, info)


def test_noalloc_adjoint_rejects_too_many_gaussians(gsc, gctx):
    cam = synth.orbit_camera(64, 64, azimuth_deg=10.0)
    g = gsc.level_to_device(synth.random_gaussians(600_000, 3))
    b, T, last = _forward(gsc, gctx, [g], cam)
    grads = [{k: torch.empty_like(g[k]) for k in gsc.PARAM_NAMES}]
    dL = torch.zeros((1, cam.h, cam.w, 3), device="cuda")
    with pytest.raises(gsc.GscError) as e:
        gsc.gsc_splat_backward_noalloc(gctx, b, [g], cam, T, last, dL, grads)
    assert e.value.status == 1 and "at most 524288 Gaussians" in str(e.value)
