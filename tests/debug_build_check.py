"""Run by tests/test_gpu_debug_build.py in a process of its own with GSC_DEBUG=1, so that the
binding loads libgsc_debug.so (device bounds checks): training frames, the separate binning and
splat calls at both tile sizes (compared with the oracle), then the self-test, which must fail
with the check's message while the context keeps working."""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2507_19718_amd as gsc  # noqa: E402
import synth  # noqa: E402
from paper_2507_19718_amd import _abi  # noqa: E402


def main():
    assert _abi.library_path().endswith("libgsc_debug.so"), _abi.library_path()
    ctx = gsc.Context(0)
    wl = synth.workload("tiny")
    cam = wl.camera()
    levels = wl.gaussians()
    scene = gsc.Scene(ctx, gsc.Volume.from_synth(wl.volume()), [gsc.level_to_device(g) for g in levels])
    image = torch.empty((cam.h, cam.w, 3), device="cuda")
    for tile in (16, 32):
        ctx.set_frame_tiles(tile)
        for f in range(3):
            req = gsc.frame_request(cam, wl.seed, f, wl.K, wl.max_bounces, loss=wl.loss, lr=wl.lr,
                                    weight_decay=wl.weight_decay, C=wl.C, viewport_frames=f + 1)
            st = gsc.gsc_render_frame(ctx, scene, req, image, stats=True)
            assert np.isfinite(st["loss"]) and st["instances"] > 0, st
    print("frames ok", flush=True)
    # The separate calls: the 16x16 binning against the oracle's lists, then a forward and an
    # adjoint under the frames' binning (32x32 tiles, list cut).
    g = levels[0]
    dev = [gsc.level_to_device(g)]
    b = gsc.gsc_project_bin(ctx, dev, cam)
    view = gsc.gsc_binning_view(ctx, b)
    ob = oracle.bin_levels([oracle.project(g, cam)], cam)
    assert np.array_equal(view["values"].cpu().numpy().view(np.uint32), ob["values"])
    b.release()
    ctx.set_frame_binning(True)
    b = gsc.gsc_project_bin(ctx, dev, cam)
    img = torch.empty((1, cam.h, cam.w, 3), device="cuda")
    T = torch.empty((1, cam.h, cam.w), device="cuda")
    last = torch.empty((1, cam.h, cam.w), dtype=torch.int32, device="cuda")
    gsc.gsc_splat_forward(ctx, b, img, T, last)
    dimg = torch.randn((1, cam.h, cam.w, 3), device="cuda")
    grads = [{k: torch.empty_like(dev[0][k]) for k in gsc.PARAM_NAMES}]
    gsc.gsc_splat_backward(ctx, b, dev, cam, T, last, dimg, grads)
    assert all(bool(torch.isfinite(x).all()) for x in grads[0].values())
    b.release()
    ctx.synchronize()
    print("separate calls ok", flush=True)
    st, msg = ctx.debug_selftest()
    assert st == _abi.GSC_E_DEVICE and "self-test" in msg, (st, msg)
    ctx.synchronize()                     # the check is not sticky: the context still works
    st, msg = ctx.debug_selftest()
    assert st == _abi.GSC_E_DEVICE, (st, msg)
    print("debug build ok", flush=True)


if __name__ == "__main__":
    main()
