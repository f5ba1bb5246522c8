"""The deterministic adjoint: with gsc_ctx_set_deterministic on, the splat adjoint sums each
Gaussian's per-tile partials as fixed-point integers, so its gradients repeat bit for bit, stay
within the gradient bar of the fp64 oracle, and agree with the float-atomic mode up to rounding.
Training frames built on it repeat bit for bit too, and since a cut tile list drops only
instances no pixel reaches, a frame with the cut and one without then write the same parameters
bit for bit."""
import math

import numpy as np
import pytest
import torch

import synth
from tests.gpu_common import grads_close, to_np
from tests.test_gpu_splat import forward_levels, grad_case_backward

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


@pytest.fixture
def dctx(gsc):
    ctx = gsc.Context(0)
    ctx.set_deterministic(True)
    yield ctx
    ctx.set_deterministic(False)


@pytest.mark.parametrize("case", ["crop32_64", "tiny"])
def test_deterministic_backward_parity(gsc, dctx, case):
    rng = np.random.default_rng(3)
    if case == "crop32_64":
        cam = synth.orbit_camera(1920, 1080, azimuth_deg=30.0).crop(944, 524, 32, 32)
        g = synth.frustum_gaussians(cam, 64, seed=31)
    else:
        cam = synth.workload("tiny").camera()
        g = synth.random_gaussians(4096, 5, log_scale_mean=math.log(0.03), log_scale_std=0.2)
    print(f"deterministic backward parity {case}", flush=True)
    got, ref = grad_case_backward(gsc, dctx, cam, g, rng)
    for k in gsc.PARAM_NAMES:
        good, info = grads_close(to_np(got[k]).reshape(ref[k].shape), ref[k])
        assert good, (k, info)


def adjoint(gsc, ctx, levels, cam, dL):
    b, _, T, last = forward_levels(gsc, ctx, levels, cam, len(levels))
    grads = [{k: torch.empty_like(lv[k]) for k in gsc.PARAM_NAMES} for lv in levels]
    gsc.gsc_splat_backward(ctx, b, levels, cam, T, last, dL, grads)
    torch.cuda.synchronize()
    return [{k: to_np(v) for k, v in g.items()} for g in grads]


def test_deterministic_backward_repeats_bit_for_bit(gsc, dctx):
    # Large, heavily overlapping splats: each Gaussian collects partials from many tiles, the
    # case where the order of float atomics changes the sums from run to run.
    cam = synth.orbit_camera(640, 480, azimuth_deg=20.0)
    levels_np = [synth.frustum_gaussians(cam, 20000, seed=7, index=l) for l in range(2)]
    levels = [gsc.level_to_device(g) for g in levels_np]
    dL = torch.randn((2, cam.h, cam.w, 3), device="cuda", generator=torch.Generator("cuda").manual_seed(5))
    print("deterministic backward repeats", flush=True)
    runs = [adjoint(gsc, dctx, levels, cam, dL) for _ in range(3)]
    for r in runs[1:]:
        for l in range(2):
            for k in gsc.PARAM_NAMES:
                assert np.array_equal(r[l][k].view(np.uint32), runs[0][l][k].view(np.uint32)), (l, k)
    dctx.set_deterministic(False)
    atomic = adjoint(gsc, dctx, levels, cam, dL)
    for l in range(2):
        for k in gsc.PARAM_NAMES:
            good, info = grads_close(runs[0][l][k], atomic[l][k], tol=1e-4)
            assert good, (l, k, info)


def train_frame(gsc, ctx, vol, levels, cam, wl, cut):
    scene = gsc.Scene(ctx, vol, [{k: v.clone() for k, v in lv.items()} for lv in levels])
    ctx.set_list_cut(cut)
    img = torch.empty((cam.h, cam.w, 3), device="cuda")
    req = gsc.frame_request(cam, wl.seed, 0, wl.K, wl.max_bounces, loss=wl.loss, lr=wl.lr,
                            weight_decay=wl.weight_decay, C=wl.C, train=True)
    st = gsc.gsc_render_frame(ctx, scene, req, img, stats=True)
    out = dict(img=to_np(img), loss=st["loss"],
               params=[to_np(scene.state(l)["params"]) for l in range(wl.K)])
    scene.destroy()
    ctx.set_list_cut(True)
    return out


def test_deterministic_frames_repeat_and_ignore_the_list_cut(gsc, dctx):
    wl = synth.workload("orbit1k", volume_res=64)
    cam = wl.camera()
    vol = gsc.Volume.from_synth(wl.volume())
    levels = [gsc.level_to_device(g) for g in wl.gaussians()]
    print("deterministic frames", flush=True)
    a = train_frame(gsc, dctx, vol, levels, cam, wl, True)
    b = train_frame(gsc, dctx, vol, levels, cam, wl, True)
    c = train_frame(gsc, dctx, vol, levels, cam, wl, False)
    for o in (b, c):
        assert np.array_equal(o["img"], a["img"]) and o["loss"] == a["loss"]
        for pa, po in zip(a["params"], o["params"]):
            assert np.array_equal(pa.view(np.uint32), po.view(np.uint32))
