"""GPU parity of the tracer with spherical area lights, for both estimators (next-event
estimation combined with phase sampling by MIS, and phase sampling alone), through the C ABI.

Same bar as the point-light tracer: the Philox streams and the operation order are shared, so
paths are expected to be bit-identical (diagnostic); the parity criterion is statistical at
1024 spp.  Also: argument validation of the new inputs, and a scene whose lights are replaced
by area lights rendering a whole frame like the oracle pipeline."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_common import adamw_params_close, frame_exclusions, rel_l2, to_np
from tests.test_gpu_train import oracle_frame, unpack

pytestmark = pytest.mark.gpu

NEE, UNIFORM = 0, 1


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


@pytest.fixture(scope="module")
def gctx(gsc):
    return gsc.Context(0)


def area_volume(wl, radius=0.3, radiance=20.0, keep_points=False, **kw):
    vol = wl.volume() if not kw else wl.volume(**kw)
    if not keep_points:
        vol.lights = np.zeros((0, 6), np.float32)
    vol.spheres = synth.sphere_lights(2, radius=radius, radiance=radiance)
    return vol


def gpu_trace(gsc, gctx, vol, cam, seed, frame, spp, B, K, C, strategy, records=True):
    gv = gsc.Volume.from_synth(vol)
    tg = torch.empty((K, cam.h, cam.w, 3), device="cuda")
    rec = torch.empty((cam.h, cam.w, 5), dtype=torch.int32, device="cuda") if records else None
    gsc.gsc_trace_targets(gctx, gv, cam, gsc.trace_params(seed, frame, spp, B, K, C, strategy=strategy),
                          tg, rec)
    return tg, rec


@pytest.mark.parametrize("strategy,C,points", [(NEE, 0.5, False), (NEE, math.inf, True),
                                               (UNIFORM, 0.5, False), (UNIFORM, math.inf, True)])
def test_area_lights_bit_identical_tiny(gsc, gctx, strategy, C, points):
    wl = synth.workload("tiny")
    vol = area_volume(wl, keep_points=points)
    cam = wl.camera()
    print(f"area lights tiny strategy={strategy} C={C} points={points}", flush=True)
    tg, rec = gpu_trace(gsc, gctx, vol, cam, wl.seed, 3, 1, 3, 3, C, strategy)
    ora = oracle.trace(vol, cam, wl.seed, 3, 1, 3, 3, C=C, strategy=strategy)
    t = to_np(tg)
    assert (ora["targets"] > 0).any()
    same = np.all(t == ora["targets"], axis=(0, 3))
    r = to_np(rec).view(np.uint32)
    same_rec = np.all(r[..., :3].view(np.float32) == ora["L"], axis=-1) & \
        (r[..., 3].view(np.float32) == ora["beta"]) & \
        ((r[..., 4] & 0xFFFF) == ora["n"]) & ((r[..., 4] >> 16) == ora["kind"])
    assert same.mean() >= 0.999, same.mean()
    assert same_rec.mean() >= 0.999, same_rec.mean()


@pytest.mark.parametrize("strategy", [NEE, UNIFORM])
def test_area_lights_3sigma_1024spp_fbm_crop(gsc, gctx, strategy):
    wl = synth.workload("orbit1k", volume_res=64)
    vol = area_volume(wl)
    cam = wl.camera().crop(496, 496, 24, 24)
    spp = 1024
    print(f"area lights 3 sigma strategy={strategy}", flush=True)
    tg, _ = gpu_trace(gsc, gctx, vol, cam, 77, 0, spp, 3, 3, 0.5, strategy, records=False)
    ora = oracle.trace(vol, cam, 77, 0, spp, 3, 3, C=0.5, records=False, second_moment=True,
                       strategy=strategy)
    mu_g = to_np(tg).astype(np.float64)
    mu_o = ora["targets"].astype(np.float64)
    var = np.maximum(ora["targets_sq"].astype(np.float64) - mu_o * mu_o, 0.0)
    zero = var == 0
    assert np.array_equal(mu_g[zero], mu_o[zero])
    z = (mu_g - mu_o)[~zero] / np.sqrt(2 * var[~zero] / spp)
    assert np.mean(np.abs(z) > 3) <= 0.005
    assert abs(np.mean(z)) <= 3
    assert np.mean(mu_g == mu_o) > 0.99


def test_area_light_arguments_validated(gsc, gctx):
    wl = synth.workload("tiny")
    cam = wl.camera().crop(0, 0, 16, 16)
    bad = area_volume(wl)
    bad.spheres[0, :3] = [1.1, 0.5, 0.5]       # radius 0.3 reaches into the cube
    with pytest.raises(gsc.GscError):
        gpu_trace(gsc, gctx, bad, cam, 1, 0, 1, 3, 1, 0.5, NEE)
    bad = area_volume(wl)
    bad.spheres[1, 3] = 0.0
    with pytest.raises(gsc.GscError):
        gpu_trace(gsc, gctx, bad, cam, 1, 0, 1, 3, 1, 0.5, NEE)
    dark = area_volume(wl)
    dark.spheres = np.zeros((0, 7), np.float32)
    with pytest.raises(gsc.GscError):            # no light at all
        gpu_trace(gsc, gctx, dark, cam, 1, 0, 1, 3, 1, 0.5, NEE)
    with pytest.raises(gsc.GscError):
        gpu_trace(gsc, gctx, area_volume(wl), cam, 1, 0, 1, 3, 1, 0.5, 2)


@pytest.mark.parametrize("spp", [1, 4])
def test_scene_with_area_lights_matches_oracle_frame(gsc, gctx, spp):
    """A resident scene built with point lights, its lights then replaced by sphere lights: two
    training frames (1 and 4 samples per pixel) match the oracle pipeline (loss, composite,
    parameters)."""
    wl = synth.workload("tiny")
    vol = wl.volume()
    cam = wl.camera()
    levels_np = wl.gaussians()
    K = wl.K
    scene = gsc.Scene(gctx, gsc.Volume.from_synth(vol), [gsc.level_to_device(g) for g in levels_np])
    area = area_volume(wl)
    scene.set_optics(area.tf, area.lights, area.spheres)
    image = torch.empty((cam.h, cam.w, 3), device="cuda")
    for frame in range(2):
        state = []
        for l in range(K):
            s = scene.state(l)
            state.append(dict(params=to_np(s["params"]), m=to_np(s["m"]), v=to_np(s["v"]), step=s["step"]))
        cur = [unpack(state[l]["params"], levels_np[l].n) for l in range(K)]
        req = gsc.frame_request(cam, wl.seed, frame, K, wl.max_bounces, loss=wl.loss, lr=wl.lr,
                                weight_decay=wl.weight_decay, C=wl.C, spp=spp)
        stats = gsc.gsc_render_frame(gctx, scene, req, image, stats=True)
        assert stats["paths"] == spp * cam.w * cam.h
        ref = oracle_frame(state, cur, area, cam, wl, frame, K, wl.loss, wl.lr, wl.weight_decay, 1,
                           spp=spp)
        assert abs(stats["loss"] - ref["loss"]) <= 1e-4 * abs(ref["loss"]), (frame, stats["loss"], ref["loss"])
        okpix = ~ref["boundary"].any(0)
        assert rel_l2(to_np(image)[okpix], ref["composite"][okpix]) <= 1e-5
        for l in range(K):
            got = to_np(scene.state(l)["params"])
            rl = ref["levels"][l]
            assert rl["boundary_gaussians"].mean() <= 0.5, rl["boundary_gaussians"].mean()
            good, info = adamw_params_close(got, rl["params"], state[l]["params"], rl["grads"],
                                            state[l]["m"], state[l]["v"], state[l]["step"] + 1,
                                            wl.lr, levels_np[l].n,
                                            exclude=frame_exclusions(rl["boundary_gaussians"],
                                                                     cur[l].log_scale))
            assert good, (frame, l, info)
