"""The served loop on the GPU: every request completes; a request's result is the same alone
and in the mix (its scene's state is snapshotted just before the batch that holds it, and the
request is re-run alone from the snapshot); the plain loop and the served loop leave every
scene in the same state up to float-atomic order."""
import math

import numpy as np
import pytest
import torch

import synth
from tests.gpu_common import rel_l2, to_np

pytestmark = pytest.mark.gpu

RES = ((160, 90), (320, 180), (256, 144))


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


def make_scenes(gsc, ctx, n_scenes=3):
    from paper_2507_19718_amd import serve
    specs, init = [], []
    for s in range(n_scenes):
        wl = synth.workload("orbit1k", volume_res=48, levels=[3000, 1500], seed=0x5E0 + s)
        vol = wl.volume()
        levels = [gsc.level_to_device(g) for g in wl.gaussians()]
        scene = gsc.Scene(ctx, gsc.Volume.from_synth(vol), levels)
        specs.append(serve.SceneSpec(scene, wl.K, wl.max_bounces, 1, wl.lr, 1e-2, 0.5))
        init.append((vol, levels))
    return specs, init


def cam_of(e):
    return synth.orbit_camera(e["width"], e["height"], e["azimuth"], e["elevation"], e["radius"])


def requests(n=36, seed=11):
    log = synth.poisson_requests(2000.0, 1.0, 9, 3, seed, resolutions=RES)[:n]
    import paper_2507_19718_amd.serve as serve
    return serve.make_requests(log, cam_of)


def test_alone_equals_mix(gsc):
    import paper_2507_19718_amd.serve as serve
    ctx = gsc.Context(0)
    specs, init = make_scenes(gsc, ctx)
    snaps = {}
    results = {}
    sample = set(range(0, 36, 5))
    snap_scene = {}

    def before(slot, batch):
        for r in batch:
            if r.idx in sample:
                sc = specs[r.scene].scene
                vol, levels = init[r.scene]
                sn = gsc.Scene(ctx, gsc.Volume.from_synth(vol), levels)
                sn.copy_state_from(sc)
                ctx.synchronize()
                snaps[r.idx] = sn

    def after(slot, batch, images):
        for r, img in zip(batch, images):
            if r.idx in sample:
                results[r.idx] = (img.clone(), [specs[r.scene].scene.state(l) for l in range(specs[r.scene].K)])

    b = serve.ContinuousBatcher(specs, slots=2, before_launch=before, after_batch=after, max_batch=3)
    reqs = requests()
    res = b.run(reqs, realtime=False)
    torch.cuda.synchronize()
    assert res["frames"] == len(reqs)
    assert any(len(x) > 1 for x in b.batches), "no batching happened"
    alone_ctx = gsc.Context(0)
    for r in reqs:
        if r.idx not in sample:
            continue
        sn = snaps[r.idx]
        spec = specs[r.scene]
        img = torch.empty((r.cam.h, r.cam.w, 3), device="cuda")
        gsc.gsc_render_frame(alone_ctx, sn, serve._req_struct(spec, r), img)
        alone_ctx.synchronize()
        mix_img, mix_state = results[r.idx]
        assert rel_l2(to_np(img), to_np(mix_img)) <= 1e-5, r.idx
        for l in range(spec.K):
            st = sn.state(l)
            got, want = to_np(st["params"]), to_np(mix_state[l]["params"])
            lr = max(spec.lr)
            assert np.max(np.abs(got - want)) <= 2 * lr + 1e-7
            assert np.mean(np.abs(got - want) <= 1e-3 * lr + 1e-7) > 0.99
            assert st["step"] == mix_state[l]["step"]


def test_alone_equals_mix_bit_for_bit_with_the_deterministic_adjoint(gsc):
    """With fixed-point adjoint sums nothing in a frame depends on the order of atomics, so a
    request served in a mixed batch and the same request run alone from a snapshot give the
    same image and the same parameters, moments and step counts bit for bit."""
    import paper_2507_19718_amd.serve as serve
    ctx = gsc.Context(0)
    ctx.set_deterministic(True)
    specs, init = make_scenes(gsc, ctx)
    snaps, results = {}, {}
    sample = set(range(1, 36, 4))

    def before(slot, batch):
        for r in batch:
            if r.idx in sample:
                vol, levels = init[r.scene]
                sn = gsc.Scene(ctx, gsc.Volume.from_synth(vol), levels)
                sn.copy_state_from(specs[r.scene].scene)
                ctx.synchronize()
                snaps[r.idx] = sn

    def after(slot, batch, images):
        for r, img in zip(batch, images):
            if r.idx in sample:
                sc = specs[r.scene].scene
                results[r.idx] = (img.clone(), [sc.state(l) for l in range(specs[r.scene].K)])

    b = serve.ContinuousBatcher(specs, slots=2, before_launch=before, after_batch=after, max_batch=3,
                                deterministic=True)
    reqs = requests(seed=12)
    b.run(reqs, realtime=False)
    torch.cuda.synchronize()
    assert any(len(x) > 1 for x in b.batches), "no batching happened"
    alone = gsc.Context(0)
    alone.set_deterministic(True)
    checked = 0
    for r in reqs:
        if r.idx not in sample:
            continue
        sn, spec = snaps[r.idx], specs[r.scene]
        img = torch.empty((r.cam.h, r.cam.w, 3), device="cuda")
        gsc.gsc_render_frame(alone, sn, serve._req_struct(spec, r), img)
        alone.synchronize()
        mix_img, mix_state = results[r.idx]
        assert torch.equal(img, mix_img), r.idx
        for l in range(spec.K):
            st = sn.state(l)
            for k in ("params", "m", "v"):
                assert torch.equal(st[k], mix_state[l][k]), (r.idx, l, k)
            assert st["step"] == mix_state[l]["step"]
        checked += 1
    assert checked == len(sample)


def test_plain_and_served_reach_same_state(gsc):
    import paper_2507_19718_amd.serve as serve
    ctx = gsc.Context(0)
    specs_a, _ = make_scenes(gsc, ctx)
    specs_b, _ = make_scenes(gsc, ctx)
    reqs_a, reqs_b = requests(24, 5), requests(24, 5)
    ra = serve.run_plain(ctx, specs_a, reqs_a, realtime=False)
    rb = serve.ContinuousBatcher(specs_b, slots=2).run(reqs_b, realtime=False)
    assert ra["frames"] == rb["frames"] == 24
    for s in range(3):
        for l in range(specs_a[s].K):
            a = specs_a[s].scene.state(l)
            bb = specs_b[s].scene.state(l)
            assert a["step"] == bb["step"]
            pa, pb = to_np(a["params"]), to_np(bb["params"])
            assert np.mean(np.abs(pa - pb) <= 1e-3 * max(specs_a[s].lr) + 1e-7) > 0.98
