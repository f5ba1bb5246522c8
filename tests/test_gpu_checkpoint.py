"""Checkpoint and resume of the cache state through the C ABI (gsc_scene_save / gsc_scene_load).

A scene trained for a few frames and saved, then loaded into a fresh scene built from the same
initial Gaussians, holds the same parameters, AdamW moments and step counts bit for bit, and with
the deterministic adjoint the next training frame of both gives the same image, loss and state
bit for bit.  Files of another shape, truncated or with a damaged header are rejected before the
scene is touched."""
import numpy as np
import pytest
import torch

import synth
from tests.gpu_common import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


def fresh(gsc, ctx, vol, levels):
    return gsc.Scene(ctx, vol, [{k: v.clone() for k, v in lv.items()} for lv in levels])


def train(gsc, ctx, scene, cam, wl, frame):
    img = torch.empty((cam.h, cam.w, 3), device="cuda")
    req = gsc.frame_request(cam, wl.seed, frame, wl.K, wl.max_bounces, loss=wl.loss, lr=wl.lr,
                            weight_decay=wl.weight_decay, C=wl.C, train=True,
                            viewport_frames=frame + 1)
    st = gsc.gsc_render_frame(ctx, scene, req, img, stats=True)
    return to_np(img), st["loss"]


def same_state(a, b, K):
    for l in range(K):
        sa, sb = a.state(l), b.state(l)
        assert sa["n"] == sb["n"] and sa["step"] == sb["step"], (l, sa["step"], sb["step"])
        for k in ("params", "m", "v"):
            assert np.array_equal(to_np(sa[k]).view(np.uint32), to_np(sb[k]).view(np.uint32)), (l, k)


def test_save_load_resume_bit_for_bit(gsc, tmp_path):
    wl = synth.workload("orbit1k", volume_res=64)
    cam = wl.camera().crop(256, 256, 512, 384)
    vol = gsc.Volume.from_synth(wl.volume())
    levels = [gsc.level_to_device(g) for g in wl.gaussians()]
    ctx = gsc.Context(0)
    ctx.set_deterministic(True)
    print("checkpoint: train 3 frames, save, load, resume", flush=True)
    a = fresh(gsc, ctx, vol, levels)
    for f in range(3):
        train(gsc, ctx, a, cam, wl, f)
    path = tmp_path / "cache.gscstate"
    a.save(str(path))
    header = path.read_bytes().split(b"\n", 1)[0]
    assert header.startswith(b'{"format":"gsc-scene-state","version":1')
    assert path.stat().st_size == len(header) + 1 + sum(3 * 14 * 4 * n for n in wl.levels)
    b = fresh(gsc, ctx, vol, levels)
    b.load(str(path))
    same_state(a, b, wl.K)
    assert all(b.state(l)["step"] == 3 for l in range(wl.K))
    ia, la = train(gsc, ctx, a, cam, wl, 3)
    ib, lb = train(gsc, ctx, b, cam, wl, 3)
    assert np.array_equal(ia, ib) and la == lb
    same_state(a, b, wl.K)
    for s in (a, b):
        s.destroy()


def test_load_rejects_other_shapes_and_damaged_files(gsc, tmp_path):
    vol = gsc.Volume.from_synth(synth.workload("tiny").volume())
    ctx = gsc.Context(0)
    lv = [gsc.level_to_device(synth.random_gaussians(n, 9, index=i)) for i, n in enumerate((300, 200))]
    a = fresh(gsc, ctx, vol, lv)
    good = tmp_path / "a.gscstate"
    a.save(str(good))
    raw = good.read_bytes()
    before = [{k: to_np(v) for k, v in a.state(l).items() if k in ("params", "m", "v")} for l in range(2)]
    other = fresh(gsc, ctx, vol, lv[:1])
    cases = {
        "levels": None,
        "truncated": raw[:-4],
        "header": raw.replace(b'"version":1', b'"version":2', 1),
        "size": raw.replace(b'{"n":300,', b'{"n":301,', 1),
    }
    print("checkpoint: rejected files", flush=True)
    with pytest.raises(gsc.GscError, match="number of levels"):
        other.load(str(good))
    for name, data in cases.items():
        if data is None:
            continue
        p = tmp_path / f"{name}.gscstate"
        p.write_bytes(data)
        with pytest.raises(gsc.GscError):
            a.load(str(p))
    with pytest.raises(gsc.GscError, match="cannot open"):
        a.load(str(tmp_path / "missing.gscstate"))
    for l in range(2):
        st = a.state(l)
        for k in ("params", "m", "v"):
            assert np.array_equal(to_np(st[k]), before[l][k])
    a.load(str(good))
    for s in (a, other):
        s.destroy()
