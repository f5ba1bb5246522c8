"""Parity at the benchmark's full size (1920x1080, 512^3 fBm, 4 levels x 1M Gaussians), in the
same launch configuration as the benchmark (all four levels in one batch), on sampled outputs
the oracle can compute one by one: per-tile instance lists (brute force over the tile
rectangles), per-pixel forward results (the oracle on 1x1 windows reproduces full-frame pixels
exactly), traced targets of sampled pixels, and invariants of the whole binning."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_common import to_np, u32, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


@pytest.fixture(scope="module")
def full(gsc):
    wl = synth.workload("fhd")
    cam = wl.camera()
    levels_np = wl.gaussians()
    ctx = gsc.Context(0)
    levels = [gsc.level_to_device(g) for g in levels_np]
    b = gsc.gsc_project_bin(ctx, levels, cam)
    K = len(levels)
    img = torch.empty((K, cam.h, cam.w, 3), device="cuda")
    T = torch.empty((K, cam.h, cam.w), device="cuda")
    last = torch.empty((K, cam.h, cam.w), dtype=torch.int32, device="cuda")
    gsc.gsc_splat_forward(ctx, b, img, T, last)
    view = gsc.gsc_binning_view(ctx, b)
    projs = [oracle.project(g, cam) for g in levels_np]
    return dict(wl=wl, cam=cam, levels_np=levels_np, ctx=ctx, b=b, img=img, T=T, last=last,
                view=view, projs=projs)


def test_fullsize_projection_bit_exact(full):
    v = full["view"]
    off = v["gauss_offset"]
    for l, pr in enumerate(full["projs"]):
        sl = slice(off[l], off[l + 1])
        assert np.array_equal(to_np(v["tiles_touched"][sl]).astype(np.uint32), pr["tiles"])
        assert np.array_equal(to_np(v["window"][sl]), pr["window"])
    total = sum(int(p["tiles"].sum()) for p in full["projs"])
    assert v["n_instances"] == total
    assert total > 100_000_000


def test_fullsize_sampled_tile_lists(full):
    v = full["view"]
    cam = full["cam"]
    TX, TY = (cam.w + 15) // 16, (cam.h + 15) // 16
    ranges = u64(v["ranges"]).astype(np.int64)
    values = v["values"]
    rng = np.random.default_rng(0)
    tiles = list(rng.integers(0, 4 * TX * TY, size=24)) + [0, TX - 1, TX * TY - 1, 4 * TX * TY - 1]
    for t in tiles:
        l, lt = divmod(int(t), TX * TY)
        ty, tx = divmod(lt, TX)
        pr = full["projs"][l]
        r = pr["rect"]
        cover = (pr["tiles"] > 0) & (r[:, 0] <= tx) & (tx <= r[:, 1]) & (r[:, 2] <= ty) & (ty <= r[:, 3])
        ids = np.nonzero(cover)[0]
        keys = pr["depth"][ids].view(np.uint32)
        order = np.lexsort((ids, keys))
        want = ids[order].astype(np.uint32)
        s, e = ranges[t]
        if want.size == 0:
            assert s == 0 and e == 0
            continue
        got = u32(values[s:e])
        assert np.array_equal(got, want), (t, got[:5], want[:5])


def test_fullsize_binning_invariants(full):
    v = full["view"]
    ranges = u64(v["ranges"]).astype(np.int64)
    ne = ranges[:, 1] > ranges[:, 0]
    r = ranges[ne]
    assert r[0, 0] == 0 and r[-1, 1] == v["n_instances"]
    assert np.array_equal(r[1:, 0], r[:-1, 1])


def test_fullsize_sampled_pixels_forward(full):
    cam = full["cam"]
    rng = np.random.default_rng(1)
    px = np.concatenate([rng.integers(0, cam.w, 20), [0, cam.w - 1]])
    py = np.concatenate([rng.integers(0, cam.h, 20), [cam.h - 1, 0]])
    img, T, last = to_np(full["img"]), to_np(full["T"]), to_np(full["last"])
    for x, y in zip(px, py):
        pc = cam.crop(int(x), int(y), 1, 1)
        for l, g in enumerate(full["levels_np"]):
            pr = oracle.project(g, pc)
            fw = oracle.forward(pr, g.rgb, pc)
            if fw["boundary"][0, 0]:
                continue
            ref = fw["image"][0, 0].astype(np.float64)
            got = img[l, y, x].astype(np.float64)
            assert np.all(np.abs(got - ref) <= 1e-5 * max(1.0, np.abs(ref).max())), (x, y, l, got, ref)
            assert abs(float(T[l, y, x]) - float(fw["final_T"][0, 0])) <= 1e-5
            assert last[l, y, x] == fw["last_id"][0, 0]


def test_fullsize_sampled_trace(full, gsc):
    wl = full["wl"]
    cam = full["cam"]
    vol = wl.volume()
    gv = gsc.Volume.from_synth(vol)
    K = wl.K
    tg = torch.empty((K, cam.h, cam.w, 3), device="cuda")
    rec = torch.empty((cam.h, cam.w, 5), dtype=torch.int32, device="cuda")
    gsc.gsc_trace_targets(full["ctx"], gv, cam, gsc.trace_params(wl.seed, 7, 1, wl.max_bounces, K), tg, rec)
    t = to_np(tg)
    crop = cam.crop(900, 500, 48, 32)
    ora = oracle.trace(vol, crop, wl.seed, 7, 1, wl.max_bounces, K, C=wl.C)
    sub = t[:, 500:532, 900:948]
    same = np.all(sub == ora["targets"], axis=(0, 3))
    assert same.mean() >= 0.999, same.mean()


def test_fullsize_frame_composite_sampled(full, gsc):
    """The benchmark's own configuration: one gsc_render_frame of the whole 1080p workload (all
    levels in one batch, the trace on its second stream, cut tile lists), render only.  Sampled
    composite pixels equal the oracle's composite of the oracle's per-level forward and the
    oracle's traced record at that pixel."""
    wl = full["wl"]
    cam = full["cam"]
    vol = wl.volume()
    K = wl.K
    scene = gsc.Scene(full["ctx"], gsc.Volume.from_synth(vol),
                      [gsc.level_to_device(g) for g in full["levels_np"]])
    image = torch.empty((cam.h, cam.w, 3), device="cuda")
    req = gsc.frame_request(cam, wl.seed, 7, K, wl.max_bounces, loss=wl.loss, train=False, C=wl.C)
    gsc.gsc_render_frame(full["ctx"], scene, req, image)
    comp = to_np(image)
    scene.destroy()
    # The frame's own trace, for the rare pixel whose path differs from the oracle's in the last
    # bit (the trace's bar is statistical): such pixels are skipped.
    rec = torch.empty((cam.h, cam.w, 5), dtype=torch.int32, device="cuda")
    tg = torch.empty((K, cam.h, cam.w, 3), device="cuda")
    gsc.gsc_trace_targets(full["ctx"], gsc.Volume.from_synth(vol), cam,
                          gsc.trace_params(wl.seed, 7, 1, wl.max_bounces, K, wl.C), tg, rec)
    rec = to_np(rec).view(np.uint32)
    rng = np.random.default_rng(2)
    px = np.concatenate([rng.integers(0, cam.w, 14), [cam.w // 2, cam.w - 1]])
    py = np.concatenate([rng.integers(0, cam.h, 14), [cam.h // 2, cam.h - 1]])
    checked = 0
    for x, y in zip(px, py):
        pc = cam.crop(int(x), int(y), 1, 1)
        imgs, boundary = [], False
        for g in full["levels_np"]:
            fw = oracle.forward(oracle.project(g, pc), g.rgb, pc)
            boundary = boundary or bool(fw["boundary"][0, 0])
            imgs.append(fw["image"])
        if boundary:
            continue
        tr = oracle.trace(vol, pc, wl.seed, 7, 1, wl.max_bounces, K, C=wl.C)
        r = rec[y, x]
        if not (np.array_equal(r[:3].view(np.float32), tr["L"][0, 0]) and
                (r[4] & 0xFFFF) == tr["n"][0, 0] and (r[4] >> 16) == tr["kind"][0, 0]):
            continue
        ref = oracle.composite(tr["n"], tr["kind"], tr["L"], tr["beta"], np.stack(imgs))[0, 0]
        got = comp[y, x].astype(np.float64)
        assert np.all(np.abs(got - ref) <= 1e-5 * max(1.0, float(np.abs(ref).max()))), (x, y, got, ref)
        checked += 1
    assert checked >= 10


def test_fullsize_backward_in_the_frame_binning(gsc):
    """The adjoint at full size, binned the way the frames bin (32x32 tiles, list cut on,
    heaviest-first tile order, long lists walked in many 64-entry batches): dL/dimage nonzero
    only on a 64x64 window of the 1920x1080 frame (random values, boundary pixels zeroed), every
    Gaussian's 14 gradients against the oracle's exact fp64 gradient on that window (a crop
    reproduces the full frame's pixels exactly), per parameter group within the gradient bar;
    Gaussians that touch no pixel of the window get exactly zero."""
    from oracle import backward as obwd
    from tests.gpu_common import grads_close
    wl = synth.workload("fhd")
    cam = wl.camera()
    levels_np = wl.gaussians()
    ctx = gsc.Context(0)
    ctx.set_frame_binning(True)
    levels = [gsc.level_to_device(g) for g in levels_np]
    K = len(levels)
    x0, y0, n = 904, 508, 64
    crop = cam.crop(x0, y0, n, n)
    rng = np.random.default_rng(11)
    dL = np.zeros((K, cam.h, cam.w, 3), np.float32)
    fws = []
    for l, g in enumerate(levels_np):
        pr = oracle.project(g, crop)
        fw = oracle.forward(pr, g.rgb, crop, lists=True)
        fws.append(fw)
        G = rng.normal(size=(n, n, 3)).astype(np.float32) * (~fw["boundary"])[..., None]
        dL[l, y0:y0 + n, x0:x0 + n] = G
    print("full-size adjoint: binning 4 x 1M in 32x32 tiles with the list cut", flush=True)
    b = gsc.gsc_project_bin(ctx, levels, cam)
    img = torch.empty((K, cam.h, cam.w, 3), device="cuda")
    T = torch.empty((K, cam.h, cam.w), device="cuda")
    last = torch.empty((K, cam.h, cam.w), dtype=torch.int32, device="cuda")
    gsc.gsc_splat_forward(ctx, b, img, T, last)
    view = gsc.gsc_binning_view(ctx, b)
    assert view["tiles_x"] == (cam.w + 31) // 32 and view["tiles_y"] == (cam.h + 31) // 32
    grads = [{k: torch.empty_like(lv[k]) for k in gsc.PARAM_NAMES} for lv in levels]
    gsc.gsc_splat_backward(ctx, b, levels, cam, T, last, torch.from_numpy(dL).cuda(), grads)
    torch.cuda.synchronize()
    for l, g in enumerate(levels_np):
        ref = obwd.backward(g, crop, fws[l], dL[l, y0:y0 + n, x0:x0 + n].astype(np.float64))
        touched = np.zeros(g.n, bool)
        touched[np.unique(fws[l]["list_ids"])] = True
        assert touched.sum() > 1000
        for k in gsc.PARAM_NAMES:
            got = to_np(grads[l][k]).reshape(ref[k].shape)
            good, info = grads_close(got, ref[k])
            assert good, (l, k, info)
            assert not np.any(got[~touched]), (l, k)
