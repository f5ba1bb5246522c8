"""GPU parity of the splat path through the C ABI: projection and binning bit-exact against the
oracle (per-Gaussian windows and tile counts, 64-bit keys, ids, per-tile ranges), the forward
within 1e-5 relative (non-boundary pixels, last contributor exact), the adjoint within 1e-4
relative against the fp64 oracle gradient, and the autograd wrapper."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import backward as obwd
from tests.gpu_common import forward_close, grads_close, to_np, u32, u64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gsc():
    import paper_2507_19718_amd as m
    return m


@pytest.fixture(scope="module")
def gctx(gsc):
    return gsc.Context(0)


def run_bin(gsc, gctx, levels_np, cam):
    levels = [gsc.level_to_device(g) for g in levels_np]
    b = gsc.gsc_project_bin(gctx, levels, cam)
    view = gsc.gsc_binning_view(gctx, b)
    keys = gsc.gsc_binning_keys(gctx, b, view["n_instances"])
    return levels, b, view, keys


def check_binning(view, keys, levels_np, cam):
    projs = [oracle.project(g, cam) for g in levels_np]
    ob = oracle.bin_levels(projs, cam)
    off = view["gauss_offset"]
    for l, pr in enumerate(projs):
        sl = slice(off[l], off[l + 1])
        assert np.array_equal(to_np(view["tiles_touched"][sl]).astype(np.uint32), pr["tiles"]), l
        assert np.array_equal(to_np(view["window"][sl]), pr["window"]), l
        live = pr["tiles"] > 0
        assert np.array_equal(u32(view["depth_key"][sl])[live], pr["depth"].view(np.uint32)[live])
        scr = to_np(view["screen"][sl])
        assert np.array_equal(scr[live].view(np.uint32), pr["screen"][live].view(np.uint32)), l
    assert view["n_instances"] == ob["keys"].size
    assert np.array_equal(u64(keys), ob["keys"])
    assert np.array_equal(u32(view["values"]), ob["values"])
    assert np.array_equal(u64(view["ranges"]), ob["ranges"])
    return projs


def test_binning_bit_exact_tiny(gsc, gctx):
    wl = synth.workload("tiny")
    cam = wl.camera()
    levels_np = wl.gaussians()
    _, _, view, keys = run_bin(gsc, gctx, levels_np, cam)
    check_binning(view, keys, levels_np, cam)


def test_binning_bit_exact_multilevel_crop_ragged(gsc, gctx):
    cam = synth.orbit_camera(300, 200, azimuth_deg=75.0).crop(37, 21, 229, 157)   # ragged tiles
    levels_np = [synth.random_gaussians(n, 17, l) for l, n in enumerate((5000, 2500, 1, 0))]
    _, _, view, keys = run_bin(gsc, gctx, levels_np, cam)
    check_binning(view, keys, levels_np, cam)


def test_binning_empty_frame(gsc, gctx):
    # All Gaussians behind the camera: no instance, every range (0, 0).
    cam = synth.orbit_camera(64, 64, azimuth_deg=0.0)
    g = synth.random_gaussians(300, 3)
    g.pos[:] = g.pos * 0.01 + np.array([0.5, 0.5 + 0.62, 0.5 + 1.7], np.float32)
    _, _, view, keys = run_bin(gsc, gctx, [g], cam)
    check_binning(view, keys, [g], cam)


def test_binning_bit_exact_one_orbit1k_level(gsc, gctx):
    wl = synth.workload("orbit1k")
    cam = wl.camera()
    g = synth.random_gaussians(200_000, wl.seed, 0)
    _, _, view, keys = run_bin(gsc, gctx, [g], cam)
    assert view["n_instances"] > 10_000_000
    check_binning(view, keys, [g], cam)


def forward_levels(gsc, gctx, levels, cam, K):
    b = gsc.gsc_project_bin(gctx, levels, cam)
    img = torch.empty((K, cam.h, cam.w, 3), device="cuda")
    T = torch.empty((K, cam.h, cam.w), device="cuda")
    last = torch.empty((K, cam.h, cam.w), dtype=torch.int32, device="cuda")
    gsc.gsc_splat_forward(gctx, b, img, T, last)
    return b, img, T, last


@pytest.mark.parametrize("case", ["tiny", "multilevel"])
def test_forward_parity(gsc, gctx, case):
    if case == "tiny":
        wl = synth.workload("tiny")
        cam = wl.camera()
        levels_np = wl.gaussians()
    else:
        cam = synth.orbit_camera(240, 180, azimuth_deg=40.0).crop(11, 7, 200, 150)
        levels_np = [synth.random_gaussians(n, 23, l) for l, n in enumerate((8000, 4000, 2000))]
    levels = [gsc.level_to_device(g) for g in levels_np]
    K = len(levels)
    _, img, T, last = forward_levels(gsc, gctx, levels, cam, K)
    n_boundary = 0
    for l, g in enumerate(levels_np):
        pr = oracle.project(g, cam)
        fw = oracle.forward(pr, g.rgb, cam)
        ok = ~fw["boundary"]
        n_boundary += int(fw["boundary"].sum())
        good, info = forward_close(to_np(img[l]), fw["image"], ok)
        assert good, ("image", l, info)
        good, info = forward_close(to_np(T[l]), fw["final_T"], ok)
        assert good, ("final_T", l, info)
        assert np.array_equal(to_np(last[l])[ok], fw["last_id"][ok])
    assert n_boundary <= 1e-3 * K * cam.w * cam.h + 4


def grad_case_backward(gsc, gctx, cam, g, rng):
    lv = gsc.level_to_device(g)
    b, img, T, last = forward_levels(gsc, gctx, [lv], cam, 1)
    pr = oracle.project(g, cam)
    fw = oracle.forward(pr, g.rgb, cam, lists=True)
    keep = ~fw["boundary"]
    G = (rng.normal(size=(cam.h, cam.w, 3)) * keep[..., None]).astype(np.float32)
    grads = [{k: torch.empty_like(lv[k]) for k in gsc.PARAM_NAMES}]
    gsc.gsc_splat_backward(gctx, b, [lv], cam, T, last,
                           torch.from_numpy(G[None]).cuda().contiguous(), grads)
    ref = obwd.backward(g, cam, fw, G.astype(np.float64))
    return grads[0], ref


@pytest.mark.parametrize("case", ["crop32_64", "tiny"])
def test_backward_parity(gsc, gctx, case):
    rng = np.random.default_rng(3)
    if case == "crop32_64":
        cam = synth.orbit_camera(1920, 1080, azimuth_deg=30.0).crop(944, 524, 32, 32)
        g = synth.frustum_gaussians(cam, 64, seed=31)
    else:
        wl = synth.workload("tiny")
        cam = wl.camera()
        g = synth.random_gaussians(4096, 5, log_scale_mean=math.log(0.03), log_scale_std=0.2)
    got, ref = grad_case_backward(gsc, gctx, cam, g, rng)
    for k in gsc.PARAM_NAMES:
        good, info = grads_close(to_np(got[k]).reshape(ref[k].shape), ref[k])
        assert good, (k, info)


def test_autograd_function_matches_direct_backward(gsc, gctx):
    cam = synth.orbit_camera(1920, 1080, azimuth_deg=30.0).crop(900, 500, 96, 64)
    levels_np = [synth.frustum_gaussians(cam, 300, seed=41, index=l) for l in range(2)]
    levels = [gsc.level_to_device(g) for g in levels_np]
    leaf = [{k: v.clone().requires_grad_(True) for k, v in lv.items()} for lv in levels]
    images, T, last = gsc.splat(gctx, cam, leaf)
    w = torch.randn_like(images)
    (images * w).sum().backward()
    b, img2, T2, last2 = forward_levels(gsc, gctx, levels, cam, 2)
    assert torch.equal(images.detach(), img2) and torch.equal(T, T2) and torch.equal(last, last2)
    grads = [{k: torch.empty_like(lv[k]) for k in gsc.PARAM_NAMES} for lv in levels]
    gsc.gsc_splat_backward(gctx, b, levels, cam, T2, last2, w.contiguous(), grads)
    for l in range(2):
        for k in gsc.PARAM_NAMES:
            # Both are the GPU's fp32 gradient; they differ only in float-atomic order.
            good, info = grads_close(to_np(leaf[l][k].grad), to_np(grads[l][k]), tol=1e-4)
            assert good, (l, k, info)


def test_invalid_arguments_rejected(gsc, gctx):
    cam = synth.orbit_camera(64, 64, 0.0)
    g = gsc.level_to_device(synth.random_gaussians(10, 1))
    bad = cam.crop(0, 0, 65, 64)
    with pytest.raises(gsc.GscError) as e:
        gsc.gsc_project_bin(gctx, [g], bad)
    assert e.value.status == 1
    with pytest.raises(gsc.GscError):
        gsc.gsc_project_bin(gctx, [g] * 9, cam)


def test_splat_counters_match_oracle(gsc, gctx):
    """The work counters behind the splat roofline: blended pairs and the adjoint's walk length
    (position of each pixel's last blended entry in its tile list) equal the oracle's, on a
    frame without boundary pixels."""
    wl = synth.workload("tiny")
    levels_np = wl.gaussians()
    base = wl.camera()
    for cam in [base, base.crop(8, 8, 96, 96), base.crop(3, 40, 80, 64), base.crop(50, 2, 64, 100)]:
        projs = [oracle.project(g, cam) for g in levels_np]
        fws = [oracle.forward(pr, g.rgb, cam) for pr, g in zip(projs, levels_np)]
        if not any(f["boundary"].any() for f in fws):
            break
    else:
        pytest.skip("no boundary-free crop among the candidates")
    ob = oracle.bin_levels(projs, cam)
    TX, TY = (cam.w + 15) // 16, (cam.h + 15) // 16
    ranges = ob["ranges"].astype(np.int64)
    want_blend = sum(int(f["n_blend"].sum()) for f in fws)
    want_walk = 0
    for l, f in enumerate(fws):
        for y in range(cam.h):
            for x in range(cam.w):
                gid = f["last_id"][y, x]
                if gid < 0:
                    continue
                t = l * TX * TY + (y // 16) * TX + (x // 16)
                lst = ob["values"][ranges[t, 0]:ranges[t, 1]]
                want_walk += int(np.nonzero(lst == gid)[0][0]) + 1
    levels = [gsc.level_to_device(g) for g in levels_np]
    gctx.profile(True)
    gctx.set_work_counters(True)
    try:
        forward_levels(gsc, gctx, levels, cam, len(levels))
    finally:
        gctx.set_work_counters(False)
    c = gctx.counters()
    gctx.profile(False)
    assert c["blended"] == want_blend
    assert c["contributors"] == want_walk
    assert c["evaluations"] >= c["contributors"]
    assert 0 < c["tile_entries"] <= ob["keys"].size
    assert c["binnings"] == 1 and c["instances"] == ob["keys"].size


def test_capacity_overflow_reports_the_need_and_a_retry_succeeds(gsc, gctx):
    """A capacity hint one instance short makes gsc_project_bin fail with GSC_E_CAPACITY and
    report the exact instance count; binning again with that count gives the oracle's binning,
    as does a generous hint."""
    wl = synth.workload("tiny")
    cam = wl.camera()
    levels_np = wl.gaussians()
    levels = [gsc.level_to_device(g) for g in levels_np]
    ob = oracle.bin_levels([oracle.project(g, cam) for g in levels_np], cam)
    need = int(ob["keys"].size)
    with pytest.raises(gsc.GscError) as e:
        gsc.gsc_project_bin(gctx, levels, cam, capacity_hint=need - 1)
    assert e.value.status == gsc.GSC_E_CAPACITY
    assert gctx.required_capacity() == need
    for hint in (gctx.required_capacity(), 3 * need):
        view = gsc.gsc_binning_view(gctx, gsc.gsc_project_bin(gctx, levels, cam, capacity_hint=hint))
        assert view["n_instances"] == need
        assert np.array_equal(u32(view["values"]), ob["values"])
        assert np.array_equal(u64(view["ranges"]), ob["ranges"])


def test_degenerate_levels_and_windows(gsc, gctx):
    """An empty level between two non-empty ones, a 1x1 window and a level of transparent
    Gaussians (alpha below 1/255 everywhere): binning stays bit-exact, an empty or transparent
    level renders background (T = 1, last id -1) with zero gradients, and the 1x1 window's pixel
    matches the oracle."""
    base = synth.orbit_camera(96, 72, azimuth_deg=15.0)
    full = synth.random_gaussians(400, 21, 0, log_scale_mean=math.log(0.05))
    empty = synth.random_gaussians(0, 22, 1)
    faint = synth.random_gaussians(300, 23, 2, log_scale_mean=math.log(0.05))
    faint.opacity_logit[:] = np.float32(np.log(0.001 / 0.999))      # o = 0.001 < 1/255
    levels_np = [full, empty, faint]
    for cam in (base, base.crop(40, 30, 1, 1)):
        print(f"degenerate: window {cam.w}x{cam.h}", flush=True)
        levels, b, view, keys = run_bin(gsc, gctx, levels_np, cam)
        check_binning(view, keys, levels_np, cam)
        K = len(levels)
        img = torch.empty((K, cam.h, cam.w, 3), device="cuda")
        T = torch.empty((K, cam.h, cam.w), device="cuda")
        last = torch.empty((K, cam.h, cam.w), dtype=torch.int32, device="cuda")
        gsc.gsc_splat_forward(gctx, b, img, T, last)
        for l in (1, 2):
            assert torch.all(img[l] == 0) and torch.all(T[l] == 1) and torch.all(last[l] == -1)
        pr = oracle.project(full, cam)
        fw = oracle.forward(pr, full.rgb, cam)
        ok = ~fw["boundary"]
        good, info = forward_close(to_np(img[0]), fw["image"], ok)
        assert good, info
        assert np.array_equal(to_np(last[0])[ok], fw["last_id"][ok])
        dL = torch.ones((K, cam.h, cam.w, 3), device="cuda")
        grads = [{k: torch.full_like(lv[k], 7.0) for k in gsc.PARAM_NAMES} for lv in levels]
        gsc.gsc_splat_backward(gctx, b, levels, cam, T, last, dL, grads)
        for l in (1, 2):
            for k in gsc.PARAM_NAMES:
                assert torch.all(grads[l][k] == 0), (l, k)
