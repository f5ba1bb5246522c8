"""Pins of the oracle's projection, binning, forward splatting and exact-gradient backward (CPU).

Projection: the closed-form 2D covariance of an isotropic Gaussian on the optical axis, and
agreement of the fp32 bit-exact projection with an independent fp64 statement of the same
mathematics.  Binning: equality with a brute-force Python construction + sort of every
(tile, Gaussian) pair, plus range invariants.  Forward: the analytic integral of one isolated
splat, sum_k alpha_k T_k = 1 - T_final, the two-splat over operator, and id order at equal
depth.  Backward: fp64 central differences (Richardson-extrapolated, h = 1e-4) of the C++ fp64
forward against the autograd gradient on a 32x32 crop with 64 Gaussians.
"""
import math
import types

import numpy as np
import pytest

import synth


def gauss_from(pos, rot, ls, rgb, logit):
    return synth.Gaussians(np.atleast_2d(pos), np.atleast_2d(rot), np.atleast_2d(ls),
                           np.atleast_2d(rgb), np.atleast_1d(logit))


# ------------------------------------------------------------------------------------------
# Projection
# ------------------------------------------------------------------------------------------
def test_projection_on_axis_isotropic_closed_form(ora):
    cam = synth.orbit_camera(256, 256, azimuth_deg=30.0)
    for s in (0.01, 0.05, 0.1):
        g = gauss_from([0.5, 0.5, 0.5], [1, 0, 0, 0], [math.log(s)] * 3, [1, 1, 1], 0.0)
        pr = ora.project(g, cam)
        z = float(pr["depth"][0])
        assert abs(z - 1.8) < 1e-5
        var = (cam.fx * s / z) ** 2 + 0.3
        u, v, A, B, Cc, o = pr["screen"][0]
        assert abs(A * var - 1) < 2e-5 and abs(Cc * var - 1) < 2e-5
        assert abs(B) < 1e-5 * A
        assert abs(u - (cam.cx - 0.5)) < 1e-3 and abs(v - (cam.cy - 0.5)) < 1e-3
        assert o == 0.5
        r = math.ceil(3 * math.sqrt(var))
        assert abs(pr["radius"][0] - r) <= 1


def test_fp32_projection_agrees_with_fp64_statement(ora):
    import torch
    from oracle import backward as B
    cam = synth.orbit_camera(320, 240, azimuth_deg=70.0)
    g = synth.random_gaussians(5000, 3)
    pr = ora.project(g, cam)
    live = ~pr["culled"]
    t = [torch.tensor(np.asarray(a, np.float64)) for a in (g.pos, g.rot, g.log_scale, g.opacity_logit)]
    P = B.project_f64(t[0], t[1], t[2], t[3], cam)
    names = ["u", "v", "A", "B", "Cc", "o"]
    for k, name in enumerate(names):
        a = pr["screen"][live, k].astype(np.float64)
        b = P[name].numpy()[live]
        scale = np.abs(b).max() if name in ("B",) else np.maximum(np.abs(b), 1e-3 * np.abs(b).max())
        assert np.max(np.abs(a - b) / scale) < 5e-5, name


def test_culling_and_window_rules(ora):
    cam = synth.orbit_camera(64, 64, azimuth_deg=0.0)
    # Behind the camera / too near.
    eye = -np.asarray(cam.R, np.float64).reshape(3, 3).T @ cam.t
    g = gauss_from([eye + 0.1 * np.asarray(cam.R).reshape(3, 3)[2], [0.5, 0.5, 0.5]],
                   [[1, 0, 0, 0]] * 2, [[math.log(0.05)] * 3] * 2, [[1, 1, 1]] * 2, [0.0, 0.0])
    pr = ora.project(g, cam)
    assert pr["culled"][0] and not pr["culled"][1]
    w = pr["window"][1]
    assert 0 <= w[0] <= w[1] <= 63 and 0 <= w[2] <= w[3] <= 63
    rect = pr["rect"][1]
    assert tuple(rect) == (w[0] // 16, w[1] // 16, w[2] // 16, w[3] // 16)
    assert pr["tiles"][1] == (rect[1] - rect[0] + 1) * (rect[3] - rect[2] + 1)


# ------------------------------------------------------------------------------------------
# Binning
# ------------------------------------------------------------------------------------------
def brute_bin(projs, cam):
    TX, TY = (cam.w + 15) // 16, (cam.h + 15) // 16
    pairs = []
    for l, pr in enumerate(projs):
        for gid in range(pr["depth"].shape[0]):
            if pr["tiles"][gid] == 0:
                continue
            x0, x1, y0, y1 = [int(v) for v in pr["rect"][gid]]
            zb = int(np.float32(pr["depth"][gid]).view(np.uint32))
            for ty in range(y0, y1 + 1):
                for tx in range(x0, x1 + 1):
                    tile = l * TX * TY + ty * TX + tx
                    pairs.append(((tile << 32) | zb, gid))
    pairs.sort()
    return pairs, TX * TY * len(projs)


def test_binning_equals_brute_force_sort(ora):
    cam = synth.orbit_camera(80, 56, azimuth_deg=10.0).crop(3, 5, 70, 45)
    projs = [ora.project(synth.random_gaussians(n, 4, l), cam) for l, n in enumerate((60, 35))]
    b = ora.bin_levels(projs, cam)
    pairs, n_tiles = brute_bin(projs, cam)
    assert b["keys"].tolist() == [p[0] for p in pairs]
    assert b["values"].tolist() == [p[1] for p in pairs]
    ranges = np.zeros((n_tiles, 2), np.int64)
    for i, (k, _) in enumerate(pairs):
        t = k >> 32
        if i == 0 or (pairs[i - 1][0] >> 32) != t:
            ranges[t, 0] = i
        ranges[t, 1] = i + 1
    assert np.array_equal(b["ranges"].astype(np.int64), ranges)


def test_binning_invariants_tiny_workload(ora):
    wl = synth.workload("tiny")
    cam = wl.camera()
    projs = [ora.project(g, cam) for g in wl.gaussians()]
    b = ora.bin_levels(projs, cam)
    keys, ranges = b["keys"], b["ranges"].astype(np.int64)
    assert keys.size == sum(int(p["tiles"].sum()) for p in projs)
    nonempty = ranges[:, 1] > ranges[:, 0]
    r = ranges[nonempty]
    assert r[0, 0] == 0 and r[-1, 1] == keys.size
    assert np.array_equal(r[1:, 0], r[:-1, 1])          # a partition of [0, I)
    for t in np.nonzero(nonempty)[0][:64]:
        s, e = ranges[t]
        assert np.all((keys[s:e] >> np.uint64(32)) == t)
        assert np.all(np.diff((keys[s:e] & np.uint64(0xFFFFFFFF)).astype(np.int64)) >= 0)


# ------------------------------------------------------------------------------------------
# Forward
# ------------------------------------------------------------------------------------------
def test_single_isolated_splat_integral(ora):
    cam = synth.orbit_camera(160, 160, azimuth_deg=30.0)
    o = 0.33
    s = 0.016                       # screen sigma ~ fx s / z ~ 17 px
    g = gauss_from([0.5, 0.5, 0.5], [1, 0, 0, 0], [math.log(s)] * 3, [1, 1, 1],
                   math.log(o / (1 - o)))
    pr = ora.project(g, cam)
    fw = ora.forward(pr, g.rgb, cam)
    z = float(pr["depth"][0])
    s2 = (cam.fx * s / z) ** 2 + 0.3
    o32 = float(pr["screen"][0, 5])
    exact = 2 * math.pi * s2 * (o32 - 1 / 255)
    got = float(fw["image"][..., 0].astype(np.float64).sum())
    assert abs(got - exact) / exact < 2e-3, (got, exact)
    # Single layer: T = 1 - alpha exactly where it blended.
    assert np.allclose(fw["image"][..., 0], 1 - fw["final_T"], atol=1e-6)


def test_sum_alpha_T_equals_one_minus_final_T(ora):
    wl = synth.workload("tiny")
    cam = wl.camera()
    g = synth.random_gaussians(3000, 8)
    g.rgb[:] = 1.0
    pr = ora.project(g, cam)
    fw = ora.forward(pr, g.rgb, cam)
    for c in range(3):
        assert np.allclose(fw["image"][..., c], 1 - fw["final_T"], atol=2e-5)
    assert (fw["final_T"] >= 1e-4).all() and (fw["final_T"] <= 1).all()


def test_two_splats_over_operator(ora):
    cam = synth.orbit_camera(48, 48, azimuth_deg=30.0)
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    eye = -R.T @ cam.t
    fwd = R[2]
    p1 = eye + 1.5 * fwd
    p2 = eye + 2.0 * fwd + 0.02 * R[0]
    g = gauss_from([p1, p2], [[1, 0, 0, 0]] * 2, [[math.log(0.02)] * 3] * 2,
                   [[1, 0, 0], [0, 1, 0]], [0.2, -0.3])
    pr = ora.project(g, cam)
    fw = ora.forward(pr, g.rgb, cam)
    ii, jj = np.meshgrid(np.arange(48), np.arange(48))
    alphas = []
    for k in range(2):
        u, v, A, B, Cc, o = [np.float64(x) for x in pr["screen"][k]]
        dx, dy = u - ii, v - jj
        a = np.minimum(0.99, o * np.exp(-0.5 * (A * dx * dx + Cc * dy * dy) - B * dx * dy))
        w = pr["window"][k]
        inside = (ii >= w[0]) & (ii <= w[1]) & (jj >= w[2]) & (jj <= w[3])
        alphas.append(np.where(inside & (a >= 1 / 255), a, 0.0))
    a1, a2 = alphas
    assert np.allclose(fw["image"][..., 0], a1, atol=1e-5)
    assert np.allclose(fw["image"][..., 1], a2 * (1 - a1), atol=1e-5)
    assert np.allclose(fw["final_T"], (1 - a1) * (1 - a2), atol=1e-5)


def test_equal_depth_orders_by_id(ora):
    cam = synth.orbit_camera(32, 32, azimuth_deg=30.0)
    g = gauss_from([[0.5, 0.5, 0.5]] * 2, [[1, 0, 0, 0]] * 2, [[math.log(0.05)] * 3] * 2,
                   [[1, 0, 0], [0, 1, 0]], [3.0, 3.0])
    pr = ora.project(g, cam)
    fw = ora.forward(pr, g.rgb, cam)
    c = fw["image"][16, 16]
    assert c[0] > c[1] > 0
    assert fw["last_id"][16, 16] == 1


# ------------------------------------------------------------------------------------------
# Backward: FD of the independent fp64 forward vs the autograd gradient
# ------------------------------------------------------------------------------------------
def grad_case():
    cam = synth.orbit_camera(1920, 1080, azimuth_deg=30.0).crop(944, 524, 32, 32)
    g = synth.frustum_gaussians(cam, 64, seed=31)
    return cam, g


def f64_params(g):
    return types.SimpleNamespace(**{k: np.asarray(getattr(g, k), np.float64).copy()
                                    for k in ("pos", "rot", "log_scale", "rgb", "opacity_logit")},
                                 n=g.n)


@pytest.mark.parametrize("loss", ["weighted", "l2", "hdr"])
def test_backward_matches_central_differences(ora, loss):
    from oracle import backward as B
    cam, g = grad_case()
    pr = ora.project(g, cam)
    fw = ora.forward(pr, g.rgb, cam, lists=True)
    assert fw["contributing"] > 1000
    rng = np.random.default_rng(5)
    gp = f64_params(g)
    img0, sig0 = B.forward_f64(gp, cam)
    keep = ~fw["boundary"]
    if loss == "weighted":
        W = rng.normal(size=img0.shape) * keep[..., None]
        lossf = lambda img: float((W * img).sum())
        G = W
    else:
        target = rng.uniform(0, 1, size=img0.shape) * keep[..., None]
        hdr = loss == "hdr"
        # Stop-gradient denominator evaluated at the nominal prediction (Eq. 4).
        den = (np.maximum(img0, 0) + 0.01) ** 2 if hdr else np.ones_like(img0)
        k = float(img0.size)
        lossf = lambda img: float(((img - target) ** 2 / den * keep[..., None]).sum() / k)
        G = 2 * (img0 - target) / den / k * keep[..., None]
    ana = B.backward(g, cam, fw, G)
    checked = skipped = 0
    worst = 0.0
    for name in B.PARAM_NAMES:
        arr = getattr(gp, name)
        for idx in np.ndindex(arr.shape):
            base = arr[idx]

            def evalf(hh):
                arr[idx] = base + hh
                img, sig = B.forward_f64(gp, cam)
                arr[idx] = base
                return lossf(img), sig

            h = 1e-4
            fp, sp = evalf(h)
            fm, sm = evalf(-h)
            fp2, sp2 = evalf(h / 2)
            fm2, sm2 = evalf(-h / 2)
            if not (np.array_equal(sp, sig0) and np.array_equal(sm, sig0)
                    and np.array_equal(sp2, sig0) and np.array_equal(sm2, sig0)):
                skipped += 1
                continue
            d1 = (fp - fm) / (2 * h)
            d2 = (fp2 - fm2) / h
            fd = (4 * d2 - d1) / 3
            a = float(ana[name][idx])
            err = abs(fd - a)
            worst = max(worst, err / (1e-6 + 1e-5 * abs(a)))
            assert err <= 1e-6 + 1e-5 * abs(a), (name, idx, fd, a)
            checked += 1
    assert checked >= 0.8 * 64 * 14, (checked, skipped)


# ------------------------------------------------------------------------------------------
# Loss, Adam, schedule, composite
# ------------------------------------------------------------------------------------------
def test_loss_hand_values(ora):
    y = np.zeros((1, 2, 2, 3), np.float32)
    x = np.zeros_like(y)
    y[0, 0, 0, 0] = 1.0
    x[0, 1, 1, 2] = 2.0
    loss, g = ora.loss_grad(y, x, hdr=False)
    assert abs(loss - (1 + 4) / 12) < 1e-15
    assert abs(g[0, 0, 0, 0] - 2 / 12) < 1e-15 and abs(g[0, 1, 1, 2] + 4 / 12) < 1e-15
    loss, g = ora.loss_grad(y, x, hdr=True)
    assert abs(loss - (1 / 1.01 ** 2 + 4 / 0.01 ** 2) / 12) < 1e-9
    assert abs(g[0, 0, 0, 0] - 2 / 1.01 ** 2 / 12) < 1e-12
    assert abs(g[0, 1, 1, 2] + 4 / 0.01 ** 2 / 12) < 1e-9
    # Two levels sum.
    l2, _ = ora.loss_grad(np.concatenate([y, y]), np.concatenate([x, x]), hdr=False)
    assert abs(l2 - 2 * (5 / 12)) < 1e-15


def test_adam_first_step_closed_form(ora):
    g = np.float32([0.3, -2.0, 1e-3, 0.0])
    p0 = np.float32([1.0, -1.0, 0.5, 2.0])
    p, m, v = ora.adamw_step(p0, np.zeros(4, np.float32), np.zeros(4, np.float32), g, lr=1e-2,
                             beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0, step=1)
    exact = p0.astype(np.float64) - 1e-2 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p, exact, rtol=0, atol=2e-7)


def test_adamw_matches_torch_optim(ora):
    import torch
    rng = np.random.default_rng(0)
    p0 = rng.normal(size=1000).astype(np.float32)
    grads = rng.normal(size=(10, 1000)).astype(np.float32)
    for wd in (0.0, 1e-2):
        t = torch.tensor(p0.copy(), requires_grad=True)
        opt = torch.optim.AdamW([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
        p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
        for k in range(10):
            t.grad = torch.tensor(grads[k])
            opt.step()
            p, m, v = ora.adamw_step(p, m, v, grads[k], 1e-2, 0.9, 0.999, 1e-8, wd, k + 1)
        assert np.allclose(p, t.detach().numpy(), rtol=0, atol=3e-6)


def test_lr_schedule_eq5(ora):
    assert ora.lr_schedule(1e-2, 1) == 1e-2
    vals = [ora.lr_schedule(1.0, t) for t in range(1, 50)]
    assert all(a > b for a, b in zip(vals, vals[1:]))
    assert abs(ora.lr_schedule(1.0, 10) - 1 / (1 + math.log(10))) < 1e-15


def test_composite_rules(ora):
    K = 2
    cache = np.zeros((K, 1, 4, 3), np.float32)
    cache[0, 0, :, :] = 0.5
    cache[1, 0, :, :] = -1.0                     # negative cache reads are clamped to 0
    n = np.array([[1, 2, 1, 0]])
    kind = np.array([[3, 3, 1, 0]])
    L = np.zeros((1, 4, 3), np.float32)
    L[0, 2] = [0.0, 0.0, 0.0]
    beta = np.float32([[0.25, 0.5, 1.0, 1.0]])
    out = ora.composite(n, kind, L, beta, cache)
    assert np.allclose(out[0, 0], 2.0)           # early: 0.5 / 0.25
    assert np.allclose(out[0, 1], 0.0)           # early at level 2, cache clamped
    assert np.allclose(out[0, 2], 0.5)           # natural, zero radiance -> cache / beta
    assert np.allclose(out[0, 3], 0.0)           # no interaction
    L[0, 2] = [1.0, 2.0, 3.0]
    out = ora.composite(n, kind, L, beta, cache)
    assert np.allclose(out[0, 2], [1, 2, 3])     # natural, radiance kept


def test_paper_memory_footprint(ora):
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))
    fp = gold["memory_footprint"]
    total = sum(n * fp["floats_per_gaussian"] * 4 for n in fp["level_sizes"])
    assert total == fp["total_bytes"]
    for n, mb in zip(fp["level_sizes"], fp["level_MB"]):
        assert abs(n * 14 * 4 / 2**20 - mb) < 0.006
