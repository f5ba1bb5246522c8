"""Pins of the oracle's volume lookup and path tracer (CPU).

Closed forms: escape probability exp(-sigma l) of delta tracking in a homogeneous medium;
the ratio-tracking transmittance mean exp(-sigma d); the single-scattering pixel integral
(B = 1, no early termination) by fp64 quadrature.  Invariants of Algorithm 1 / Eq. 3: the
expected total target does not depend on C (the Russian-roulette argument of the throughput
importance sampling section); C = 0 terminates every path at its first vertex, so levels >= 2
are identically zero.  Degenerate scenes: zero albedo gives zero targets; zero density gives
no interaction at all.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import synth


def homogeneous(res, d, tf_rgba, lights, dmax=None):
    dens = np.full((res, res, res), d, dtype=np.float32)
    tf = np.asarray(tf_rgba, dtype=np.float32)
    return synth.Volume(dens, float(dmax if dmax is not None else d), tf,
                        np.asarray(lights, dtype=np.float32).reshape(-1, 6))


def centre_pixel_cam(width=33, height=33):
    cam = synth.orbit_camera(width, height, azimuth_deg=30.0)
    return cam.crop(width // 2, height // 2, 1, 1)


def primary_ray(cam):
    R = np.asarray(cam.R, np.float64).reshape(3, 3)
    i, j = cam.x0, cam.y0
    dc = np.array([(i + 0.5 - cam.cx) / cam.fx, (j + 0.5 - cam.cy) / cam.fy, 1.0])
    dc /= np.linalg.norm(dc)
    return -R.T @ np.asarray(cam.t, np.float64), R.T @ dc


def chord(o, w):
    t0, t1 = -np.inf, np.inf
    for a in range(3):
        ta, tb = (0 - o[a]) / w[a], (1 - o[a]) / w[a]
        t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
    return max(t0, 0.0), t1


def test_trilinear_exact_at_voxel_centres_and_linear_fields(ora):
    g = np.random.default_rng(0)
    d = g.random((8, 9, 10)).astype(np.float32)
    nz, ny, nx = d.shape
    idx = np.stack(np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij"), -1).reshape(-1, 3)
    pts = (idx + 0.5) / np.array([nx, ny, nz])
    got = ora.density_at(d, pts)
    assert np.array_equal(got, d[idx[:, 2], idx[:, 1], idx[:, 0]])
    # A linear field sampled at cell centres is reproduced inside the centre hull.
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    lin = (0.3 + 2 * x[None, None, :] - 1.5 * y[None, :, None] + 0.7 * z[:, None, None]).astype(np.float32)
    p = g.uniform(0.1, 0.9, size=(1000, 3))
    ref = 0.3 + 2 * p[:, 0] - 1.5 * p[:, 1] + 0.7 * p[:, 2]
    assert np.allclose(ora.density_at(lin, p), ref, atol=2e-6)
    # Clamp to edge outside the centre hull.
    assert ora.density_at(d, np.array([[0.0, 0.0, 0.0]]))[0] == d[0, 0, 0]


def test_transfer_function_interpolates_control_points(ora):
    tf = synth.transfer_function(16, 5)
    dmax = 7.0
    d = (np.arange(16) / 15.0 * dmax).astype(np.float32)
    assert np.allclose(ora.tf_at(tf, dmax, d), tf, atol=2e-6)
    mid = ((np.arange(15) + 0.5) / 15.0 * dmax).astype(np.float32)
    assert np.allclose(ora.tf_at(tf, dmax, mid), 0.5 * (tf[:-1] + tf[1:]), atol=2e-6)
    # Clamped outside [0, dmax].
    assert np.allclose(ora.tf_at(tf, dmax, np.float32([-1.0, 2 * dmax])), tf[[0, -1]], atol=0)


def test_free_flight_escape_probability(ora):
    sigma = 3.0
    vol = homogeneous(4, sigma, [[1, 1, 1, 1], [1, 1, 1, 1]], [[2.0, 2.0, 2.0, 1, 1, 1]])
    cam = centre_pixel_cam()
    n = 200_000
    out = ora.trace(vol, cam, seed=7, frame=0, spp=n, max_bounces=1, K=1, C=math.inf,
                    records=False, kinds=True)
    esc = int(out["kind_counts"][0, 0, 0])
    o, w = primary_ray(cam)
    t0, t1 = chord(o, w)
    p = math.exp(-sigma * (t1 - t0))
    sd = math.sqrt(n * p * (1 - p))
    assert abs(esc - n * p) <= 3 * sd, (esc, n * p, sd)


def test_ratio_tracking_mean_transmittance(ora):
    # Loose majorant: density 2 everywhere with d_max = 4 and A = 1, so sigma_t = 2 and the
    # majorant is 4; each tentative collision multiplies T by 1 - 2/4.
    vol = homogeneous(4, 2.0, [[1, 1, 1, 1], [1, 1, 1, 1]], [[0, 0, 0, 0, 0, 0]], dmax=4.0)
    o = np.array([0.1, 0.2, 0.3])
    w = np.array([0.6, 0.48, 0.64])
    w = w / np.linalg.norm(w)
    dist = 0.6
    n = 400_000
    mean = ora.ratio_tracking_mean(vol, o, w, dist, seed=3, n=n)
    exact = math.exp(-2.0 * dist)
    # Each estimate is (1/2)^k with k ~ Poisson(4 d): variance = e^{-4d(1 - 1/4)} - e^{-4d}.
    var = math.exp(-4 * dist * 0.75) - math.exp(-4 * dist)
    assert abs(mean - exact) <= 3 * math.sqrt(var / n)


def single_scatter_integral(o, w, sigma, albedo, light_pos, intensity):
    t0, t1 = chord(o, w)
    lp = np.asarray(light_pos, np.float64)

    def f(t):
        x = o + t * w
        dl = lp - x
        dist = np.linalg.norm(dl)
        _, texit = chord(x, dl / dist)
        lin = min(dist, texit)
        return sigma * math.exp(-sigma * (t - t0)) * albedo * intensity / (4 * math.pi) \
            * math.exp(-sigma * lin) / (dist * dist)

    val, err = integrate.quad(f, t0, t1, epsabs=1e-12, epsrel=1e-10, limit=200)
    return val


def test_single_scattering_matches_quadrature(ora):
    sigma, albedo, I = 2.5, 0.8, 30.0
    light = [1.6, 1.4, -0.5]
    vol = homogeneous(4, sigma, [[albedo] * 3 + [1.0], [albedo] * 3 + [1.0]], [light + [I, I, I]])
    cam = centre_pixel_cam()
    n = 200_000
    out = ora.trace(vol, cam, seed=11, frame=0, spp=n, max_bounces=1, K=1, C=math.inf,
                    records=False, second_moment=True)
    mean = float(out["targets"][0, 0, 0, 0])
    var = float(out["targets_sq"][0, 0, 0, 0]) - mean * mean
    o, w = primary_ray(cam)
    exact = single_scatter_integral(o, w, sigma, albedo, light, I)
    assert abs(mean - exact) <= 3 * math.sqrt(var / n), (mean, exact)


def test_degenerate_scenes(ora):
    cam = synth.orbit_camera(24, 24, 30.0)
    lights = [[1.6, 1.4, -0.5, 10, 10, 10]]
    black = homogeneous(4, 5.0, [[0, 0, 0, 1], [0, 0, 0, 1]], lights)
    out = ora.trace(black, cam, seed=1, frame=0, spp=1, max_bounces=3, K=3, C=0.5)
    assert not out["targets"].any()
    assert (out["kind"] != 0).sum() > 0            # paths do interact
    empty = homogeneous(4, 0.0, [[1, 1, 1, 1], [1, 1, 1, 1]], lights, dmax=1.0)
    out = ora.trace(empty, cam, seed=1, frame=0, spp=1, max_bounces=3, K=3, C=0.5)
    assert not out["targets"].any()
    assert (out["kind"] == 0).all() and (out["n"] == 0).all()


@pytest.fixture(scope="module")
def tiny_volume():
    return synth.workload("tiny").volume()


def test_C_zero_terminates_at_first_vertex(ora, tiny_volume):
    cam = synth.workload("tiny").camera()
    out = ora.trace(tiny_volume, cam, seed=5, frame=0, spp=1, max_bounces=3, K=3, C=0.0)
    assert not out["targets"][1:].any()
    assert set(np.unique(out["n"])) <= {0, 1}
    assert (out["kind"][out["n"] == 1] == 3).all()


def test_C_invariance_of_expected_radiance(ora, tiny_volume):
    """E[sum_l target_l] is the same with Algorithm 1 active (C = 0.5) and disabled."""
    cam = synth.workload("tiny").camera().crop(48, 48, 32, 32)
    spp = 64
    res = {}
    for C in (0.5, math.inf):
        out = ora.trace(tiny_volume, cam, seed=21, frame=0, spp=spp, max_bounces=64, K=1, C=C,
                        records=False, second_moment=True)
        m = out["targets"][0].astype(np.float64)
        v = out["targets_sq"][0].astype(np.float64) - m * m
        res[C] = (m.sum(), v.sum() / spp)       # pixels independent: variance of the sum
    (m1, v1), (m2, v2) = res[0.5], res[math.inf]
    assert abs(m1 - m2) <= 3 * math.sqrt(v1 + v2), (m1, m2, math.sqrt(v1 + v2))


def test_targets_have_one_level_per_pixel(ora, tiny_volume):
    cam = synth.workload("tiny").camera()
    out = ora.trace(tiny_volume, cam, seed=9, frame=3, spp=1, max_bounces=3, K=3, C=0.5)
    nz = (out["targets"] != 0).any(-1).sum(0)
    assert nz.max() <= 1
    lvl = np.minimum(out["n"], 3) - 1
    has = out["n"] >= 1
    hh, ww = np.nonzero(has)
    assert np.array_equal(out["targets"][lvl[has], hh, ww], out["L"][has])


def test_records_of_every_sample(ora, tiny_volume):
    """Several samples per pixel: sample s's record is that sample's path (sample 0 equals the
    1-spp record, the stream being the same), the level targets are the per-level means of the
    records' radiance, and with a zero cache and no early termination the composite is the
    path-traced estimate (the sum of the level targets)."""
    cam = synth.workload("tiny").camera().crop(32, 32, 40, 40)
    spp, K = 4, 3
    one = ora.trace(tiny_volume, cam, seed=4, frame=2, spp=1, max_bounces=3, K=K, C=math.inf)
    many = ora.trace(tiny_volume, cam, seed=4, frame=2, spp=spp, max_bounces=3, K=K, C=math.inf)
    assert many["L"].shape == (spp, cam.h, cam.w, 3)
    assert np.array_equal(many["L"][0], one["L"]) and np.array_equal(many["n"][0], one["n"])
    lvl = np.minimum(many["n"], K) - 1
    acc = np.zeros((K, cam.h, cam.w, 3), np.float32)
    for s in range(spp):
        for l in range(K):
            acc[l] = acc[l] + np.where((lvl[s] == l)[..., None], many["L"][s], np.float32(0))
    assert np.array_equal(acc / np.float32(spp), many["targets"])
    zero_cache = np.zeros((K, cam.h, cam.w, 3), np.float32)
    comp = ora.composite(many["n"], many["kind"], many["L"], many["beta"], zero_cache)
    assert np.allclose(comp, many["targets"].sum(0), rtol=1e-6, atol=0)
    # Two identical samples average to the single-sample composite exactly.
    cache = np.abs(np.random.default_rng(0).normal(size=(K, cam.h, cam.w, 3))).astype(np.float32)
    two = [np.stack([one[k]] * 2) for k in ("n", "kind", "L", "beta")]
    assert np.array_equal(ora.composite(*two, cache),
                          ora.composite(one["n"], one["kind"], one["L"], one["beta"], cache))
