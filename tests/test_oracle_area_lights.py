"""Pins of the oracle's spherical area lights, their MIS combination and the uniform baseline.

The evaluation lights every scene with two small spherical area lights outside the volume and
compares against a uniform (phase-sampling only) path tracer and one with next-event
estimation (Evaluation: scenes and baselines); next-event estimation is combined with the
continued path by multiple importance sampling (Method: path termination heuristics).

Pins, chosen so that a wrong cone pdf, MIS weight, hit test, occlusion rule or a dropped
continuation fails one of them:
  * single scattering (B = 1, homogeneous, one sphere light) against fp64 quadrature over the
    view ray and the cone of directions the sphere subtends, for both estimators;
  * the two estimators have the same expected path radiance in a heterogeneous volume, with
    two lights, one of them partly hiding the other (summed over levels: a path's radiance goes
    to the level of its final length, and next-event estimation gathers at earlier vertices
    what phase sampling gathers on escape);
  * a vanishing sphere of radiance Le is a point light of intensity Le pi r^2;
  * point lights give the uniform estimator nothing; a black area light gives nothing.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import synth
from tests.test_oracle_trace import centre_pixel_cam, chord, homogeneous, primary_ray

NEE, UNIFORM = 0, 1


def with_spheres(vol, spheres):
    vol.spheres = np.asarray(spheres, dtype=np.float32).reshape(-1, 7)
    return vol


def exit_distance(x, w):
    """Distance from x (inside the unit cube) along unit directions w [n][3] to the cube."""
    with np.errstate(divide="ignore", invalid="ignore"):
        ta = (0.0 - x[None, :]) / w
        tb = (1.0 - x[None, :]) / w
        t = np.where(w == 0.0, np.inf, np.maximum(ta, tb))
    return np.min(t, axis=1)


def cone_nodes(n_theta=96, n_phi=192):
    """Gauss-Legendre nodes on [0, 1] x [0, 2 pi) for the cone integral."""
    gt, wt = np.polynomial.legendre.leggauss(n_theta)
    gp, wp = np.polynomial.legendre.leggauss(n_phi)
    return (gt + 1) / 2, wt / 2, math.pi * (gp + 1), math.pi * wp


def single_scatter_sphere(o, w, sigma, albedo, centre, radius, le):
    """fp64: integral over the view chord of sigma e^{-sigma (t - t0)} albedo times
    (1/4pi) integral over the cone of Le e^{-sigma l(x, w')} dw'."""
    t0, t1 = chord(o, w)
    c = np.asarray(centre, np.float64)
    ut, wt, ph, wph = cone_nodes()

    def inner(x):
        dvec = c - x
        d = np.linalg.norm(dvec)
        a = dvec / d
        cos_max = math.sqrt(1.0 - (radius / d) ** 2)
        # theta from 0 to theta_max: substitute cos(theta) = 1 - u (1 - cos_max), dw = (1-cos_max) du dphi
        cth = 1.0 - np.outer(ut, np.ones_like(ph)) * (1.0 - cos_max)
        sth = np.sqrt(np.maximum(0.0, 1.0 - cth * cth))
        tmp = np.array([1.0, 0.0, 0.0]) if abs(a[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        b1 = np.cross(a, tmp)
        b1 /= np.linalg.norm(b1)
        b2 = np.cross(a, b1)
        cp, sp = np.cos(ph)[None, :], np.sin(ph)[None, :]
        dirs = (sth * cp)[..., None] * b1 + (sth * sp)[..., None] * b2 + cth[..., None] * a
        ell = exit_distance(x, dirs.reshape(-1, 3)).reshape(cth.shape)
        f = np.exp(-sigma * ell)
        return (1.0 - cos_max) * float(wt @ f @ wph)

    def g(t):
        x = o + t * w
        return sigma * math.exp(-sigma * (t - t0)) * albedo * le / (4 * math.pi) * inner(x)

    val, _ = integrate.quad(g, t0, t1, epsabs=1e-12, epsrel=1e-9, limit=200)
    return val


def test_cone_quadrature_matches_closed_form_without_medium():
    # sigma = 0: the inner integral is the solid angle 2 pi (1 - cos_max).
    x = np.array([0.5, 0.5, 0.5])
    ut, wt, ph, wph = cone_nodes(24, 48)
    centre, r = np.array([0.5, 1.9, 0.5]), 0.6
    d = np.linalg.norm(centre - x)
    cos_max = math.sqrt(1 - (r / d) ** 2)
    assert abs((1 - cos_max) * wt.sum() * wph.sum() - 2 * math.pi * (1 - cos_max)) < 1e-12


@pytest.mark.parametrize("strategy", [NEE, UNIFORM])
def test_single_scattering_sphere_light_matches_quadrature(ora, strategy):
    sigma, albedo, le = 2.0, 0.8, 10.0
    centre, radius = [0.5, 1.9, 0.5], 0.6
    vol = with_spheres(homogeneous(4, sigma, [[albedo] * 3 + [1.0]] * 2, np.zeros((0, 6))),
                       [centre + [radius, le, le, le]])
    cam = centre_pixel_cam()
    n = 200_000
    out = ora.trace(vol, cam, seed=13, frame=0, spp=n, max_bounces=1, K=1, C=math.inf,
                    records=False, second_moment=True, strategy=strategy)
    mean = float(out["targets"][0, 0, 0, 0])
    var = float(out["targets_sq"][0, 0, 0, 0]) - mean * mean
    o, w = primary_ray(cam)
    exact = single_scatter_sphere(o, w, sigma, albedo, centre, radius, le)
    assert exact > 0
    assert abs(mean - exact) <= 3 * math.sqrt(var / n), (strategy, mean, exact, math.sqrt(var / n))


def occluding_pair():
    # A black sphere between the volume and a bright one: their cones overlap from every
    # point of the cube, so next-event estimation has to drop the blocked samples.
    return [[0.5, 0.5, -0.6, 0.3, 0.0, 0.0, 0.0],
            [0.45, 0.55, -1.4, 0.6, 12.0, 9.0, 6.0]]


@pytest.mark.parametrize("spheres,C", [("synth", math.inf), ("synth", 0.5),
                                       ("occluding", math.inf)])
def test_estimators_agree(ora, spheres, C):
    wl = synth.workload("tiny")
    vol = wl.volume()
    vol.lights = np.zeros((0, 6), np.float32)
    vol = with_spheres(vol, synth.sphere_lights(2, radius=0.3, radiance=20.0)
                       if spheres == "synth" else occluding_pair())
    cam = wl.camera().crop(40, 40, 48, 48)
    spp, K = 256, 3
    res = {}
    for strategy in (NEE, UNIFORM):
        out = ora.trace(vol, cam, seed=31, frame=0, spp=spp, max_bounces=K, K=K, C=C,
                        records=False, second_moment=True, strategy=strategy)
        # One level per path: the per-pixel total over levels is the path radiance, and its
        # second moment the sum of the levels' second moments.
        m = out["targets"].astype(np.float64).sum(0)
        v = out["targets_sq"].astype(np.float64).sum(0) - m * m
        res[strategy] = (m.sum(axis=(0, 1)), v.sum(axis=(0, 1)) / spp)   # per channel
    (m1, v1), (m2, v2) = res[NEE], res[UNIFORM]
    assert (m1 > 0).all()
    z = (m1 - m2) / np.sqrt(v1 + v2)
    assert np.all(np.abs(z) <= 3), z
    # MIS lowers the variance against phase sampling alone.
    assert (v1 < v2).all()


def test_small_sphere_is_a_point_light(ora):
    sigma, albedo = 2.5, 0.7
    c = [1.6, 1.4, -0.5]
    r, le = 0.01, 2.0e4
    intensity = le * math.pi * r * r
    tf = [[albedo] * 3 + [1.0]] * 2
    cam = centre_pixel_cam()
    n = 100_000
    sph = with_spheres(homogeneous(4, sigma, tf, np.zeros((0, 6))), [c + [r, le, le, le]])
    pt = homogeneous(4, sigma, tf, [c + [intensity] * 3])
    a = ora.trace(sph, cam, seed=5, frame=0, spp=n, max_bounces=2, K=2, C=math.inf,
                  records=False, second_moment=True)
    b = ora.trace(pt, cam, seed=5, frame=0, spp=n, max_bounces=2, K=2, C=math.inf,
                  records=False, second_moment=True)
    for lvl in range(2):
        ma, mb = float(a["targets"][lvl, 0, 0, 0]), float(b["targets"][lvl, 0, 0, 0])
        va = float(a["targets_sq"][lvl, 0, 0, 0]) - ma * ma
        vb = float(b["targets_sq"][lvl, 0, 0, 0]) - mb * mb
        # O((r/d)^2) ~ 1e-5 relative geometry difference, far below the noise.
        assert abs(ma - mb) <= 3 * math.sqrt((va + vb) / n), (lvl, ma, mb)


def test_degenerate_light_setups(ora):
    wl = synth.workload("tiny")
    cam = wl.camera()
    vol = wl.volume()
    assert vol.lights.shape[0] >= 1 and vol.spheres.shape[0] == 0
    out = ora.trace(vol, cam, seed=2, frame=0, spp=1, max_bounces=3, K=3, C=0.5, strategy=UNIFORM)
    assert not out["targets"].any() and (out["n"] > 0).any()
    vol.lights = np.zeros((0, 6), np.float32)
    dark = synth.sphere_lights(2)
    dark[:, 4:] = 0.0
    vol = with_spheres(vol, dark)
    for strategy in (NEE, UNIFORM):
        out = ora.trace(vol, cam, seed=2, frame=0, spp=1, max_bounces=3, K=3, C=0.5,
                        strategy=strategy)
        assert not out["targets"].any()


def test_point_lights_unchanged_by_area_light_code(ora):
    """Without area lights the path stops at the last vertex as before: the kind counts
    reach MAXDEPTH and no extra random numbers are drawn (records identical with an explicit
    empty sphere list)."""
    wl = synth.workload("tiny")
    cam = wl.camera().crop(0, 0, 64, 64)
    vol = wl.volume()
    a = ora.trace(vol, cam, seed=3, frame=1, spp=1, max_bounces=2, K=2, C=0.5)
    vol = with_spheres(vol, np.zeros((0, 7)))
    b = ora.trace(vol, cam, seed=3, frame=1, spp=1, max_bounces=2, K=2, C=0.5)
    assert np.array_equal(a["targets"], b["targets"])
    assert (a["kind"] == 2).any()


def test_escape_to_light_after_last_vertex(ora):
    """With an area light the continuation after the B-th vertex still runs: some paths that
    reached B vertices end as escapes (kind 1) with radiance."""
    wl = synth.workload("tiny")
    vol = wl.volume()
    vol.lights = np.zeros((0, 6), np.float32)
    vol = with_spheres(vol, synth.sphere_lights(2, radius=0.5))
    cam = wl.camera()
    out = ora.trace(vol, cam, seed=8, frame=0, spp=1, max_bounces=1, K=1, C=math.inf,
                    strategy=UNIFORM)
    hit = (out["n"] == 1) & (out["kind"] == 1) & (out["L"].max(-1) > 0)
    assert hit.any()
    assert ((out["kind"] == 2) | (out["kind"] == 1) | (out["n"] == 0)).all()
