"""Pins of the cache-initialisation oracle (Method: "Cache Initialization", Eq. 2) against
closed forms, invariants and a brute-force neighbour search."""
import numpy as np
import pytest

import oracle
import synth
from oracle import init as oinit


def box_volume(lo=0.4, hi=0.6, res=32, density=10.0):
    """Density `density` in the voxels whose centres lie in [lo, hi]^3, zero elsewhere."""
    c = (np.arange(res) + 0.5) / res
    inside = (c >= lo) & (c <= hi)
    d = np.zeros((res, res, res), np.float32)
    d[np.ix_(inside, inside, inside)] = density
    tf = np.array([[0.3, 0.6, 0.9, 0.0], [0.8, 0.2, 0.5, 1.0]], np.float32)
    return synth.Volume(d, float(density), tf, np.zeros((0, 6), np.float32))


def test_points_lie_in_the_support_and_carry_their_albedo():
    vol = box_volume()
    pos, alb, att = oinit.points(vol, 2000, seed=11)
    res = vol.density.shape[0]
    margin = 1.0 / res            # trilinear support reaches one voxel beyond the centres
    assert np.all(pos >= 0.4 - margin) and np.all(pos <= 0.6 + margin)
    d = np.zeros(len(pos), np.float32)
    oracle.lib().ora_density_at(oracle._p(vol.density), res, res, res, oracle._p(pos),
                                len(pos), oracle._p(d))
    assert np.all(d > 0.0)
    rgba = np.zeros((len(pos), 4), np.float32)
    oracle.lib().ora_tf_at(oracle._p(vol.tf), vol.tf.shape[0], oracle.ctypes.c_float(vol.density_max),
                           oracle._p(d), len(pos), oracle._p(rgba))
    assert np.array_equal(alb, rgba[:, :3])
    # A ray through a uniform point of the cube hits the small box rarely: several attempts.
    assert att.min() >= 1 and att.mean() > 2.0


def test_dense_medium_interacts_at_the_entry_face():
    # sigma = 1e4 per unit length: the first interaction lies within ~1e-3 of where the ray
    # enters the cube, i.e. on its surface.
    d = np.full((8, 8, 8), 1e4, np.float32)
    tf = np.array([[1, 1, 1, 1.0], [1, 1, 1, 1.0]], np.float32)
    vol = synth.Volume(d, 1e4, tf, np.zeros((0, 6), np.float32))
    pos, _, att = oinit.points(vol, 5000, seed=3)
    face = np.minimum(pos, 1.0 - pos).min(axis=1)
    assert np.all(att == 1)
    assert np.percentile(face, 99) < 2e-3
    # Entry faces are hit in proportion to... every face is used.
    for a in range(3):
        assert (pos[:, a] < 1e-2).sum() > 300 and (pos[:, a] > 1 - 1e-2).sum() > 300


def test_points_are_deterministic_per_seed():
    vol = box_volume()
    a, _, _ = oinit.points(vol, 300, seed=5)
    b, _, _ = oinit.points(vol, 300, seed=5)
    c, _, _ = oinit.points(vol, 300, seed=6)
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_knn_matches_brute_force():
    rng = np.random.default_rng(0)
    p = rng.random((600, 3)).astype(np.float32)
    d = np.sqrt(((p[:, None, :].astype(np.float64) - p[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    want = np.sort(d, axis=1)[:, :3].mean(axis=1)
    assert np.allclose(oinit.knn_mean3(p), want, rtol=1e-12, atol=0)


def test_eq2_lattice_is_half_the_spacing():
    h = 0.05
    g = np.arange(6) * h
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    m = oinit.knn_mean3(p)
    assert np.allclose(m, h, rtol=1e-12)
    s = oinit.eq2_scales(m)
    assert np.allclose(s, h / 2, rtol=1e-12)


def test_eq2_caps_outliers_at_two_sigma():
    h = 0.05
    g = np.arange(6) * h
    p = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    far = np.array([[3.0, 3.0, 3.0], [3.2, 3.0, 3.0], [3.0, 3.3, 3.0], [3.0, 3.0, 3.4]])
    p = np.concatenate([p, far])
    m = oinit.knn_mean3(p)
    s = oinit.eq2_scales(m)
    cap = m.mean() + 2 * m.std()
    out = m > cap
    assert out.sum() == 4                       # the four far points exceed the cap
    assert np.all(s[out] == cap / 2)            # ... and are capped at mu + 2 sigma
    assert np.all(s[~out] == m[~out] / 2)       # everyone else is halved
    assert np.allclose(s[:216], h / 2)


def test_level_sizes_follow_the_halving_schedule():
    # Sum_{i=0}^{K} N / 2^i with the paper's N = 300k and three levels.
    assert oinit.level_sizes(300_000, 3) == [300_000, 150_000, 75_000]
    assert sum(oinit.level_sizes(300_000, 3)) * 14 * 4 == 29_400_000


def test_cache_levels_shapes_and_invariants():
    wl = synth.workload("tiny")
    vol = wl.volume()
    lv = oinit.cache_levels(vol, 4000, 3, seed=9)
    assert [l["pos"].shape[0] for l in lv] == [4000, 2000, 1000]
    for l in lv:
        assert np.all(l["rot"][:, 0] == 1) and np.all(l["rot"][:, 1:] == 0)
        assert np.all(l["log_scale"][:, 0] == l["log_scale"][:, 1])
        assert np.allclose(1 / (1 + np.exp(-l["opacity_logit"])), 0.1)
    # Sparser levels have larger Gaussians.
    med = [np.median(l["scale"]) for l in lv]
    assert med[0] < med[1] < med[2]
