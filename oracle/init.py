"""Cache initialisation oracle (Method: "Cache Initialization", Eq. 2) -- TEST INFRASTRUCTURE.

  * `points` -- N first interactions of random rays with the volume (delta tracking), with
    their albedo; the C++ sampler `ora_init_points` follows the section's description and the
    stream layout of the library's sampler (one Philox stream per point and attempt).
  * `knn_mean3` -- for every point the mean Euclidean distance to its 3 nearest other points
    (scipy's k-d tree serves as the library routine of this step).
  * `eq2_scales` -- Eq. 2: s_i = min(mu + 2 sigma, mean 3-NN distance_i) / 2, mu and sigma
    the mean and standard deviation of the mean 3-NN distances over the level's points.
  * `cache_levels` -- the levels: level l keeps the first floor(N / 2^l) points (the points are
    i.i.d., so a prefix is a uniform sub-sample), isotropic scale from Eq. 2, identity
    rotation, albedo as colour, opacity 0.1 (the 3D Gaussian splatting initial opacity).
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import lib, _p

INIT_OPACITY = 0.1


def points(vol, n: int, seed: int, max_attempts: int = 4096):
    """Returns (pos [n, 3] float32, albedo [n, 3] float32, attempts [n] int32)."""
    d = np.ascontiguousarray(vol.density, np.float32)
    nz, ny, nx = d.shape
    tf = np.ascontiguousarray(vol.tf, np.float32)
    pos = np.zeros((n, 3), np.float32)
    alb = np.zeros((n, 3), np.float32)
    att = np.zeros(n, np.int32)
    rc = lib().ora_init_points(_p(d), ctypes.c_int(nx), ctypes.c_int(ny), ctypes.c_int(nz),
                               ctypes.c_float(vol.density_max), _p(tf), ctypes.c_int(tf.shape[0]),
                               ctypes.c_int64(n), ctypes.c_uint64(seed), ctypes.c_int(max_attempts),
                               _p(pos), _p(alb), _p(att))
    if rc != 0:
        raise RuntimeError("no interaction within the attempt limit (empty volume?)")
    return pos, alb, att


def knn_mean3(pos: np.ndarray) -> np.ndarray:
    """Mean distance to the 3 nearest other points, float64."""
    from scipy.spatial import cKDTree
    p = np.asarray(pos, np.float64)
    if p.shape[0] < 4:
        raise ValueError("need at least 4 points")
    dist, _ = cKDTree(p).query(p, k=4)
    return dist[:, 1:].mean(axis=1)


def eq2_scales(mean3: np.ndarray) -> np.ndarray:
    """Eq. 2 in float64."""
    m = np.asarray(mean3, np.float64)
    mu = m.mean()
    sigma = m.std()
    return np.minimum(mu + 2.0 * sigma, m) / 2.0


def level_sizes(n: int, K: int):
    return [n >> l for l in range(K)]


def cache_levels(vol, n: int, K: int, seed: int):
    pos, alb, _ = points(vol, n, seed)
    out = []
    for nl in level_sizes(n, K):
        p = pos[:nl]
        s = eq2_scales(knn_mean3(p))
        out.append(dict(pos=p.copy(), rot=np.tile(np.array([1, 0, 0, 0], np.float32), (nl, 1)),
                        log_scale=np.repeat(np.log(s)[:, None], 3, axis=1),
                        rgb=alb[:nl].copy(),
                        opacity_logit=np.full(nl, math.log(INIT_OPACITY / (1.0 - INIT_OPACITY))),
                        mean3=knn_mean3(p), scale=s))
    return out
