"""GSCache CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously-correct CPU statement of what the GSCache hot path computes, written
independently of the HIP implementation (no shared code, headers, constants or helpers; this
package never imports `paper_2507_19718_amd`, and the product never imports this package).
Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of `bench.py` may use it.

Parts and what they follow (sections of the paper, arXiv 2507.19718):
  * `liboracle.so` (gsc_oracle.cpp): Philox4x32-10, portable exp/log/sincos, the volume path
    tracer with NEE, Algorithm 1 and Eq. 3 (Method: path termination heuristics, cache
    sampling, cache training), fp32 projection, binning by plain sort, brute-force forward
    splatting (Method: a path space radiance cache; the 3D Gaussian splatting rasteriser).
  * `loss_grad` -- Eq. 4 (HDR loss) and plain L2 (Method: optimization and hyperparameters).
  * `adamw_step` -- AdamW (Method: regularization), learning-rate schedule Eq. 5.
  * `composite` -- natural / early termination cache use (Method: natural path termination,
    early path termination, cascaded cache radiance importance sampling, Eq. 3).
  * `backward.py` -- the exact fp64 gradient of the forward (reverse mode through torch
    autograd on CPU), for the blended sets the fp32 forward decided.

Parity pins: see tests/test_oracle_*.py.  The composite is "parity unpinned" against truth
(biased by design); it is pinned only between the oracle and the GPU path.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsc_oracle.cpp")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

KIND_ESCAPE0, KIND_ESCAPE, KIND_MAXDEPTH, KIND_EARLY = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (fp32 in program order, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = ctypes.CDLL(_LIB_PATH)
        _lib.ora_ratio_tracking_mean.restype = ctypes.c_double
        _lib.ora_bin_level.restype = ctypes.c_int64
        _lib.ora_num_threads.restype = ctypes.c_int
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def num_threads() -> int:
    return int(lib().ora_num_threads())


# ------------------------------------------------------------------------------------------
# RNG and transcendentals
# ------------------------------------------------------------------------------------------
def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ora_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def path_uniforms(seed: int, pixel: int, sample: int, frame: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.float32)
    lib().ora_path_uniforms(ctypes.c_uint64(seed), ctypes.c_uint32(pixel), ctypes.c_uint32(sample),
                            ctypes.c_uint32(frame), ctypes.c_int(n), _p(out))
    return out


def expf(x) -> np.ndarray:
    x = _f32(x).ravel()
    y = np.empty_like(x)
    lib().ora_expf(_p(x), _p(y), ctypes.c_int64(x.size))
    return y


def logf(x) -> np.ndarray:
    x = _f32(x).ravel()
    y = np.empty_like(x)
    lib().ora_logf(_p(x), _p(y), ctypes.c_int64(x.size))
    return y


def sincosf(x):
    x = _f32(x).ravel()
    s, c = np.empty_like(x), np.empty_like(x)
    lib().ora_sincosf(_p(x), _p(s), _p(c), ctypes.c_int64(x.size))
    return s, c


# ------------------------------------------------------------------------------------------
# Volume
# ------------------------------------------------------------------------------------------
def density_at(density: np.ndarray, points: np.ndarray) -> np.ndarray:
    d = _f32(density)
    p = _f32(points).reshape(-1, 3)
    out = np.empty(p.shape[0], dtype=np.float32)
    nz, ny, nx = d.shape
    lib().ora_density_at(_p(d), nx, ny, nz, _p(p), ctypes.c_int64(p.shape[0]), _p(out))
    return out


def tf_at(tf: np.ndarray, dmax: float, d: np.ndarray) -> np.ndarray:
    tf = _f32(tf)
    d = _f32(d).ravel()
    out = np.empty((d.size, 4), dtype=np.float32)
    lib().ora_tf_at(_p(tf), tf.shape[0], ctypes.c_float(dmax), _p(d), ctypes.c_int64(d.size), _p(out))
    return out


def ratio_tracking_mean(vol, o, w, tmax: float, seed: int, n: int) -> float:
    d = _f32(vol.density)
    nz, ny, nx = d.shape
    tf = _f32(vol.tf)
    o, w = _f32(o), _f32(w)
    return float(lib().ora_ratio_tracking_mean(_p(d), nx, ny, nz, ctypes.c_float(vol.density_max),
                                               _p(tf), tf.shape[0], _p(o), _p(w),
                                               ctypes.c_float(tmax), ctypes.c_uint64(seed), n))


def _cam_args(cam):
    R = _f32(cam.R)
    t = _f32(cam.t)
    intr = np.array([cam.fx, cam.fy, cam.cx, cam.cy], dtype=np.float32)
    win = np.array([cam.full_w, cam.full_h, cam.x0, cam.y0, cam.w, cam.h], dtype=np.int32)
    return (R, t, intr, win), [_p(R), _p(t), _p(intr), _p(win), ctypes.c_float(cam.znear)]


# ------------------------------------------------------------------------------------------
# Tracer
# ------------------------------------------------------------------------------------------
STRATEGY_NEE, STRATEGY_UNIFORM = 0, 1


def trace(vol, cam, seed: int, frame: int, spp: int, max_bounces: int, K: int, C: float = 0.5,
          eps: float = 0.0, records: bool = True, second_moment: bool = False,
          kinds: bool = False, strategy: int = STRATEGY_NEE):
    """Per-path-length targets [K][h][w][3] (mean over spp), optional second moments and
    per-path records (L[3], beta, n, kind): [h][w] for spp == 1, [spp][h][w] otherwise.
    C = inf disables Algorithm 1.
    strategy: next-event estimation with MIS for area lights (0) or phase sampling only (1)."""
    d = _f32(vol.density)
    nz, ny, nx = d.shape
    tf, lights = _f32(vol.tf), _f32(vol.lights).reshape(-1, 6)
    spheres = getattr(vol, "spheres", None)
    spheres = _f32(np.zeros((0, 7)) if spheres is None else spheres).reshape(-1, 7)
    keep, cargs = _cam_args(cam)
    H, W = cam.h, cam.w
    targets = np.zeros((K, H, W, 3), dtype=np.float32)
    tsq = np.zeros_like(targets) if second_moment else None
    rec = np.zeros((spp, H, W, 5), dtype=np.uint32) if records else None
    stats = np.zeros(2, dtype=np.uint32)
    kc = np.zeros((H, W, 4), dtype=np.uint32) if kinds else None
    c_inf = 1 if math.isinf(C) else 0
    lib().ora_trace(_p(d), nx, ny, nz, ctypes.c_float(vol.density_max), _p(tf), tf.shape[0],
                    _p(lights), lights.shape[0], _p(spheres), spheres.shape[0], int(strategy),
                    *cargs, ctypes.c_uint64(seed),
                    ctypes.c_uint32(frame), ctypes.c_uint32(spp), ctypes.c_uint32(max_bounces),
                    ctypes.c_uint32(K), ctypes.c_float(0.0 if c_inf else C), ctypes.c_int(c_inf),
                    ctypes.c_float(eps), _p(targets), _p(tsq), _p(rec), _p(stats), _p(kc))
    out = dict(targets=targets, path_vertices=int(stats[0]) | (int(stats[1]) << 32))
    if second_moment:
        out["targets_sq"] = tsq
    if kinds:
        out["kind_counts"] = kc
    if records:
        if spp == 1:
            rec = rec[0]
        out["L"] = rec[..., :3].copy().view(np.float32)
        out["beta"] = rec[..., 3].copy().view(np.float32)
        out["n"] = (rec[..., 4] & 0xFFFF).astype(np.int32)
        out["kind"] = (rec[..., 4] >> 16).astype(np.int32)
    return out


# ------------------------------------------------------------------------------------------
# Projection, binning, forward
# ------------------------------------------------------------------------------------------
def project(g, cam) -> dict:
    """fp32 projection of one level (bit-exact contract)."""
    n = g.n
    keep, cargs = _cam_args(cam)
    arrs = [_f32(a) for a in (g.pos, g.rot, g.log_scale, g.opacity_logit)]
    screen = np.zeros((n, 6), dtype=np.float32)
    depth = np.zeros(n, dtype=np.float32)
    window = np.zeros((n, 4), dtype=np.int32)
    rect = np.zeros((n, 4), dtype=np.int32)
    tiles = np.zeros(n, dtype=np.uint32)
    radius = np.zeros(n, dtype=np.float32)
    lib().ora_project(*[_p(a) for a in arrs], ctypes.c_int64(n), *cargs, _p(screen), _p(depth),
                      _p(window), _p(rect), _p(tiles), _p(radius))
    return dict(screen=screen, depth=depth, window=window, rect=rect, tiles=tiles, radius=radius,
                culled=(tiles == 0))


def tiles_x(cam) -> int:
    return (cam.w + 15) // 16


def tiles_y(cam) -> int:
    return (cam.h + 15) // 16


def bin_levels(projs: Sequence[dict], cam) -> dict:
    """Keys, values and per-tile ranges over all levels in one key space: level l's tiles
    start at l * TX * TY."""
    TX, TY = tiles_x(cam), tiles_y(cam)
    keys_all, vals_all = [], []
    for l, pr in enumerate(projs):
        n = pr["depth"].shape[0]
        total = lib().ora_bin_level(_p(pr["depth"]), _p(pr["rect"]), _p(pr["tiles"]),
                                    ctypes.c_int64(n), TX, ctypes.c_uint32(l * TX * TY), None, None)
        keys = np.zeros(total, dtype=np.uint64)
        vals = np.zeros(total, dtype=np.uint32)
        lib().ora_bin_level(_p(pr["depth"]), _p(pr["rect"]), _p(pr["tiles"]), ctypes.c_int64(n), TX,
                            ctypes.c_uint32(l * TX * TY), _p(keys), _p(vals))
        keys_all.append(keys)
        vals_all.append(vals)
    keys = np.concatenate(keys_all) if keys_all else np.zeros(0, np.uint64)
    vals = np.concatenate(vals_all) if vals_all else np.zeros(0, np.uint32)
    n_tiles = TX * TY * len(projs)
    ranges = np.zeros((n_tiles, 2), dtype=np.uint64)
    lib().ora_tile_ranges(_p(keys), ctypes.c_int64(keys.size), ctypes.c_int64(n_tiles), _p(ranges))
    return dict(keys=keys, values=vals, ranges=ranges)


def forward(pr: dict, rgb: np.ndarray, cam, lists: bool = False) -> dict:
    """Brute-force fp32 forward of one level over the camera's render window."""
    n = pr["depth"].shape[0]
    H, W = cam.h, cam.w
    win = np.array([cam.full_w, cam.full_h, cam.x0, cam.y0, cam.w, cam.h], dtype=np.int32)
    rgb = _f32(rgb)
    image = np.zeros((H, W, 3), dtype=np.float32)
    final_T = np.zeros((H, W), dtype=np.float32)
    last_id = np.zeros((H, W), dtype=np.int32)
    n_blend = np.zeros((H, W), dtype=np.int32)
    boundary = np.zeros((H, W), dtype=np.uint8)
    tests = np.zeros(1, dtype=np.int64)
    contrib = np.zeros(1, dtype=np.int64)
    args = [_p(pr["screen"]), _p(pr["depth"]), _p(pr["window"]), _p(pr["tiles"]), _p(rgb),
            ctypes.c_int64(n), _p(win), _p(image), _p(final_T), _p(last_id), _p(n_blend),
            _p(boundary)]
    lib().ora_forward(*args, None, None, _p(tests), _p(contrib))
    out = dict(image=image, final_T=final_T, last_id=last_id, n_blend=n_blend,
               boundary=boundary.astype(bool), pair_tests=int(tests[0]),
               contributing=int(contrib[0]))
    if lists:
        off = np.zeros(H * W + 1, dtype=np.int64)
        off[1:] = np.cumsum(n_blend.ravel())
        ids = np.zeros(int(off[-1]), dtype=np.int32)
        lib().ora_forward(*args, _p(off), _p(ids), None, None)
        out["list_off"] = off
        out["list_ids"] = ids
    return out


# ------------------------------------------------------------------------------------------
# Loss (Eq. 4 and L2), composite (Eq. 3), AdamW + Eq. 5
# ------------------------------------------------------------------------------------------
def loss_grad(images: np.ndarray, targets: np.ndarray, hdr: bool):
    """Per level, mean over the 3*w*h elements, summed over levels.  HDR (Eq. 4):
    (y - x)^2 / (sg(max(y, 0)) + 0.01)^2 with y the prediction and x the noisy target.
    Returns (loss, dL/dimages) in fp64."""
    y = images.astype(np.float64)
    x = targets.astype(np.float64)
    K = y.shape[0]
    k = float(np.prod(y.shape[1:]))
    diff = y - x
    if hdr:
        den = (np.maximum(y, 0.0) + 0.01) ** 2
        loss = float(np.sum(diff * diff / den) / k)
        grad = 2.0 * diff / den / k
    else:
        loss = float(np.sum(diff * diff) / k)
        grad = 2.0 * diff / k
    return loss, grad


def composite(n: np.ndarray, kind: np.ndarray, L: np.ndarray, beta: np.ndarray,
              cache: np.ndarray) -> np.ndarray:
    """Per pixel: EARLY -> max(cache[l], 0) / beta; natural termination with n >= 1 -> the
    unbiased path radiance when its luminance is positive, else max(cache[l], 0) / beta;
    no interaction -> 0.  l = min(n, K) - 1.  fp32, elementwise.  With a leading sample axis
    (records of several samples per pixel) the pixel is the mean of its samples' values,
    summed in sample order."""
    if n.ndim == 3:
        acc = np.zeros(n.shape[1:] + (3,), dtype=np.float32)
        for s in range(n.shape[0]):
            acc = (acc + composite(n[s], kind[s], L[s], beta[s], cache)).astype(np.float32)
        return (acc / np.float32(n.shape[0])).astype(np.float32)
    K = cache.shape[0]
    H, W = n.shape
    out = np.zeros((H, W, 3), dtype=np.float32)
    lvl = np.clip(np.minimum(n, K) - 1, 0, K - 1)
    cv = np.maximum(cache[lvl, np.arange(H)[:, None], np.arange(W)[None, :]], np.float32(0))
    lum = (np.float32(0.2126) * L[..., 0] + np.float32(0.7152) * L[..., 1]) + np.float32(0.0722) * L[..., 2]
    from_cache = cv / beta[..., None]
    use_cache = (kind == KIND_EARLY) | ((n >= 1) & (lum <= 0))
    out = np.where(use_cache[..., None], from_cache, L).astype(np.float32)
    out[n == 0] = 0
    return out


def lr_schedule(lr0: float, t_view: int) -> float:
    """Eq. 5: eta_t = eta_0 / (1 + ln t), t >= 1 frames in the current viewport."""
    return lr0 / (1.0 + math.log(max(t_view, 1)))


def adamw_step(param: np.ndarray, m: np.ndarray, v: np.ndarray, grad: np.ndarray, lr: float,
               beta1: float, beta2: float, eps: float, weight_decay: float, step: int):
    """One AdamW step (decoupled weight decay), fp32, every operation separately rounded:
    m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;  p = p (1 - lr wd);
    p = p - s1 m / (sqrt(v) s2 + eps) with s1 = lr/(1-b1^t), s2 = 1/sqrt(1-b2^t) from fp64."""
    f = np.float32
    b1, b2 = f(beta1), f(beta2)
    omb1, omb2 = f(1.0 - beta1), f(1.0 - beta2)
    s1 = f(lr / (1.0 - beta1 ** step))
    s2 = f(1.0 / math.sqrt(1.0 - beta2 ** step))
    wdf = f(1.0 - lr * weight_decay)
    g = grad.astype(np.float32)
    m_new = (b1 * m.astype(f)) + (omb1 * g)
    v_new = (b2 * v.astype(f)) + (omb2 * (g * g))
    p = param.astype(f) * wdf
    den = (np.sqrt(v_new) * s2) + f(eps)
    p = p - (s1 * m_new) / den
    return p.astype(f), m_new.astype(f), v_new.astype(f)
