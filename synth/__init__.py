"""Seeded synthetic inputs for the GSCache hot path.

This module only *draws inputs*: procedural density grids, transfer functions, point lights,
Gaussian cache levels, orbit cameras and request arrival logs.  It holds none of the method's
arithmetic (no tracing, projection, blending, loss or optimiser step), so both the CPU oracle
(`oracle/`) and the HIP path (`paper_2507_19718_amd/`) may take their inputs from here.

The paper measures on six real volumes with fixed transfer functions and volume-initialised
caches (Evaluation, "Datasets" and "System Specifications and Setup").  None of those are
available, so the volumes here are procedural stand-ins whose sizes bracket the paper's
(64^3 ... 1024^3 fp32), lit by point lights, with randomly initialised Gaussian levels.

Every generator is driven by numpy's Philox bit generator keyed by (seed, fixture id), so the
same seed yields byte-identical inputs on every machine running this image.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Camera", "Volume", "Gaussians", "Workload",
    "rng", "orbit_camera", "crop_camera", "blob_volume", "fbm_volume", "slab_volume",
    "transfer_function", "point_lights", "sphere_lights", "tiny_gaussians", "random_gaussians",
    "frustum_gaussians", "workload", "WORKLOADS", "poisson_requests",
]

# Fixture ids: one independent Philox stream per kind of input.
_FID = {"volume": 1, "tf": 2, "lights": 3, "gauss": 4, "camera": 5, "arrivals": 6, "slabs": 7,
        "misc": 8}


def rng(seed: int, kind: str, index: int = 0) -> np.random.Generator:
    """A numpy Generator over Philox4x64-10 keyed by (seed, fixture id, index)."""
    key = np.array([seed & 0xFFFFFFFFFFFFFFFF,
                    ((_FID[kind] << 32) | (index & 0xFFFFFFFF)) & 0xFFFFFFFFFFFFFFFF],
                   dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


# --------------------------------------------------------------------------------------------
# Cameras
# --------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    """Pinhole camera.  R is world->camera (row-major 3x3), camera axes x right, y down,
    z forward.  Intrinsics are in full-frame pixels; pixel i spans [i, i+1).  (x0, y0, w, h)
    is the render window inside the full frame."""
    R: np.ndarray          # (9,) float32
    t: np.ndarray          # (3,) float32
    fx: float
    fy: float
    cx: float
    cy: float
    full_w: int
    full_h: int
    x0: int = 0
    y0: int = 0
    w: int = 0
    h: int = 0
    znear: float = 0.2

    def __post_init__(self):
        self.R = np.ascontiguousarray(self.R, dtype=np.float32).reshape(9)
        self.t = np.ascontiguousarray(self.t, dtype=np.float32).reshape(3)
        self.fx, self.fy = float(np.float32(self.fx)), float(np.float32(self.fy))
        self.cx, self.cy = float(np.float32(self.cx)), float(np.float32(self.cy))
        if self.w == 0:
            self.w = self.full_w
        if self.h == 0:
            self.h = self.full_h

    def crop(self, x0: int, y0: int, w: int, h: int) -> "Camera":
        return dataclasses.replace(self, x0=x0, y0=y0, w=w, h=h)


def orbit_camera(width: int, height: int, azimuth_deg: float, elevation_deg: float = 20.0,
                 radius: float = 1.8, fov_y_deg: float = 45.0,
                 target=(0.5, 0.5, 0.5)) -> Camera:
    """Camera on an orbit around `target`, world +y up, looking at the target."""
    c = np.asarray(target, dtype=np.float64)
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    eye = c + radius * np.array([math.cos(el) * math.sin(az), math.sin(el),
                                 math.cos(el) * math.cos(az)])
    fwd = c - eye
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = -np.cross(right, fwd)
    R = np.stack([right, down, fwd])
    t = -R @ eye
    f = height / (2.0 * math.tan(math.radians(fov_y_deg) / 2.0))
    return Camera(R=R.reshape(9), t=t, fx=f, fy=f, cx=width / 2.0, cy=height / 2.0,
                  full_w=width, full_h=height)


def crop_camera(cam: Camera, x0: int, y0: int, w: int, h: int) -> Camera:
    return cam.crop(x0, y0, w, h)


# --------------------------------------------------------------------------------------------
# Volumes, transfer functions, lights
# --------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Volume:
    """Density grid [nz][ny][nx] fp32 over the unit cube, an RGBA transfer function with
    `P` control points at i/(P-1), point lights (xyz, rgb intensity) and spherical area
    lights (centre xyz, radius, rgb radiance)."""
    density: np.ndarray    # (nz, ny, nx) float32
    density_max: float
    tf: np.ndarray         # (P, 4) float32
    lights: np.ndarray     # (L, 6) float32
    spheres: np.ndarray = dataclasses.field(
        default_factory=lambda: np.zeros((0, 7), dtype=np.float32))   # (S, 7) float32

    @property
    def shape(self) -> Tuple[int, int, int]:
        return tuple(self.density.shape)


def _centres(n: int) -> np.ndarray:
    return ((np.arange(n, dtype=np.float64) + 0.5) / n)


def blob_volume(res: int, seed: int, n_blobs: int = 4, peak: float = 10.0) -> np.ndarray:
    """Sum of isotropic Gaussian blobs, centres U[0.2,0.8]^3, sigma U[0.05,0.15]."""
    g = rng(seed, "volume")
    centres = g.uniform(0.2, 0.8, size=(n_blobs, 3))
    sigmas = g.uniform(0.05, 0.15, size=n_blobs)
    x = _centres(res)
    d = np.zeros((res, res, res), dtype=np.float64)
    for c, s in zip(centres, sigmas):
        ex = np.exp(-(x - c[0]) ** 2 / (2 * s * s))
        ey = np.exp(-(x - c[1]) ** 2 / (2 * s * s))
        ez = np.exp(-(x - c[2]) ** 2 / (2 * s * s))
        d += peak * ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
    return d.astype(np.float32)


def _interp_axis(a: np.ndarray, res: int, cells: int, axis: int) -> np.ndarray:
    """Value-noise interpolation along one axis with smoothstep weights (separable)."""
    g = _centres(res) * cells
    i0 = np.minimum(np.floor(g).astype(np.int64), cells - 1)
    f = g - i0
    w = (3 * f * f - 2 * f * f * f).astype(np.float32)
    shape = [1] * a.ndim
    shape[axis] = res
    w = w.reshape(shape)
    lo = np.take(a, i0, axis=axis)
    hi = np.take(a, i0 + 1, axis=axis)
    return lo + w * (hi - lo)


def fbm_volume(res: int, seed: int, octaves: int = 6, threshold: float = 0.4,
               scale: float = 20.0) -> np.ndarray:
    """6-octave fBm of value noise (4*2^o lattice cells per axis at octave o), thresholded at
    `threshold` and scaled so that the maximum density is exactly `scale`.  The separable
    smoothstep interpolation runs on torch CPU threads (elementwise, so thread-count
    independent and deterministic)."""
    import torch
    g = rng(seed, "volume")
    acc = torch.zeros((res, res, res), dtype=torch.float32)
    total = 0.0

    def weights(cells):
        gg = _centres(res) * cells
        i0 = np.minimum(np.floor(gg).astype(np.int64), cells - 1)
        f = gg - i0
        return torch.from_numpy(i0), torch.from_numpy((3 * f * f - 2 * f * f * f).astype(np.float32))

    for o in range(octaves):
        cells = 4 * 2 ** o
        lat = torch.from_numpy(g.random(size=(cells + 1, cells + 1, cells + 1), dtype=np.float32))
        i0, w = weights(cells)
        a = lat.index_select(2, i0)
        a = a + w.view(1, 1, res) * (lat.index_select(2, i0 + 1) - a)          # x
        b = a.index_select(1, i0)
        a = b + w.view(1, res, 1) * (a.index_select(1, i0 + 1) - b)            # y
        amp = float(np.float32(0.5 ** o))
        for z0 in range(0, res, 64):                                           # z, in slabs
            z1 = min(res, z0 + 64)
            lo = a.index_select(0, i0[z0:z1])
            hi = a.index_select(0, i0[z0:z1] + 1)
            acc[z0:z1] += amp * (lo + w[z0:z1].view(-1, 1, 1) * (hi - lo))
        del a, b
        total += 0.5 ** o
    acc /= float(np.float32(total))
    m = float(acc.max())
    d = torch.clamp_min(acc - threshold, 0) * float(np.float32(scale / (m - threshold)))
    d = torch.clamp_max(d, scale)
    return d.numpy().astype(np.float32, copy=False)


def slab_volume(d: np.ndarray, seed: int, n_slabs: int = 32, density: float = 50.0) -> np.ndarray:
    """Adds thin sheet-like slabs (density max(d, 50)) to a grid, in place."""
    g = rng(seed, "slabs")
    res = d.shape[0]
    x = _centres(res).astype(np.float32)
    for _ in range(n_slabs):
        nrm = g.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        c = g.uniform(0.2, 0.8, size=3)
        half = g.uniform(0.0025, 0.01)
        rad = g.uniform(0.1, 0.3)
        # Voxels farther than rad + half from the centre along any axis cannot be in the slab
        # (|p - c|^2 = dist^2 + inplane^2 <= half^2 + rad^2), so only that box is visited.
        lo = np.searchsorted(x, c - (rad + half) - 2.0 / res)
        hi = np.searchsorted(x, c + (rad + half) + 2.0 / res)
        py = x[None, lo[1]:hi[1], None] - c[1]
        px = x[None, None, lo[0]:hi[0]] - c[0]
        for z0 in range(lo[2], hi[2], 32):
            z1 = min(hi[2], z0 + 32)
            pz = x[z0:z1, None, None] - c[2]
            dist = px * nrm[0] + py * nrm[1] + pz * nrm[2]
            inplane2 = px * px + py * py + pz * pz - dist * dist
            m = (np.abs(dist) <= half) & (inplane2 <= rad * rad)
            sl = d[z0:z1, lo[1]:hi[1], lo[0]:hi[0]]
            sl[m] = np.maximum(sl[m], np.float32(density))
    return d


def transfer_function(points: int, seed: int, index: int = 0) -> np.ndarray:
    """RGBA control points at i/(P-1): RGB ~ U[0.2, 1], A ~ U[0, 1] with A_0 = 0, then scaled
    so that max A = 1."""
    g = rng(seed, "tf", index)
    rgb = g.uniform(0.2, 1.0, size=(points, 3))
    a = g.uniform(0.0, 1.0, size=points)
    a[0] = 0.0
    a /= a.max()
    return np.concatenate([rgb, a[:, None]], axis=1).astype(np.float32)


def sphere_lights(n: int, radius: float = 0.25, radiance: float = 20.0,
                  centre=(0.5, 0.5, 0.5), distance: float = 1.5) -> np.ndarray:
    """Up to two spherical area lights (centre xyz, radius, rgb radiance) at the same fixed
    directions as `point_lights`, `distance` from the centre: outside the unit cube for
    radius < 0.6 at the default distance.  The second light is tinted."""
    c = np.asarray(centre, dtype=np.float64)
    dirs = [np.array([1.0, 1.5, -1.0]), np.array([-1.2, 0.8, 0.6])]
    tints = [np.array([1.0, 1.0, 1.0]), np.array([0.6, 0.8, 1.0])]
    out = []
    for i in range(n):
        d = dirs[i % 2] / np.linalg.norm(dirs[i % 2])
        out.append(np.concatenate([c + distance * d, [radius], radiance * tints[i % 2]]))
    return np.asarray(out, dtype=np.float32).reshape(-1, 7)


def point_lights(n: int, centre=(0.5, 0.5, 0.5), intensity: float = 3.0,
                 rotate_first_deg: float = 0.0) -> np.ndarray:
    """Up to two point lights at fixed directions 1.5 from the centre; radiant intensity
    4*pi*intensity per channel.  `rotate_first_deg` turns the first light about the vertical
    axis through the centre (a light move)."""
    c = np.asarray(centre, dtype=np.float64)
    dirs = [np.array([1.0, 1.5, -1.0]), np.array([-1.2, 0.8, 0.6])]
    out = []
    for i in range(n):
        d = dirs[i % 2] / np.linalg.norm(dirs[i % 2])
        if i == 0 and rotate_first_deg:
            a = math.radians(rotate_first_deg)
            d = np.array([math.cos(a) * d[0] + math.sin(a) * d[2], d[1],
                          -math.sin(a) * d[0] + math.cos(a) * d[2]])
        p = c + 1.5 * d
        out.append(np.concatenate([p, np.full(3, 4.0 * math.pi * intensity)]))
    return np.asarray(out, dtype=np.float32)


# --------------------------------------------------------------------------------------------
# Gaussian cache levels
# --------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Gaussians:
    """One cache level as SoA: pos [n][3], rot [n][4] (w,x,y,z), log_scale [n][3],
    rgb [n][3], opacity_logit [n].  14 fp32 per Gaussian."""
    pos: np.ndarray
    rot: np.ndarray
    log_scale: np.ndarray
    rgb: np.ndarray
    opacity_logit: np.ndarray

    def __post_init__(self):
        for f in ("pos", "rot", "log_scale", "rgb", "opacity_logit"):
            setattr(self, f, np.ascontiguousarray(getattr(self, f), dtype=np.float32))

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def arrays(self):
        return [self.pos, self.rot, self.log_scale, self.rgb, self.opacity_logit]

    def copy(self) -> "Gaussians":
        return Gaussians(*[a.copy() for a in self.arrays()])


def tiny_gaussians(n: int, seed: int, index: int = 0) -> Gaussians:
    """Means U[0,1]^3, isotropic scale 0.05, identity rotation, RGB 0.5, opacity 0.5."""
    g = rng(seed, "gauss", index)
    pos = g.uniform(0.0, 1.0, size=(n, 3))
    rot = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    ls = np.full((n, 3), math.log(0.05))
    rgb = np.full((n, 3), 0.5)
    op = np.zeros(n)
    return Gaussians(pos, rot, ls, rgb, op)


def random_gaussians(n: int, seed: int, index: int = 0, log_scale_mean: float = -3.0,
                     log_scale_std: float = 0.3) -> Gaussians:
    """Means U[0,1]^3, log-scales N(-3, 0.3) per axis, uniform random rotations (normalised
    N(0, I4)), RGB U[0,1], opacity U[0.1, 0.9] stored as a logit."""
    g = rng(seed, "gauss", index)
    pos = g.uniform(0.0, 1.0, size=(n, 3))
    ls = g.normal(log_scale_mean, log_scale_std, size=(n, 3))
    q = g.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    rgb = g.uniform(0.0, 1.0, size=(n, 3))
    o = g.uniform(0.1, 0.9, size=n)
    return Gaussians(pos, q, ls, rgb, np.log(o / (1 - o)))


def frustum_gaussians(cam: Camera, n: int, seed: int, depth=(1.3, 2.3), radius_px=(2.0, 8.0),
                      opacity=(0.1, 0.6), index: int = 0) -> Gaussians:
    """Gaussians whose means project inside the camera's crop window, at camera depth
    U[depth], with isotropic world scales chosen so that the screen sigma is U[radius_px]/3,
    random rotations and opacities U[opacity] (away from the 0.99 clamp)."""
    g = rng(seed, "gauss", index)
    R = cam.R.astype(np.float64).reshape(3, 3)
    t = cam.t.astype(np.float64)
    px = g.uniform(cam.x0 + 2, cam.x0 + cam.w - 2, size=n)
    py = g.uniform(cam.y0 + 2, cam.y0 + cam.h - 2, size=n)
    z = g.uniform(depth[0], depth[1], size=n)
    xc = np.stack([(px - cam.cx) / cam.fx * z, (py - cam.cy) / cam.fy * z, z], axis=1)
    pos = (xc - t) @ R          # R^T (xc - t)
    rpx = g.uniform(radius_px[0], radius_px[1], size=n)
    s = rpx / 3.0 * z / cam.fx
    ls = np.log(np.repeat(s[:, None], 3, axis=1)) + g.normal(0, 0.05, size=(n, 3))
    q = g.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    rgb = g.uniform(0.0, 1.0, size=(n, 3))
    o = g.uniform(opacity[0], opacity[1], size=n)
    return Gaussians(pos, q, ls, rgb, np.log(o / (1 - o)))


# --------------------------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    volume_res: int
    volume_kind: str          # "blobs" | "fbm" | "fbm_slabs"
    tf_points: int
    n_lights: int
    width: int
    height: int
    levels: Sequence[int]     # Gaussians per level
    gauss_kind: str           # "tiny" | "random"
    max_bounces: int
    loss: int                 # 0 = L2, 1 = HDR (Eq. 4)
    lr: Tuple[float, float, float, float, float]   # pos, rot, log_scale, rgb, opacity
    weight_decay: float
    azimuth: float = 30.0
    orbit_step_deg: float = 0.0
    C: float = 0.5
    seed: int = 0x47534300

    @property
    def K(self) -> int:
        return len(self.levels)

    def camera(self, frame: int = 0) -> Camera:
        return orbit_camera(self.width, self.height, self.azimuth + self.orbit_step_deg * frame)

    def volume(self, tf_index: int = 0, light_rot_deg: float = 0.0) -> Volume:
        if self.volume_kind == "blobs":
            d = blob_volume(self.volume_res, self.seed)
        else:
            d = fbm_volume(self.volume_res, self.seed)
            if self.volume_kind == "fbm_slabs":
                d = slab_volume(d, self.seed)
        tf = transfer_function(self.tf_points, self.seed, tf_index)
        return Volume(d, float(d.max()), tf, point_lights(self.n_lights,
                                                          rotate_first_deg=light_rot_deg))

    def gaussians(self) -> List[Gaussians]:
        out = []
        for i, n in enumerate(self.levels):
            if self.gauss_kind == "tiny":
                out.append(tiny_gaussians(n, self.seed, i))
            else:
                out.append(random_gaussians(n, self.seed, i))
        return out


P360_LR = (1.16e-3, 1e-3, 0.0, 1.25e-2, 1.5e-1)   # pos, rot, scale, colour, opacity

WORKLOADS = {
    # 64^3 blobs, 128^2, one level of 4096 Gaussians, L2 loss, all learning rates 1e-2.
    "tiny": Workload("tiny", 64, "blobs", 8, 1, 128, 128, [4096], "tiny", 3, 0,
                     (1e-2,) * 5, 0.0, seed=0x47534301),
    # 256^3 fBm, 1024^2, 3 levels x 200k, orbiting camera.
    "orbit1k": Workload("orbit1k", 256, "fbm", 16, 2, 1024, 1024, [200_000] * 3, "random", 3,
                        1, P360_LR, 1e-2, orbit_step_deg=3.6, seed=0x47534302),
    # 512^3 fBm, 1920x1080, 4 levels x 1M, static camera: the 1080p cache step.
    "fhd": Workload("fhd", 512, "fbm", 16, 2, 1920, 1080, [1_000_000] * 4, "random", 4, 1,
                    P360_LR, 1e-2, seed=0x47534303),
    # 1024^3 fBm + slabs, 3840x2160, 4 levels x 2M.
    "uhd": Workload("uhd", 1024, "fbm_slabs", 16, 2, 3840, 2160, [2_000_000] * 4, "random", 4,
                    1, P360_LR, 1e-2, orbit_step_deg=3.6, seed=0x47534304),
}


def workload(name: str, **overrides) -> Workload:
    return dataclasses.replace(WORKLOADS[name], **overrides)


# --------------------------------------------------------------------------------------------
# Serving: request arrival logs
# --------------------------------------------------------------------------------------------
SERVE_RESOLUTIONS = ((640, 360), (1280, 720), (1920, 1080))


def poisson_requests(rate_hz: float, duration_s: float, n_viewers: int, n_scenes: int,
                     seed: int, resolutions=SERVE_RESOLUTIONS) -> List[dict]:
    """A Poisson request log: each request picks a viewer uniformly; viewer v renders scene
    v mod n_scenes at a fixed resolution on its own orbit (random phase, elevation U[0,40] deg,
    radius U[1.8, 3.0], angular speed U[10, 60] deg/s)."""
    g = rng(seed, "arrivals")
    viewers = []
    for v in range(n_viewers):
        viewers.append(dict(scene=v % n_scenes,
                            res=resolutions[int(g.integers(len(resolutions)))],
                            phase=float(g.uniform(0, 360)), elev=float(g.uniform(0, 40)),
                            radius=float(g.uniform(1.8, 3.0)),
                            speed=float(g.uniform(10, 60))))
    t, out = 0.0, []
    while True:
        t += float(g.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        v = int(g.integers(n_viewers))
        vw = viewers[v]
        out.append(dict(t_arrival=t, viewer=v, scene=vw["scene"], width=vw["res"][0],
                        height=vw["res"][1], azimuth=vw["phase"] + vw["speed"] * t,
                        elevation=vw["elev"], radius=vw["radius"], seed=seed * 7919 + len(out)))
    return out
