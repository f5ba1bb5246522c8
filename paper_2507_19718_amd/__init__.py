"""GSCache hot path on MI355X: Python binding of the C ABI (include/gsc.h).

Every function here marshals arguments and calls into libgsc.so; all work on the path runs in
the HIP kernels.  PyTorch supplies device memory (the library's allocator hook draws from
torch's caching allocator) and the stream (the context enqueues on torch's current stream).

GSCache (arXiv 2507.19718) keeps a multi-level path-space radiance cache of 3D Gaussians,
splatted each frame into per-path-length cache images and trained on the fly against the
noisy per-length radiance a delta-tracking volume path tracer produces.
"""
from __future__ import annotations

import ctypes
import math
import os
import weakref
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import (GSC_E_CAPACITY, GSC_OK, STATUS_NAMES, gsc_adam_hparams, gsc_binning_info,
                   gsc_camera, gsc_frame_request, gsc_frame_stats, gsc_gaussians, gsc_grads,
                   gsc_trace_params, gsc_volume)

__all__ = ["GscError", "Context", "Binning", "Scene", "Volume", "camera_struct", "levels_struct",
           "gsc_ctx_create", "gsc_trace_targets", "gsc_project_bin", "gsc_binning_view",
           "gsc_binning_keys", "gsc_splat_forward", "gsc_splat_backward", "gsc_loss_composite",
           "gsc_adam_step", "gsc_render_frame", "gsc_render_frames", "GscSplat", "lib"]

PARAM_NAMES = ("pos", "rot", "log_scale", "rgb", "opacity_logit")
PARAM_WIDTH = {"pos": 3, "rot": 4, "log_scale": 3, "rgb": 3, "opacity_logit": 1}


def lib():
    return _abi.load()


class GscError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors passed to the GSCache library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _f32_cuda(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


# ----------------------------------------------------------------------------------------------
# Context (with torch's caching allocator as the device-memory hook)
# ----------------------------------------------------------------------------------------------
# The allocator hook's C thunks live at module level for the life of the process: library
# objects (scenes, binnings, context workspaces) may release memory through them during
# garbage collection, after the Python object that configured them is gone.
_ALLOC_USERS: Dict[int, tuple] = {}


def _torch_alloc(nbytes, user):
    dev, st = _ALLOC_USERS[int(user or 0)]
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
    except Exception:
        return None


def _torch_release(ptr, user):
    torch.cuda.caching_allocator_delete(int(ptr))


_ALLOC_FN = _abi.gsc_allocator._fields_[0][1](_torch_alloc)
_RELEASE_FN = _abi.gsc_allocator._fields_[1][1](_torch_release)


def _destroy_ctx(lib_, h):
    lib_.gsc_ctx_destroy(h)


def _destroy_scene(ctx, h):
    ctx._lib.gsc_scene_destroy(ctx.handle, h)


def _release_binning(ctx, h):
    ctx._lib.gsc_binning_release(ctx.handle, h)


class Context:
    """A library context on one device enqueuing on one stream (default: torch's current)."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None,
                 torch_allocator: bool = True):
        self._lib = lib()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self._alloc = None
        alloc_p = None
        if torch_allocator:
            key = len(_ALLOC_USERS) + 1
            _ALLOC_USERS[key] = (device, self.stream)
            self._alloc = _abi.gsc_allocator(_ALLOC_FN, _RELEASE_FN, ctypes.c_void_p(key))
            alloc_p = ctypes.byref(self._alloc)
        h = ctypes.c_void_p()
        st = self._lib.gsc_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream), alloc_p,
                                      ctypes.byref(h))
        if st != GSC_OK:
            raise GscError(st, "gsc_ctx_create failed")
        self.handle = h
        # Objects that belong to this context hold it (through their finalizers) until they are
        # released; nothing is released at interpreter exit.
        self._finalizer = weakref.finalize(self, _destroy_ctx, self._lib, h)
        self._finalizer.atexit = False

    def check(self, status: int):
        if status != GSC_OK:
            msg = self._lib.gsc_ctx_last_error(self.handle)
            raise GscError(status, msg.decode() if msg else "")

    def required_capacity(self) -> int:
        return int(self._lib.gsc_ctx_required_capacity(self.handle))

    def synchronize(self):
        self.check(self._lib.gsc_ctx_synchronize(self.handle))

    def profile(self, on: bool):
        self.check(self._lib.gsc_ctx_profile(self.handle, 1 if on else 0))

    def profile_read(self) -> Dict[str, dict]:
        """{kernel: {"ms": total, "launches": n}} since profiling was turned on."""
        out = {}
        idx = 0
        while True:
            buf = ctypes.create_string_buffer(64)
            ms, n = ctypes.c_double(), ctypes.c_int64()
            st = self._lib.gsc_ctx_profile_read(self.handle, idx, buf, 64, ctypes.byref(ms),
                                                ctypes.byref(n))
            if st != GSC_OK:
                break
            out[buf.value.decode()] = {"ms": ms.value, "launches": n.value}
            idx += 1
        return out

    def set_list_cut(self, on: bool):
        """Frames bin only the list prefixes that can reach a pixel (default on)."""
        self.check(self._lib.gsc_ctx_set_list_cut(self.handle, 1 if on else 0))

    def set_frame_binning(self, on: bool):
        """gsc_project_bin bins like the frames (32x32 tiles, list cut) (default off)."""
        self.check(self._lib.gsc_ctx_set_frame_binning(self.handle, 1 if on else 0))

    def set_frame_tiles(self, tile_px: int):
        """Tile edge frames bin with: 16, 32, or 0 = by batch size (default)."""
        self.check(self._lib.gsc_ctx_set_frame_tiles(self.handle, int(tile_px)))

    def set_deterministic(self, on: bool):
        """Sum the splat adjoint in fixed point so gradients repeat bit for bit (default off)."""
        self.check(self._lib.gsc_ctx_set_deterministic(self.handle, 1 if on else 0))

    def debug_selftest(self):
        """Fires the device bounds-check path on purpose (gsc_debug_selftest); returns the status
        and message instead of raising: GSC_E_DEVICE naming "self-test" with the debug library
        (GSC_DEBUG=1), GSC_E_UNSUPPORTED with the release one."""
        st = self._lib.gsc_debug_selftest(self.handle)
        return st, self._lib.gsc_ctx_last_error(self.handle).decode()

    def probe_gather(self, cells: torch.Tensor, threads: int, per_thread: int) -> float:
        """ms for threads x per_thread random 32-byte reads of `cells` (a uint8/float tensor whose
        size is a multiple of 32 bytes)."""
        out = torch.empty(threads, dtype=torch.float32, device=cells.device)
        ms = ctypes.c_double()
        self.check(self._lib.gsc_probe_gather(self.handle, cells.data_ptr(), cells.numel() * cells.element_size() // 32,
                                              threads, per_thread, out.data_ptr(), ctypes.byref(ms)))
        return ms.value

    def probe_atomics(self, buf: torch.Tensor, threads: int, per_thread: int) -> float:
        """ms for threads x per_thread float atomic adds to random elements of buf (float32)."""
        assert buf.dtype == torch.float32
        ms = ctypes.c_double()
        self.check(self._lib.gsc_probe_atomics(self.handle, buf.data_ptr(), buf.numel(), threads,
                                               per_thread, ctypes.byref(ms)))
        return ms.value

    def probe_valu(self, threads: int, iters: int, mode: int) -> float:
        """ms for threads x iters x 8 fp32 FMAs (mode 0) or exponentials (mode 1)."""
        out = torch.empty(threads, dtype=torch.float32, device="cuda")
        ms = ctypes.c_double()
        self.check(self._lib.gsc_probe_valu(self.handle, out.data_ptr(), threads, iters, mode,
                                            ctypes.byref(ms)))
        return ms.value

    def set_work_counters(self, on: bool):
        """Run the counting variants of the splat kernels (fills the fwd_* / bwd_* counters)."""
        self.check(self._lib.gsc_ctx_set_work_counters(self.handle, 1 if on else 0))

    def counters(self):
        c = _abi.gsc_counters()
        self.check(self._lib.gsc_ctx_counters(self.handle, ctypes.byref(c)))
        return c.as_dict()

    def trim(self):
        self.check(self._lib.gsc_ctx_trim(self.handle))

    def close(self):
        self._finalizer()


def gsc_ctx_create(device: int = 0, stream=None, torch_allocator: bool = True) -> Context:
    return Context(device, stream, torch_allocator)


# ----------------------------------------------------------------------------------------------
# Marshalling helpers
# ----------------------------------------------------------------------------------------------
def camera_struct(cam) -> gsc_camera:
    """From any object with R[9], t[3], fx, fy, cx, cy, full_w, full_h, x0, y0, w, h, znear."""
    c = gsc_camera()
    R = np.asarray(cam.R, dtype=np.float32).reshape(9)
    t = np.asarray(cam.t, dtype=np.float32).reshape(3)
    for i in range(9):
        c.R[i] = float(R[i])
    for i in range(3):
        c.t[i] = float(t[i])
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    c.full_w, c.full_h = int(cam.full_w), int(cam.full_h)
    c.x0, c.y0, c.w, c.h = int(cam.x0), int(cam.y0), int(cam.w), int(cam.h)
    c.znear = float(getattr(cam, "znear", 0.2))
    return c


def levels_struct(levels: Sequence[Dict[str, torch.Tensor]]):
    arr = (gsc_gaussians * len(levels))()
    for l, lv in enumerate(levels):
        n = int(lv["pos"].shape[0])
        for k in PARAM_NAMES:
            t = _f32_cuda(lv[k], k)
            if t.numel() != n * PARAM_WIDTH[k]:
                raise ValueError(f"level {l}: {k} has {t.numel()} elements, expected {n * PARAM_WIDTH[k]}")
        arr[l] = gsc_gaussians(_ptr(lv["pos"]), _ptr(lv["rot"]), _ptr(lv["log_scale"]),
                               _ptr(lv["rgb"]), _ptr(lv["opacity_logit"]), n)
    return arr


def level_to_device(g, device="cuda") -> Dict[str, torch.Tensor]:
    """A synth.Gaussians (numpy) -> dict of contiguous float32 device tensors."""
    return {k: torch.from_numpy(np.ascontiguousarray(getattr(g, k), dtype=np.float32)).to(device)
            for k in PARAM_NAMES}


def _host_rows(a, width: int) -> np.ndarray:
    return np.ascontiguousarray(np.zeros((0, width)) if a is None else a,
                                dtype=np.float32).reshape(-1, width)


def _rows_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.shape[0] else None


class Volume:
    """Device-resident density plus host TF, point lights [L][6] and sphere lights [S][7]."""

    def __init__(self, density: torch.Tensor, density_max: float, tf, lights, spheres=None):
        self.density = _f32_cuda(density, "density")
        self.density_max = float(density_max)
        self.tf = np.ascontiguousarray(tf, dtype=np.float32)
        self.lights = _host_rows(lights, 6)
        self.spheres = _host_rows(spheres, 7)

    @classmethod
    def from_synth(cls, vol, device="cuda"):
        return cls(torch.from_numpy(vol.density).to(device), vol.density_max, vol.tf, vol.lights,
                   getattr(vol, "spheres", None))

    def struct(self) -> gsc_volume:
        nz, ny, nx = self.density.shape
        return gsc_volume(_ptr(self.density), nx, ny, nz, self.density_max,
                          self.tf.ctypes.data_as(ctypes.c_void_p), self.tf.shape[0],
                          _rows_ptr(self.lights), self.lights.shape[0],
                          _rows_ptr(self.spheres), self.spheres.shape[0])


STRATEGY_NEE, STRATEGY_UNIFORM = 0, 1


def trace_params(seed: int, frame: int, spp: int, max_bounces: int, K: int, C: float = 0.5,
                 eps: float = 0.0, strategy: int = STRATEGY_NEE) -> gsc_trace_params:
    inf = math.isinf(C)
    return gsc_trace_params(seed, frame, spp, max_bounces, K, 0.0 if inf else C, 1 if inf else 0, eps,
                            strategy)


# ----------------------------------------------------------------------------------------------
# The hot-path calls (same names as the C ABI)
# ----------------------------------------------------------------------------------------------
def gsc_trace_targets(ctx: Context, vol: Volume, cam, params: gsc_trace_params,
                      targets: torch.Tensor, records: Optional[torch.Tensor] = None,
                      stats: bool = False):
    """targets: [K][h][w][3] float32; records: [spp][h][w][5] 4-byte words, or None."""
    _f32_cuda(targets, "targets")
    _check_bytes(targets, 12 * params.num_levels * cam.w * cam.h, "targets")
    _check_bytes(records, 20 * params.spp * cam.w * cam.h, "records")
    vs = vol.struct()
    cs = camera_struct(cam)
    st = gsc_frame_stats() if stats else None
    ctx.check(ctx._lib.gsc_trace_targets(ctx.handle, ctypes.byref(vs), ctypes.byref(cs),
                                         ctypes.byref(params), _ptr(targets), _ptr(records),
                                         ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


# ----------------------------------------------------------------------------------------------
# Cache initialisation (Method: "Cache Initialization", Eq. 2)
# ----------------------------------------------------------------------------------------------
def gsc_init_points(ctx: Context, vol: Volume, n: int, seed: int):
    """n first-interaction points of random rays and their albedo: (pos, albedo), [n][3] each."""
    pos = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    albedo = torch.empty((n, 3), dtype=torch.float32, device="cuda")
    vs = vol.struct()
    ctx.check(ctx._lib.gsc_init_points(ctx.handle, ctypes.byref(vs), n, seed, _ptr(pos), _ptr(albedo)))
    return pos, albedo


def gsc_knn_mean3(ctx: Context, pos: torch.Tensor) -> torch.Tensor:
    """Mean distance of every point ([n][3] float32, CUDA) to its 3 nearest other points."""
    _f32_cuda(pos, "pos")
    n = pos.shape[0]
    out = torch.empty(n, dtype=torch.float32, device="cuda")
    ctx.check(ctx._lib.gsc_knn_mean3(ctx.handle, _ptr(pos), n, _ptr(out)))
    return out


def gsc_cache_init(ctx: Context, vol: Volume, n: int, K: int, seed: int) -> List[Dict[str, torch.Tensor]]:
    """K initial cache levels (level l has n >> l Gaussians), as dicts of CUDA tensors with the
    parameter names (pos, rot, log_scale, rgb, opacity_logit)."""
    levels = []
    bufs = (_abi.gsc_level_buffers * K)()
    for l in range(K):
        nl = n >> l
        lv = {"pos": torch.empty((nl, 3), dtype=torch.float32, device="cuda"),
              "rot": torch.empty((nl, 4), dtype=torch.float32, device="cuda"),
              "log_scale": torch.empty((nl, 3), dtype=torch.float32, device="cuda"),
              "rgb": torch.empty((nl, 3), dtype=torch.float32, device="cuda"),
              "opacity_logit": torch.empty((nl,), dtype=torch.float32, device="cuda")}
        levels.append(lv)
        bufs[l] = _abi.gsc_level_buffers(_ptr(lv["pos"]), _ptr(lv["rot"]), _ptr(lv["log_scale"]),
                                         _ptr(lv["rgb"]), _ptr(lv["opacity_logit"]), nl)
    vs = vol.struct()
    ctx.check(ctx._lib.gsc_cache_init(ctx.handle, ctypes.byref(vs), n, K, seed, bufs))
    return levels


class Binning:
    """Owns a gsc_binning*; released on garbage collection (after the stream drains)."""

    def __init__(self, ctx: Context, handle: ctypes.c_void_p, K: int, cam):
        self.ctx = ctx
        self.handle = handle
        self.K = K
        self.cam = cam
        self._finalizer = weakref.finalize(self, _release_binning, ctx, handle)
        self._finalizer.atexit = False

    def release(self):
        self._finalizer()


def gsc_project_bin(ctx: Context, levels: Sequence[Dict[str, torch.Tensor]], cam,
                    capacity_hint: int = 0) -> Binning:
    arr = levels_struct(levels)
    cs = camera_struct(cam)
    h = ctypes.c_void_p()
    ctx.check(ctx._lib.gsc_project_bin(ctx.handle, arr, len(levels), ctypes.byref(cs),
                                       capacity_hint, ctypes.byref(h)))
    return Binning(ctx, h, len(levels), cam)


def _copy_out(ctx: Context, ptr: int, shape, dtype) -> torch.Tensor:
    out = torch.empty(shape, dtype=dtype, device=f"cuda:{ctx.device}")
    nbytes = out.numel() * out.element_size()
    if nbytes:
        ctx.check(ctx._lib.gsc_copy(ctx.handle, _ptr(out), ctypes.c_void_p(ptr), nbytes))
    return out


def gsc_binning_view(ctx: Context, b: Binning) -> dict:
    """Counts plus copies (torch tensors) of the binning arrays."""
    info = gsc_binning_info()
    ctx.check(ctx._lib.gsc_binning_view(ctx.handle, b.handle, ctypes.byref(info)))
    G = int(info.gauss_offset[info.num_levels])
    I = int(info.n_instances)
    T = int(info.n_tiles)
    out = dict(n_instances=I, n_tiles=T, tiles_x=info.tiles_x, tiles_y=info.tiles_y,
               gauss_offset=[int(info.gauss_offset[i]) for i in range(info.num_levels + 1)])
    out["values"] = _copy_out(ctx, info.values, (I,), torch.int32)
    out["ranges"] = _copy_out(ctx, info.ranges, (T, 2), torch.int64)
    out["window"] = _copy_out(ctx, info.window, (G, 4), torch.int32)
    out["tiles_touched"] = _copy_out(ctx, info.tiles_touched, (G,), torch.int32)
    out["depth_key"] = _copy_out(ctx, info.depth_key, (G,), torch.int32)
    out["screen"] = _copy_out(ctx, info.screen, (G, 6), torch.float32)
    return out


def gsc_binning_keys(ctx: Context, b: Binning, n_instances: int) -> torch.Tensor:
    keys = torch.empty((n_instances,), dtype=torch.int64, device=f"cuda:{ctx.device}")
    ctx.check(ctx._lib.gsc_binning_keys(ctx.handle, b.handle, _ptr(keys)))
    return keys


def gsc_splat_forward(ctx: Context, b: Binning, images: torch.Tensor, final_T: torch.Tensor,
                      last_id: torch.Tensor):
    _f32_cuda(images, "images")
    _f32_cuda(final_T, "final_T")
    if last_id.dtype != torch.int32:
        raise ValueError("last_id must be int32")
    ctx.check(ctx._lib.gsc_splat_forward(ctx.handle, b.handle, _ptr(images), _ptr(final_T),
                                         _ptr(last_id)))


def gsc_splat_backward(ctx: Context, b: Binning, levels, cam, final_T, last_id, dL_dimages,
                       grads: Sequence[Dict[str, torch.Tensor]]):
    arr = levels_struct(levels)
    cs = camera_struct(cam)
    garr = (gsc_grads * len(levels))()
    for l, g in enumerate(grads):
        garr[l] = gsc_grads(_ptr(g["pos"]), _ptr(g["rot"]), _ptr(g["log_scale"]), _ptr(g["rgb"]),
                            _ptr(g["opacity_logit"]))
    ctx.check(ctx._lib.gsc_splat_backward(ctx.handle, b.handle, arr, len(levels), ctypes.byref(cs),
                                          _ptr(final_T), _ptr(last_id), _ptr(dL_dimages), garr))


def gsc_splat_backward_noalloc(ctx: Context, b: Binning, levels, cam, final_T, last_id,
                               dL_dimages, grads: Sequence[Dict[str, torch.Tensor]]):
    """gsc_splat_backward without any device allocation (the library's static scratch array):
    for callers that cannot allocate.  The caller passes every output."""
    arr = levels_struct(levels)
    cs = camera_struct(cam)
    garr = (gsc_grads * len(levels))()
    for l, g in enumerate(grads):
        garr[l] = gsc_grads(_ptr(g["pos"]), _ptr(g["rot"]), _ptr(g["log_scale"]), _ptr(g["rgb"]),
                            _ptr(g["opacity_logit"]))
    ctx.check(ctx._lib.gsc_splat_backward_noalloc(ctx.handle, b.handle, arr, len(levels),
                                                  ctypes.byref(cs), _ptr(final_T), _ptr(last_id),
                                                  _ptr(dL_dimages), garr))


def _check_bytes(t: Optional[torch.Tensor], need: int, what: str):
    if t is not None and t.numel() * t.element_size() < need:
        raise ValueError(f"{what} holds {t.numel() * t.element_size()} bytes, needs {need}")


def gsc_loss_composite(ctx: Context, images, targets, records, K: int, w: int, h: int, loss: int,
                       dL_dimages, loss_out, composite=None, spp: int = 1):
    """records: [spp][h][w][5] 4-byte words (or None with composite None)."""
    for t, name in ((images, "images"), (targets, "targets"), (dL_dimages, "dL_dimages")):
        _check_bytes(t, 12 * K * w * h, name)
    _check_bytes(records, 20 * spp * w * h, "records")
    _check_bytes(composite, 12 * w * h, "composite")
    ctx.check(ctx._lib.gsc_loss_composite(ctx.handle, _ptr(images), _ptr(targets), _ptr(records),
                                          spp, K, w, h, loss, _ptr(dL_dimages), _ptr(loss_out),
                                          _ptr(composite)))


def gsc_adam_step(ctx: Context, param, m, v, grad, lr: float, beta1: float, beta2: float,
                  eps: float, weight_decay: float, step: int):
    hp = gsc_adam_hparams(lr, beta1, beta2, eps, weight_decay, step)
    ctx.check(ctx._lib.gsc_adam_step(ctx.handle, _ptr(param), _ptr(m), _ptr(v), _ptr(grad),
                                     param.numel(), ctypes.byref(hp)))


# ----------------------------------------------------------------------------------------------
# Autograd: the adjoint backward behind torch.autograd.Function
# ----------------------------------------------------------------------------------------------
class GscSplat(torch.autograd.Function):
    """images[K][h][w][3] = splat(levels, camera); backward = gsc_splat_backward.

    Call as GscSplat.apply(ctx, cam, *flat) with flat = (pos, rot, log_scale, rgb,
    opacity_logit) for each level in order."""

    @staticmethod
    def forward(fctx, gctx: Context, cam, *flat):
        K = len(flat) // 5
        levels = [dict(zip(PARAM_NAMES, flat[5 * l:5 * l + 5])) for l in range(K)]
        b = gsc_project_bin(gctx, levels, cam)
        dev = flat[0].device
        images = torch.empty((K, cam.h, cam.w, 3), dtype=torch.float32, device=dev)
        final_T = torch.empty((K, cam.h, cam.w), dtype=torch.float32, device=dev)
        last_id = torch.empty((K, cam.h, cam.w), dtype=torch.int32, device=dev)
        gsc_splat_forward(gctx, b, images, final_T, last_id)
        fctx.gctx, fctx.cam, fctx.binning, fctx.K = gctx, cam, b, K
        fctx.save_for_backward(final_T, last_id, *flat)
        fctx.mark_non_differentiable(final_T, last_id)
        return images, final_T, last_id

    @staticmethod
    def backward(fctx, dL_dimages, _dT, _dl):
        final_T, last_id, *flat = fctx.saved_tensors
        K = fctx.K
        levels = [dict(zip(PARAM_NAMES, flat[5 * l:5 * l + 5])) for l in range(K)]
        grads = [{k: torch.empty_like(lv[k]) for k in PARAM_NAMES} for lv in levels]
        gsc_splat_backward(fctx.gctx, fctx.binning, levels, fctx.cam, final_T, last_id,
                           dL_dimages.contiguous(), grads)
        fctx.binning.release()
        out = []
        for g in grads:
            out += [g[k] for k in PARAM_NAMES]
        return (None, None, *out)


def splat(gctx: Context, cam, levels: Sequence[Dict[str, torch.Tensor]]):
    flat = []
    for lv in levels:
        flat += [lv[k] for k in PARAM_NAMES]
    return GscSplat.apply(gctx, cam, *flat)


# ----------------------------------------------------------------------------------------------
# Scenes and frames
# ----------------------------------------------------------------------------------------------
class Scene:
    """A resident scene: volume copy, TF, lights, K levels with Adam moments."""

    def __init__(self, ctx: Context, vol: Volume, levels: Sequence[Dict[str, torch.Tensor]]):
        self.ctx = ctx
        self.K = len(levels)
        self.n = [int(lv["pos"].shape[0]) for lv in levels]
        arr = levels_struct(levels)
        vs = vol.struct()
        h = ctypes.c_void_p()
        ctx.check(ctx._lib.gsc_scene_create(ctx.handle, ctypes.byref(vs), arr, len(levels),
                                            ctypes.byref(h)))
        self.handle = h
        self._finalizer = weakref.finalize(self, _destroy_scene, ctx, h)
        self._finalizer.atexit = False

    def destroy(self):
        self._finalizer()

    def set_optics(self, tf, lights, spheres=None):
        tf = np.ascontiguousarray(tf, dtype=np.float32)
        lights, spheres = _host_rows(lights, 6), _host_rows(spheres, 7)
        self.ctx.check(self.ctx._lib.gsc_scene_set_optics(
            self.ctx.handle, self.handle, tf.ctypes.data_as(ctypes.c_void_p), tf.shape[0],
            _rows_ptr(lights), lights.shape[0], _rows_ptr(spheres), spheres.shape[0]))

    def level(self, l: int) -> Dict[str, torch.Tensor]:
        """Copies of level l's current parameters."""
        g = gsc_gaussians()
        self.ctx.check(self.ctx._lib.gsc_scene_level(self.handle, l, ctypes.byref(g)))
        n = int(g.n)
        return {k: _copy_out(self.ctx, getattr(g, k), (n, PARAM_WIDTH[k]) if PARAM_WIDTH[k] > 1 else (n,),
                             torch.float32) for k in PARAM_NAMES}

    def state(self, l: int) -> Dict[str, object]:
        """Copies of level l's parameters and AdamW moments ([14 n] each, grouped as
        [pos 3n][rot 4n][log_scale 3n][rgb 3n][opacity_logit n]) and its step count."""
        p, m, v = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        n, step = ctypes.c_int64(), ctypes.c_int64()
        self.ctx.check(self.ctx._lib.gsc_scene_state(self.handle, l, ctypes.byref(p), ctypes.byref(m),
                                                     ctypes.byref(v), ctypes.byref(n), ctypes.byref(step)))
        cnt = 14 * n.value
        return dict(params=_copy_out(self.ctx, p.value, (cnt,), torch.float32),
                    m=_copy_out(self.ctx, m.value, (cnt,), torch.float32),
                    v=_copy_out(self.ctx, v.value, (cnt,), torch.float32),
                    n=int(n.value), step=int(step.value))

    def copy_state_from(self, other: "Scene"):
        self.ctx.check(self.ctx._lib.gsc_scene_copy_state(self.ctx.handle, self.handle, other.handle))

    def save(self, path: str):
        """Checkpoints every level's parameters, AdamW moments and step count to a file."""
        self.ctx.check(self.ctx._lib.gsc_scene_save(self.ctx.handle, self.handle,
                                                    os.fsencode(path)))

    def load(self, path: str):
        """Restores a checkpoint written by save() (same level count and sizes)."""
        self.ctx.check(self.ctx._lib.gsc_scene_load(self.ctx.handle, self.handle,
                                                    os.fsencode(path)))

    def footprint_bytes(self) -> int:
        return int(self.ctx._lib.gsc_scene_footprint_bytes(self.handle))

    def frame_footprint_bytes(self, w: int, h: int, instance_estimate: int) -> int:
        return int(self.ctx._lib.gsc_frame_footprint_bytes(self.handle, w, h, instance_estimate))


def frame_request(cam, seed: int, frame: int, K: int, max_bounces: int, loss: int = 1,
                  train: bool = True, viewport_frames: int = 1,
                  lr=(1.16e-3, 1e-3, 0.0, 1.25e-2, 1.5e-1), beta1=0.9, beta2=0.999, eps=1e-8,
                  weight_decay=0.0, C: float = 0.5,
                  strategy: int = STRATEGY_NEE, spp: int = 1) -> gsc_frame_request:
    r = gsc_frame_request()
    r.cam = camera_struct(cam)
    r.trace = trace_params(seed, frame, spp, max_bounces, K, C, strategy=strategy)
    r.loss = loss
    r.train = 1 if train else 0
    r.viewport_frames = viewport_frames
    for i in range(5):
        r.lr[i] = float(lr[i])
    r.beta1, r.beta2, r.eps, r.weight_decay = beta1, beta2, eps, weight_decay
    return r


def gsc_render_frame(ctx: Context, scene: Scene, req: gsc_frame_request, image: torch.Tensor,
                     stats: bool = False):
    _f32_cuda(image, "image")
    st = gsc_frame_stats() if stats else None
    ctx.check(ctx._lib.gsc_render_frame(ctx.handle, scene.handle, ctypes.byref(req), _ptr(image),
                                        ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def gsc_render_frames(ctx: Context, scenes: Sequence[Scene], reqs: Sequence[gsc_frame_request],
                      images: Sequence[torch.Tensor], stats: bool = False):
    n = len(scenes)
    sh = (ctypes.c_void_p * n)(*[s.handle.value for s in scenes])
    rq = (gsc_frame_request * n)(*reqs)
    im = (ctypes.c_void_p * n)(*[_f32_cuda(i, "image").data_ptr() for i in images])
    st = (gsc_frame_stats * n)() if stats else None
    ctx.check(ctx._lib.gsc_render_frames(ctx.handle, sh, rq, im, n, st))
    return [s.as_dict() for s in st] if st is not None else None
