"""ctypes declarations of the C ABI in include/gsc.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32,
                    c_uint64, c_void_p, c_char_p)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsc.so")
DEBUG_LIB_PATH = os.path.join(_HERE, "libgsc_debug.so")

GSC_OK, GSC_E_INVALID_ARG, GSC_E_CAPACITY, GSC_E_OUT_OF_MEMORY, GSC_E_DEVICE, GSC_E_UNSUPPORTED = range(6)
STATUS_NAMES = {0: "GSC_OK", 1: "GSC_E_INVALID_ARG", 2: "GSC_E_CAPACITY", 3: "GSC_E_OUT_OF_MEMORY",
                4: "GSC_E_DEVICE", 5: "GSC_E_UNSUPPORTED"}


class gsc_allocator(Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p)),
                ("release", ctypes.CFUNCTYPE(None, c_void_p, c_void_p)),
                ("user", c_void_p)]


class gsc_camera(Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("full_w", c_int32), ("full_h", c_int32),
                ("x0", c_int32), ("y0", c_int32), ("w", c_int32), ("h", c_int32),
                ("znear", c_float)]


class gsc_gaussians(Structure):
    _fields_ = [("pos", c_void_p), ("rot", c_void_p), ("log_scale", c_void_p), ("rgb", c_void_p),
                ("opacity_logit", c_void_p), ("n", c_int64)]


class gsc_grads(Structure):
    _fields_ = [("pos", c_void_p), ("rot", c_void_p), ("log_scale", c_void_p), ("rgb", c_void_p),
                ("opacity_logit", c_void_p)]


class gsc_volume(Structure):
    _fields_ = [("density", c_void_p), ("nx", c_int32), ("ny", c_int32), ("nz", c_int32),
                ("density_max", c_float), ("tf_rgba", c_void_p), ("tf_points", c_int32),
                ("lights", c_void_p), ("n_lights", c_int32), ("spheres", c_void_p),
                ("n_spheres", c_int32)]


class gsc_trace_params(Structure):
    _fields_ = [("seed", c_uint64), ("frame", c_uint32), ("spp", c_uint32),
                ("max_bounces", c_uint32), ("num_levels", c_uint32), ("C", c_float),
                ("C_inf", c_int32), ("eps", c_float), ("strategy", c_uint32)]


class gsc_path_record(Structure):
    _fields_ = [("L", c_float * 3), ("beta", c_float), ("n_kind", c_uint32)]


class gsc_frame_stats(Structure):
    _fields_ = [("ms_project_bin", c_double), ("ms_forward", c_double), ("ms_trace", c_double),
                ("ms_loss", c_double), ("ms_backward", c_double), ("ms_adam", c_double),
                ("ms_total", c_double), ("gaussians", c_uint64), ("instances", c_uint64),
                ("tiles", c_uint64), ("pixels", c_uint64), ("paths", c_uint64),
                ("path_vertices", c_uint64), ("loss", c_double), ("adam_skipped", c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class gsc_binning_info(Structure):
    _fields_ = [("n_instances", c_uint64), ("n_tiles", c_uint64), ("num_levels", c_int32),
                ("tiles_x", c_int32), ("tiles_y", c_int32), ("gauss_offset", c_int64 * 9),
                ("values", c_void_p), ("ranges", c_void_p), ("window", c_void_p),
                ("tiles_touched", c_void_p), ("depth_key", c_void_p), ("screen", c_void_p)]


class gsc_adam_hparams(Structure):
    _fields_ = [("lr", c_double), ("beta1", c_double), ("beta2", c_double), ("eps", c_double),
                ("weight_decay", c_double), ("step", c_int64)]


class gsc_frame_request(Structure):
    _fields_ = [("cam", gsc_camera), ("trace", gsc_trace_params), ("loss", c_int32),
                ("train", c_int32), ("viewport_frames", c_uint32), ("lr", c_double * 5),
                ("beta1", c_double), ("beta2", c_double), ("eps", c_double),
                ("weight_decay", c_double)]


class gsc_level_buffers(Structure):
    _fields_ = [("pos", c_void_p), ("rot", c_void_p), ("log_scale", c_void_p), ("rgb", c_void_p),
                ("opacity_logit", c_void_p), ("n", c_int64)]


class gsc_counters(Structure):
    _fields_ = [("instances", c_uint64), ("binnings", c_uint64), ("evaluations", c_uint64),
                ("blended", c_uint64), ("contributors", c_uint64), ("tile_entries", c_uint64),
                ("fwd_tested", c_uint64), ("fwd_slots", c_uint64), ("bwd_tested", c_uint64),
                ("bwd_blended", c_uint64), ("bwd_slots", c_uint64), ("bwd_entries", c_uint64),
                ("bwd_atomics", c_uint64), ("bwd_records", c_uint64), ("frame_retries", c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


STRUCTS = [gsc_camera, gsc_gaussians, gsc_grads, gsc_volume, gsc_trace_params, gsc_path_record,
           gsc_frame_stats, gsc_binning_info, gsc_adam_hparams, gsc_frame_request, gsc_allocator,
           gsc_counters, gsc_level_buffers]

P = POINTER
_SIGNATURES = {
    "gsc_ctx_create": (c_int32, [c_int32, c_void_p, P(gsc_allocator), P(c_void_p)]),
    "gsc_ctx_destroy": (None, [c_void_p]),
    "gsc_ctx_last_error": (c_char_p, [c_void_p]),
    "gsc_ctx_set_stream": (c_int32, [c_void_p, c_void_p]),
    "gsc_ctx_set_deterministic": (c_int32, [c_void_p, c_int32]),
    "gsc_ctx_set_list_cut": (c_int32, [c_void_p, c_int32]),
    "gsc_ctx_set_frame_binning": (c_int32, [c_void_p, c_int32]),
    "gsc_ctx_set_frame_tiles": (c_int32, [c_void_p, c_int32]),
    "gsc_ctx_set_work_counters": (c_int32, [c_void_p, c_int32]),
    "gsc_ctx_required_capacity": (c_uint64, [c_void_p]),
    "gsc_ctx_trim": (c_int32, [c_void_p]),
    "gsc_ctx_synchronize": (c_int32, [c_void_p]),
    "gsc_debug_selftest": (c_int32, [c_void_p]),
    "gsc_copy": (c_int32, [c_void_p, c_void_p, c_void_p, c_size_t]),
    "gsc_ctx_profile": (c_int32, [c_void_p, c_int32]),
    "gsc_ctx_profile_read": (c_int32, [c_void_p, c_int32, ctypes.c_char_p, c_size_t, P(c_double),
                                       P(c_int64)]),
    "gsc_ctx_counters": (c_int32, [c_void_p, P(gsc_counters)]),
    "gsc_probe_gather": (c_int32, [c_void_p, c_void_p, c_uint64, ctypes.c_uint32, c_int32, c_void_p,
                                   P(c_double)]),
    "gsc_probe_atomics": (c_int32, [c_void_p, c_void_p, c_uint64, ctypes.c_uint32, c_int32,
                                    P(c_double)]),
    "gsc_probe_valu": (c_int32, [c_void_p, c_void_p, ctypes.c_uint32, c_int32, c_int32, P(c_double)]),
    "gsc_init_points": (c_int32, [c_void_p, P(gsc_volume), c_int64, c_uint64, c_void_p, c_void_p]),
    "gsc_knn_mean3": (c_int32, [c_void_p, c_void_p, c_int64, c_void_p]),
    "gsc_cache_init": (c_int32, [c_void_p, P(gsc_volume), c_int64, c_int32, c_uint64,
                                 P(gsc_level_buffers)]),
    "gsc_trace_targets": (c_int32, [c_void_p, P(gsc_volume), P(gsc_camera), P(gsc_trace_params),
                                    c_void_p, c_void_p, P(gsc_frame_stats)]),
    "gsc_project_bin": (c_int32, [c_void_p, P(gsc_gaussians), c_int32, P(gsc_camera), c_uint64,
                                  P(c_void_p)]),
    "gsc_binning_view": (c_int32, [c_void_p, c_void_p, P(gsc_binning_info)]),
    "gsc_binning_keys": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "gsc_binning_release": (None, [c_void_p, c_void_p]),
    "gsc_splat_forward": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "gsc_splat_backward": (c_int32, [c_void_p, c_void_p, P(gsc_gaussians), c_int32, P(gsc_camera),
                                     c_void_p, c_void_p, c_void_p, P(gsc_grads)]),
    "gsc_splat_backward_noalloc": (c_int32, [c_void_p, c_void_p, P(gsc_gaussians), c_int32, P(gsc_camera),
                                     c_void_p, c_void_p, c_void_p, P(gsc_grads)]),
    "gsc_loss_composite": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                     c_int32, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "gsc_adam_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int64,
                                P(gsc_adam_hparams)]),
    "gsc_scene_create": (c_int32, [c_void_p, P(gsc_volume), P(gsc_gaussians), c_int32, P(c_void_p)]),
    "gsc_scene_destroy": (None, [c_void_p, c_void_p]),
    "gsc_scene_set_optics": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_void_p, c_int32,
                                       c_void_p, c_int32]),
    "gsc_scene_level": (c_int32, [c_void_p, c_int32, P(gsc_gaussians)]),
    "gsc_scene_state": (c_int32, [c_void_p, c_int32, P(c_void_p), P(c_void_p), P(c_void_p),
                                  P(c_int64), P(c_int64)]),
    "gsc_scene_copy_state": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "gsc_scene_save": (c_int32, [c_void_p, c_void_p, ctypes.c_char_p]),
    "gsc_scene_load": (c_int32, [c_void_p, c_void_p, ctypes.c_char_p]),
    "gsc_scene_footprint_bytes": (c_size_t, [c_void_p]),
    "gsc_frame_footprint_bytes": (c_size_t, [c_void_p, c_int32, c_int32, c_uint64]),
    "gsc_render_frame": (c_int32, [c_void_p, c_void_p, P(gsc_frame_request), c_void_p,
                                   P(gsc_frame_stats)]),
    "gsc_render_frames": (c_int32, [c_void_p, P(c_void_p), P(gsc_frame_request), P(c_void_p),
                                    c_int32, P(gsc_frame_stats)]),
    "gsc_abi_struct_size": (c_size_t, [c_int32]),
}

_lib = None


def library_path() -> str:
    """The in-tree libgsc.so, or with GSC_DEBUG=1 in the environment the debug build
    libgsc_debug.so (device bounds checks; see gsc_debug_selftest)."""
    return DEBUG_LIB_PATH if os.environ.get("GSC_DEBUG") == "1" else LIB_PATH


def load():
    """Loads the in-tree library.  There is no fallback: without it nothing runs."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(
                f"{path} is missing: build it with `python __graft_entry__.py` or "
                "`python -m paper_2507_19718_amd.build_lib`; the GSCache path has no CPU fallback")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        for i, st in enumerate(STRUCTS):
            got = lib.gsc_abi_struct_size(i)
            if got != ctypes.sizeof(st):
                raise ImportError(f"ABI mismatch for {st.__name__}: C {got} B, Python {ctypes.sizeof(st)} B")
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGNATURES)
