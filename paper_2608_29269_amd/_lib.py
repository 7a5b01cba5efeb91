"""ctypes declarations of liblightfuse.so (include/lightfuse.h).

Argument marshalling only: every step of the tracer runs in the HIP library.
Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblightfuse.so")

LF_OK, LF_EINVAL, LF_ENOMEM, LF_EDEVICE, LF_EBUSY, LF_EOVERFLOW, LF_EUNSUPPORTED, LF_EABORTED, LF_ETIMEOUT = range(9)
STATUS_NAMES = {0: "LF_OK", 1: "LF_EINVAL", 2: "LF_ENOMEM", 3: "LF_EDEVICE", 4: "LF_EBUSY", 5: "LF_EOVERFLOW",
                6: "LF_EUNSUPPORTED", 7: "LF_EABORTED", 8: "LF_ETIMEOUT"}

FLAG_NO_SECONDARY = 1 << 0
FLAG_NO_BACKGROUND = 1 << 1
FLAG_BSDF_ONLY = 1 << 2
FLAG_DIFFUSE_ONLY = 1 << 3
FLAG_BRUTE_FORCE = 1 << 4
FLAG_COUNT = 1 << 5
FLAG_UNSORTED = 1 << 6
FLAG_NEE = 1 << 7  # the two-ray estimator: next-event + continuation per sample
FLAG_SOBOL = 1 << 8  # Owen-scrambled Sobol uniforms instead of the hash
FLAG_DETERMINISTIC = 1 << 9  # order-fixed binary64 gradient sums in the backward
MAX_CAMERAS = 16
SCHED_SHORTEST_FIRST, SCHED_OLDEST_FIRST, SCHED_ROUND_ROBIN = 0, 1, 2

_fp = C.POINTER(C.c_float)
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)


class Surfels(C.Structure):
    _fields_ = [("mu", C.c_void_p), ("q", C.c_void_p), ("scale", C.c_void_p), ("opacity", C.c_void_p),
                ("albedo", C.c_void_p), ("roughness", C.c_void_p), ("metallic", C.c_void_p), ("n", C.c_int64),
                ("n_objects", C.c_int32), ("object_offset", _i64p)]


class Transforms(C.Structure):
    _fields_ = [("R", C.c_void_p), ("t", C.c_void_p)]


class EnvMap(C.Structure):
    _fields_ = [("texels", C.c_void_p), ("h", C.c_int32), ("w", C.c_int32)]


class Rays(C.Structure):
    _fields_ = [("o", C.c_void_p), ("d", C.c_void_p), ("n", C.c_int64)]


class Camera(C.Structure):
    _fields_ = [("pose", C.c_float * 12), ("fov_y_deg", C.c_float), ("w", C.c_int32), ("h", C.c_int32)]


class Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("spp", C.c_int32), ("seed", C.c_uint64), ("alpha_min", C.c_double),
                ("alpha_cap", C.c_double), ("support_sigma", C.c_double), ("eps", C.c_double),
                ("t_min", C.c_double), ("secondary_offset", C.c_double), ("flags", C.c_uint32)]


class Outputs(C.Structure):
    _fields_ = [("radiance", C.c_void_p), ("depth", C.c_void_p), ("normal", C.c_void_p), ("alpha", C.c_void_p),
                ("hit_idx", C.c_void_p), ("sec_hit_idx", C.c_void_p)]


class GradOut(C.Structure):
    _fields_ = [("d_radiance", C.c_void_p), ("d_depth", C.c_void_p), ("d_normal", C.c_void_p),
                ("d_alpha", C.c_void_p)]


class GradIn(C.Structure):
    _fields_ = [("d_mu", C.c_void_p), ("d_q", C.c_void_p), ("d_scale", C.c_void_p), ("d_opacity", C.c_void_p),
                ("d_albedo", C.c_void_p), ("d_roughness", C.c_void_p), ("d_metallic", C.c_void_p),
                ("d_env", C.c_void_p)]


class SceneInfo(C.Structure):
    _fields_ = [("n_instances", C.c_int32), ("n_surfels", C.c_int64), ("n_nodes", C.c_int64),
                ("max_depth", C.c_int32), ("stack_size", C.c_int32), ("n_wide_nodes", C.c_int64),
                ("wide_levels", C.c_int32), ("node_width", C.c_int32)]


class RenderStats(C.Structure):
    _fields_ = [("rays_primary", C.c_int64), ("rays_secondary", C.c_int64)]


class ServerConfig(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("hbm_budget_bytes", C.c_int64), ("tile_rays", C.c_int32),
                ("batch_rays", C.c_int32), ("max_spp", C.c_int32), ("max_pending", C.c_int32),
                ("policy", C.c_int32), ("max_in_flight", C.c_int32), ("params", Params)]


class Request(C.Structure):
    _fields_ = [("xf", Transforms), ("env", EnvMap), ("cam", Camera), ("spp", C.c_int32), ("seed", C.c_uint64),
                ("out", Outputs)]


class ServerStats(C.Structure):
    _fields_ = [("p50_ms", C.c_double), ("p99_ms", C.c_double), ("rays_per_s", C.c_double),
                ("completed", C.c_int64), ("rejected", C.c_int64), ("rays_primary", C.c_int64),
                ("rays_secondary", C.c_int64), ("iterations", C.c_int64)]


NUM_PHASES = 17
NUM_COUNTERS = 22  # LF_NUM_COUNTERS
PHASES = ("refit", "state_env", "trace1", "shade1", "sort2", "trace2", "shade2", "resolve", "replay_primary",
          "replay_secondary", "adj_shade", "unused11", "zero_grads", "loss", "composite1", "composite2", "adj_hits")

# every symbol include/lightfuse.h declares, with its ctypes signature
SIGNATURES = {
    "lf_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]),
    "lf_destroy": (None, [C.c_void_p]),
    "lf_last_error": (C.c_char_p, [C.c_void_p]),
    "lf_sync": (C.c_int, [C.c_void_p]),
    "lf_abort": (C.c_int, [C.c_void_p]),
    "lf_sync_timeout": (C.c_int, [C.c_void_p, C.c_double]),
    "lf_scene_set": (C.c_int, [C.c_void_p, C.POINTER(Surfels)]),
    "lf_scene_refit": (C.c_int, [C.c_void_p]),
    "lf_params_default": (None, [C.POINTER(Params)]),
    "lf_render": (C.c_int, [C.c_void_p, C.POINTER(Transforms), C.POINTER(EnvMap), C.POINTER(Rays),
                            C.POINTER(Camera), C.c_int32, C.POINTER(Params), C.POINTER(Outputs)]),
    "lf_render_backward": (C.c_int, [C.c_void_p, C.POINTER(Transforms), C.POINTER(EnvMap), C.POINTER(Rays),
                                     C.POINTER(Camera), C.c_int32, C.POINTER(Params), C.POINTER(GradOut),
                                     C.POINTER(GradIn)]),
    "lf_l1_loss": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "lf_l1_loss_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "lf_loss_alpha": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "lf_loss_scale": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p, C.c_void_p]),
    "lf_loss_depth": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_float, C.c_void_p,
                                C.c_void_p]),
    "lf_loss_normal": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "lf_loss_tv": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "lf_loss_depth_normal": (C.c_int, [C.c_void_p, C.POINTER(Camera), C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "lf_raygen": (C.c_int, [C.c_void_p, C.POINTER(Camera), C.c_void_p, C.c_void_p]),
    "lf_scene_get_info": (C.c_int, [C.c_void_p, C.POINTER(SceneInfo)]),
    "lf_scene_copy_bvh": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "lf_scene_copy_wide": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]),
    "lf_stats_get": (C.c_int, [C.c_void_p, C.POINTER(RenderStats)]),
    "lf_profile_enable": (C.c_int, [C.c_void_p, C.c_int]),
    "lf_trace_counters": (C.c_int, [C.c_void_p, C.POINTER(C.c_uint64)]),
    "lf_profile_read": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "lf_server_config_default": (None, [C.POINTER(ServerConfig)]),
    "lf_server_create": (C.c_int, [C.c_void_p, C.POINTER(ServerConfig), C.POINTER(C.c_void_p)]),
    "lf_server_submit": (C.c_int, [C.c_void_p, C.POINTER(Request), C.POINTER(C.c_uint64)]),
    "lf_server_poll": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_int)]),
    "lf_server_wait": (C.c_int, [C.c_void_p, C.c_uint64]),
    "lf_server_latency": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(C.c_double)]),
    "lf_server_stats_get": (C.c_int, [C.c_void_p, C.POINTER(ServerStats)]),
    "lf_server_last_error": (C.c_char_p, [C.c_void_p]),
    "lf_server_destroy": (None, [C.c_void_p]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads liblightfuse.so and binds every declared symbol; raises if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"liblightfuse.so not found at {path}: build it with paper_2608_29269_amd/build.py "
                           "(or __graft_entry__.build()); there is no CPU fallback")
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


class LFError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, ctx=None):
    if status != LF_OK:
        msg = load().lf_last_error(ctx).decode() if ctx else ""
        raise LFError(status, msg)
