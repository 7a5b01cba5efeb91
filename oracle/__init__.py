"""ctypes wrapper of the FP64 CPU oracle (lf_oracle.c).

TEST INFRASTRUCTURE ONLY: this package is imported by tests, by the smoke
check and by the benchmark's CPU-baseline leg, never by the GPU library or its
binding.  All computation happens in lf_oracle.c in double precision; this
module only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblf_oracle.so")

NO_SECONDARY = 1 << 0
NO_BACKGROUND = 1 << 1
BSDF_ONLY = 1 << 2
DIFFUSE_ONLY = 1 << 3
SOBOL = 1 << 8  # Owen-scrambled Sobol uniforms instead of the hash
NEE = 1 << 7  # two rays per path sample (next-event + continuation); outputs per slot 2s, 2s+1

M_TGAP_PRI, M_RHO_PRI, M_TGAP_SEC, M_RHO_SEC, M_ENV, M_LOBE, M_COS, M_TMIN = range(8)
NMARGIN = 8
C_TOUCH_PRI, C_COMP_PRI, C_SEC_RAYS, C_TOUCH_SEC, C_COMP_SEC, C_ENV = range(6)
NCOUNT = 6

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_fp = C.POINTER(C.c_float)


class _Scene(C.Structure):
    _fields_ = [("mu", _dp), ("q", _dp), ("scale", _dp), ("opacity", _dp), ("albedo", _dp),
                ("roughness", _dp), ("metallic", _dp), ("n", C.c_int64), ("n_objects", C.c_int32),
                ("object_offset", _i64p), ("R", _dp), ("t", _dp), ("env", _dp),
                ("env_h", C.c_int32), ("env_w", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("k", C.c_int32), ("spp", C.c_int32), ("seed", C.c_uint64), ("alpha_min", C.c_double),
                ("alpha_cap", C.c_double), ("support_sigma", C.c_double), ("eps", C.c_double),
                ("t_min", C.c_double), ("secondary_offset", C.c_double), ("flags", C.c_uint32)]


class _Rays(C.Structure):
    _fields_ = [("o", _dp), ("d", _dp), ("id", _i64p), ("n", C.c_int64)]


class _Outputs(C.Structure):
    _fields_ = [("radiance", _dp), ("depth", _dp), ("normal", _dp), ("alpha", _dp),
                ("transmittance", _dp), ("hit_idx", _i32p), ("sec_hit_idx", _i32p),
                ("sec_alpha", _dp), ("margins", _dp), ("counts", _dp)]


class _Upstream(C.Structure):
    _fields_ = [("radiance", _dp), ("depth", _dp), ("normal", _dp), ("alpha", _dp)]


class _Grads(C.Structure):
    _fields_ = [("mu", _dp), ("q", _dp), ("scale", _dp), ("opacity", _dp), ("albedo", _dp),
                ("roughness", _dp), ("metallic", _dp), ("env", _dp)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        _lib = bind(LIB_PATH)
    return _lib


def bind(path: str):
    """Loads an oracle build at `path` and declares its C signatures (the
    tests also bind deliberately broken copies to show that the pins catch
    them)."""
    L = C.CDLL(path)
    L.ors_render.argtypes = [C.POINTER(_Scene), C.POINTER(_Rays), C.POINTER(_Params), C.POINTER(_Outputs), C.c_int]
    L.ors_render.restype = C.c_int
    L.ors_frozen_eval.argtypes = [C.POINTER(_Scene), C.POINTER(_Scene), C.POINTER(_Rays), C.POINTER(_Params),
                                  C.POINTER(_Outputs), C.c_int]
    L.ors_frozen_eval.restype = C.c_int
    L.ors_backward.argtypes = [C.POINTER(_Scene), C.POINTER(_Rays), C.POINTER(_Params), C.POINTER(_Upstream),
                               C.POINTER(_Grads), C.c_int]
    L.ors_backward.restype = C.c_int
    L.ors_raygen.argtypes = [_fp, C.c_float, C.c_int32, C.c_int32, _i64p, C.c_int64, _fp, _fp]
    L.ors_raygen.restype = None
    L.ors_tan_half.argtypes = [C.c_float]
    L.ors_tan_half.restype = C.c_float
    L.ors_splitmix64.argtypes = [C.c_uint64]
    L.ors_splitmix64.restype = C.c_uint64
    L.ors_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32]
    L.ors_uniform.restype = C.c_double
    L.ors_sobol.argtypes = [C.c_uint32, C.c_uint32]
    L.ors_sobol.restype = C.c_uint32
    L.ors_sobol_poly.argtypes = [C.c_uint32, C.POINTER(C.c_int32), C.POINTER(C.c_uint32)]
    L.ors_sobol_poly.restype = None
    L.ors_owen_scramble.argtypes = [C.c_uint32, C.c_uint32]
    L.ors_owen_scramble.restype = C.c_uint32
    L.ors_sobol_uniform.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32]
    L.ors_sobol_uniform.restype = C.c_double
    L.ors_quat_to_frame.argtypes = [_dp, _dp, _dp, _dp]
    L.ors_onb.argtypes = [_dp, _dp, _dp]
    L.ors_brdf.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_uint32, _dp]
    L.ors_ggx_D.argtypes = [C.c_double, C.c_double]
    L.ors_ggx_D.restype = C.c_double
    L.ors_smith_G1.argtypes = [C.c_double, C.c_double]
    L.ors_smith_G1.restype = C.c_double
    L.ors_q_spec.argtypes = [_dp, C.c_double, C.c_uint32]
    L.ors_q_spec.restype = C.c_double
    L.ors_pdf_bsdf.argtypes = [_dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_uint32]
    L.ors_pdf_bsdf.restype = C.c_double
    L.ors_sample_bsdf.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double, C.c_uint32, C.c_double, C.c_double,
                                  C.c_double, _dp]
    L.ors_sample_bsdf.restype = C.c_int
    L.ors_env_pdf.argtypes = [C.POINTER(_Scene), _dp]
    L.ors_env_pdf.restype = C.c_double
    L.ors_env_sample.argtypes = [C.POINTER(_Scene), C.c_double, C.c_double, _dp]
    L.ors_env_sample.restype = C.c_double
    L.ors_env_lookup.argtypes = [C.POINTER(_Scene), _dp, _dp]
    return L


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_dp):
    return None if a is None else a.ctypes.data_as(t)


@dataclasses.dataclass
class Params:
    k: int = 32
    spp: int = 1
    seed: int = 0
    alpha_min: float = 1.0 / 255.0
    alpha_cap: float = 0.99
    support_sigma: float = 3.0
    eps: float = 1e-6
    t_min: float = 1e-4
    secondary_offset: float = 1e-3
    flags: int = 0

    @property
    def slots(self) -> int:
        """Secondary-ray slots per primary ray (2 per sample in the two-ray form)."""
        return self.spp * (2 if self.flags & NEE else 1)

    def c(self) -> _Params:
        return _Params(self.k, self.spp, self.seed, self.alpha_min, self.alpha_cap, self.support_sigma,
                       self.eps, self.t_min, self.secondary_offset, self.flags)


class SceneArrays:
    """FP64 copies of a scene + one state's transforms and env, kept alive for
    the C call."""

    def __init__(self, scene, R, t, env, overrides: Optional[dict] = None):
        ov = overrides or {}
        self.mu = _d(ov.get("mu", scene.mu))
        self.q = _d(ov.get("q", scene.q))
        self.scale = _d(ov.get("scale", scene.scale))
        self.opacity = _d(ov.get("opacity", scene.opacity))
        self.albedo = _d(ov.get("albedo", scene.albedo))
        self.roughness = _d(ov.get("roughness", scene.roughness))
        self.metallic = _d(ov.get("metallic", scene.metallic))
        self.off = np.ascontiguousarray(scene.object_offset, dtype=np.int64)
        M = len(self.off) - 2
        self.R = _d(np.asarray(R).reshape(M, 3, 3)) if M > 0 else np.zeros((1, 9))
        self.t = _d(np.asarray(t).reshape(M, 3)) if M > 0 else np.zeros((1, 3))
        self.env = _d(ov.get("env", env))
        self.M = M
        self.struct = _Scene(_ptr(self.mu), _ptr(self.q), _ptr(self.scale), _ptr(self.opacity),
                             _ptr(self.albedo), _ptr(self.roughness), _ptr(self.metallic),
                             self.mu.shape[0], M, _ptr(self.off, _i64p), _ptr(self.R), _ptr(self.t),
                             _ptr(self.env), self.env.shape[0], self.env.shape[1])


def _rays(o, d, ids):
    o = _d(o).reshape(-1, 3)
    d = _d(d).reshape(-1, 3)
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    assert o.shape == d.shape and ids.shape[0] == o.shape[0]
    return (o, d, ids), _Rays(_ptr(o), _ptr(d), _ptr(ids, _i64p), o.shape[0])


def _alloc_out(n, p: Params, lists: bool):
    out = dict(radiance=np.zeros((n, 3)), depth=np.zeros(n), normal=np.zeros((n, 3)), alpha=np.zeros(n),
               transmittance=np.zeros(n), margins=np.zeros((n, NMARGIN)), counts=np.zeros((n, NCOUNT)),
               sec_alpha=np.zeros((n, p.slots)))
    if lists:
        out["hit_idx"] = np.zeros((n, p.k), dtype=np.int32)
        out["sec_hit_idx"] = np.zeros((n, p.slots, p.k), dtype=np.int32)
    s = _Outputs(_ptr(out["radiance"]), _ptr(out["depth"]), _ptr(out["normal"]), _ptr(out["alpha"]),
                 _ptr(out["transmittance"]), _ptr(out.get("hit_idx"), _i32p), _ptr(out.get("sec_hit_idx"), _i32p),
                 _ptr(out["sec_alpha"]), _ptr(out["margins"]), _ptr(out["counts"]))
    return out, s


def render(sa: SceneArrays, o, d, ids, p: Params, lists: bool = True, threads: int = 0) -> dict:
    keep, r = _rays(o, d, ids)
    out, s = _alloc_out(r.n, p, lists)
    pc = p.c()
    rc = lib().ors_render(C.byref(sa.struct), C.byref(r), C.byref(pc), C.byref(s), threads)
    if rc != 0:
        raise RuntimeError(f"ors_render failed: {rc}")
    return out


def frozen_eval(sa0: SceneArrays, sa: SceneArrays, o, d, ids, p: Params, threads: int = 0) -> dict:
    keep, r = _rays(o, d, ids)
    out, s = _alloc_out(r.n, p, False)
    pc = p.c()
    rc = lib().ors_frozen_eval(C.byref(sa0.struct), C.byref(sa.struct), C.byref(r), C.byref(pc), C.byref(s), threads)
    if rc != 0:
        raise RuntimeError(f"ors_frozen_eval failed: {rc}")
    return out


def backward(sa: SceneArrays, o, d, ids, p: Params, g_radiance=None, g_depth=None, g_normal=None,
             g_alpha=None, threads: int = 0) -> dict:
    keep, r = _rays(o, d, ids)
    n = sa.mu.shape[0]
    ups = [None if a is None else _d(a) for a in (g_radiance, g_depth, g_normal, g_alpha)]
    for a, shape in zip(ups, ((r.n, 3), (r.n,), (r.n, 3), (r.n,))):
        if a is not None and a.shape != shape:
            raise ValueError(f"upstream gradient of shape {a.shape}, expected {shape}")
    up = _Upstream(*[_ptr(a) for a in ups])
    g = dict(mu=np.zeros((n, 3)), q=np.zeros((n, 4)), scale=np.zeros((n, 2)), opacity=np.zeros(n),
             albedo=np.zeros((n, 3)), roughness=np.zeros(n), metallic=np.zeros(n), env=np.zeros(sa.env.shape))
    gs = _Grads(*[_ptr(g[k]) for k in ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic", "env")])
    pc = p.c()
    rc = lib().ors_backward(C.byref(sa.struct), C.byref(r), C.byref(pc), C.byref(up), C.byref(gs), threads)
    if rc != 0:
        raise RuntimeError(f"ors_backward failed: {rc}")
    return g


def tan_half(fov_y_deg: float) -> float:
    return float(lib().ors_tan_half(C.c_float(fov_y_deg)))


def raygen(camera, pix=None):
    """FP32 rays of `camera` (scenegen.Camera) for pixel indices pix (default all)."""
    if pix is None:
        pix = np.arange(camera.w * camera.h, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    pose = np.ascontiguousarray(camera.pose, dtype=np.float32)
    o = np.zeros((pix.shape[0], 3), dtype=np.float32)
    d = np.zeros((pix.shape[0], 3), dtype=np.float32)
    lib().ors_raygen(_ptr(pose, _fp), lib().ors_tan_half(C.c_float(camera.fov_y_deg)), camera.w, camera.h,
                     _ptr(pix, _i64p), pix.shape[0], _ptr(o, _fp), _ptr(d, _fp))
    return o, d, pix


def splitmix64(x: int) -> int:
    return int(lib().ors_splitmix64(C.c_uint64(x)))


def uniform(seed: int, ray: int, sample: int, dim: int) -> float:
    return float(lib().ors_uniform(seed, ray, sample, dim))


def sobol(i: int, d: int) -> int:
    """Raw 32-bit Sobol coordinate of point i in dimension d (< 11)."""
    return int(lib().ors_sobol(i, d))


def sobol_poly(d: int):
    """(degree s, inner coefficients a) of dimension d's polynomial
    x^s + a_1 x^(s-1) + ... + a_(s-1) x + 1, a_1 the top bit of a."""
    s, a = C.c_int32(), C.c_uint32()
    lib().ors_sobol_poly(d, C.byref(s), C.byref(a))
    return int(s.value), int(a.value)


def owen_scramble(x: int, seed: int) -> int:
    return int(lib().ors_owen_scramble(x, seed))


def sobol_uniform(seed: int, ray: int, sample: int, dim: int) -> float:
    return float(lib().ors_sobol_uniform(seed, ray, sample, dim))


def quat_to_frame(q):
    q = _d(q)
    tu, tv, n = np.zeros(3), np.zeros(3), np.zeros(3)
    lib().ors_quat_to_frame(_ptr(q), _ptr(tu), _ptr(tv), _ptr(n))
    return tu, tv, n


def onb(n):
    n = _d(n)
    b1, b2 = np.zeros(3), np.zeros(3)
    lib().ors_onb(_ptr(n), _ptr(b1), _ptr(b2))
    return b1, b2


def brdf(n, wi, wo, a, m, r, flags=0):
    n, wi, wo, a = _d(n), _d(wi), _d(wo), _d(a)
    f = np.zeros(3)
    lib().ors_brdf(_ptr(n), _ptr(wi), _ptr(wo), _ptr(a), m, r, flags, _ptr(f))
    return f


def ggx_D(ch, r):
    return float(lib().ors_ggx_D(ch, r))


def smith_G1(c, r):
    return float(lib().ors_smith_G1(c, r))


def q_spec(a, m, flags=0):
    a = _d(a)
    return float(lib().ors_q_spec(_ptr(a), m, flags))


def pdf_bsdf(n, wi, wo, a, m, r, flags=0):
    n, wi, wo, a = _d(n), _d(wi), _d(wo), _d(a)
    return float(lib().ors_pdf_bsdf(_ptr(n), _ptr(wi), _ptr(wo), _ptr(a), m, r, flags))


def sample_bsdf(n, wo, a, m, r, flags, u_lobe, u1, u2):
    n, wo, a = _d(n), _d(wo), _d(a)
    wi = np.zeros(3)
    ok = lib().ors_sample_bsdf(_ptr(n), _ptr(wo), _ptr(a), m, r, flags, u_lobe, u1, u2, _ptr(wi))
    return bool(ok), wi


def _env_scene(env):
    env = _d(env)
    off = np.array([0, 0], dtype=np.int64)
    z = np.zeros(3)
    s = _Scene(None, None, None, None, None, None, None, 0, 0, _ptr(off, _i64p), _ptr(z), _ptr(z), _ptr(env),
               env.shape[0], env.shape[1])
    return (env, off, z), s


def env_pdf(env, w):
    keep, s = _env_scene(env)
    w = _d(w)
    return float(lib().ors_env_pdf(C.byref(s), _ptr(w)))


def env_sample(env, ua, ub):
    keep, s = _env_scene(env)
    w = np.zeros(3)
    pdf = float(lib().ors_env_sample(C.byref(s), ua, ub, _ptr(w)))
    return pdf, w


def env_lookup(env, w):
    keep, s = _env_scene(env)
    w = _d(w)
    rgb = np.zeros(3)
    lib().ors_env_lookup(C.byref(s), _ptr(w), _ptr(rgb))
    return rgb


def workload_rays(camera, pix=None):
    """Rays for pixel indices of a camera, with ray ids equal to the pixel index."""
    o, d, pix = raygen(camera, pix)
    return o, d, pix
