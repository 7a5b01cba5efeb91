"""MI355X (gfx950) one-bounce ray tracer of 2D Gaussian surfels: the
data-parallel hot path of LightFuse (arXiv 2608.29269, Sec. 3).

Thin Python layer over liblightfuse.so (include/lightfuse.h): PyTorch only
provides device memory and the stream; every step runs in the HIP library.

    tr = Tracer()
    tr.set_scene(mu, q, scale, opacity, albedo, roughness, metallic, object_offset)
    out = tr.render(env, R, t, cameras=[cam], k=32, spp=1, seed=7)
    grads = tr.render_backward(env, R, t, cameras=[cam], ..., d_radiance=...)

`RenderFn` wraps the pair as a torch.autograd.Function.  `Server` serves
rearrange-and-relight requests against the tracer's scene by continuous
batching (lf_server_*).
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

from . import _lib
from ._lib import (FLAG_BRUTE_FORCE, FLAG_COUNT, FLAG_BSDF_ONLY, FLAG_DETERMINISTIC, FLAG_DIFFUSE_ONLY, FLAG_NEE,
                   FLAG_NO_BACKGROUND, FLAG_NO_SECONDARY, FLAG_SOBOL, LFError)

__all__ = ["Tracer", "RenderFn", "Server", "LFError", "FLAG_NO_SECONDARY", "FLAG_NO_BACKGROUND", "FLAG_BSDF_ONLY",
           "FLAG_DIFFUSE_ONLY", "FLAG_BRUTE_FORCE", "FLAG_NEE", "FLAG_SOBOL", "FLAG_DETERMINISTIC", "camera_struct"]


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_tensor(t, name, shape_tail, n=None):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
        raise ValueError(f"{name} must be a float32 CUDA tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape[1:]) != tuple(shape_tail) or (n is not None and t.shape[0] != n):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [{n}, {', '.join(map(str, shape_tail))}]")


def _check_f32(t):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 CUDA tensor")


def camera_struct(cam) -> _lib.Camera:
    """lf_camera from an object with pose[12], fov_y_deg, w, h."""
    c = _lib.Camera()
    for i, v in enumerate(list(cam.pose)):
        c.pose[i] = float(v)
    c.fov_y_deg = float(cam.fov_y_deg)
    c.w = int(cam.w)
    c.h = int(cam.h)
    return c


class Tracer:
    """One lf_ctx bound to a device and the current torch stream."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.L = _lib.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        ctx = C.c_void_p()
        st = self.L.lf_create(C.byref(ctx), device, C.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise LFError(st, "lf_create failed")
        self.ctx = ctx
        self.scene = None
        self.n = 0
        self.n_objects = 0

    def close(self):
        if getattr(self, "ctx", None):
            self.L.lf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, st):
        _lib.check(st, self.ctx)

    # ------------------------------------------------------------------ scene
    def set_scene(self, mu, q, scale, opacity, albedo, roughness, metallic, object_offset: Sequence[int]):
        n = int(mu.shape[0])
        for t, nm, tail in ((mu, "mu", (3,)), (q, "q", (4,)), (scale, "scale", (2,)), (opacity, "opacity", ()),
                            (albedo, "albedo", (3,)), (roughness, "roughness", ()), (metallic, "metallic", ())):
            _check_tensor(t, nm, tail, n)
        off = (C.c_int64 * len(object_offset))(*[int(x) for x in object_offset])
        s = _lib.Surfels(_ptr(mu), _ptr(q), _ptr(scale), _ptr(opacity), _ptr(albedo), _ptr(roughness),
                         _ptr(metallic), n, len(object_offset) - 2, C.cast(off, C.POINTER(C.c_int64)))
        # the library retains the pointers: keep the tensors alive
        self.scene = dict(mu=mu, q=q, scale=scale, opacity=opacity, albedo=albedo, roughness=roughness,
                          metallic=metallic)
        self.object_offset = [int(x) for x in object_offset]
        self._chk(self.L.lf_scene_set(self.ctx, C.byref(s)))
        self.n = n
        self.n_objects = len(object_offset) - 2

    def refit(self):
        self._chk(self.L.lf_scene_refit(self.ctx))

    def info(self) -> dict:
        i = _lib.SceneInfo()
        self._chk(self.L.lf_scene_get_info(self.ctx, C.byref(i)))
        return dict(n_instances=i.n_instances, n_surfels=i.n_surfels, n_nodes=i.n_nodes, max_depth=i.max_depth,
                    stack_size=i.stack_size, n_wide_nodes=i.n_wide_nodes, wide_levels=i.wide_levels,
                    node_width=i.node_width)

    def copy_bvh(self, inst: int):
        import numpy as np
        n = self.object_offset[inst + 1] - self.object_offset[inst]
        nn = max(n - 1, 0)
        boxes = np.zeros((nn, 2, 6), np.float32)
        ch = np.zeros((nn, 2), np.int32)
        perm = np.zeros(n, np.int32)
        leaf = np.zeros((n, 6), np.float32)
        self._chk(self.L.lf_scene_copy_bvh(self.ctx, inst, boxes.ctypes.data, ch.ctypes.data, perm.ctypes.data,
                                           leaf.ctypes.data))
        return boxes, ch, perm, leaf

    def copy_wide(self, inst: int):
        """Decoded traversal nodes of one instance: slot boxes [m, W, 6] and children [m, W]."""
        import numpy as np
        m = C.c_int64(0)
        self._chk(self.L.lf_scene_copy_wide(self.ctx, inst, C.byref(m), None, None))
        w = self.info()["node_width"]
        boxes = np.zeros((m.value, w, 6), np.float32)
        ch = np.zeros((m.value, w), np.int32)
        self._chk(self.L.lf_scene_copy_wide(self.ctx, inst, C.byref(m), boxes.ctypes.data, ch.ctypes.data))
        return boxes, ch

    # ------------------------------------------------------------------ calls
    @staticmethod
    def params(k=32, spp=1, seed=0, flags=0, **kw) -> _lib.Params:
        p = _lib.Params()
        _lib.load().lf_params_default(C.byref(p))
        p.k, p.spp, p.seed, p.flags = int(k), int(spp), int(seed), int(flags)
        for key, v in kw.items():
            setattr(p, key, v)
        return p

    def _args(self, env, R, t, rays, cameras):
        import torch
        _check_tensor(env, "env", (env.shape[1], 3))
        em = _lib.EnvMap(_ptr(env), env.shape[0], env.shape[1])
        if self.n_objects > 0:
            _check_tensor(R, "R", (3, 3), self.n_objects)
            _check_tensor(t, "t", (3,), self.n_objects)
        xf = _lib.Transforms(_ptr(R) if self.n_objects else None, _ptr(t) if self.n_objects else None)
        if rays is not None:
            o, d = rays
            _check_tensor(o, "rays.o", (3,))
            _check_tensor(d, "rays.d", (3,), o.shape[0])
            rs = _lib.Rays(_ptr(o), _ptr(d), o.shape[0])
            return em, xf, C.byref(rs), None, 0, int(o.shape[0]), rs
        cams = (_lib.Camera * len(cameras))(*[camera_struct(c) for c in cameras])
        R_ = sum(int(c.w) * int(c.h) for c in cameras)
        return em, xf, None, cams, len(cameras), R_, None

    def render(self, env, R=None, t=None, rays=None, cameras=None, k=32, spp=1, seed=0, flags=0,
               hit_idx=False, sec_hit_idx=False, out=None, **kw) -> dict:
        import torch
        em, xf, rp, cams, nc, nr, keep = self._args(env, R, t, rays, cameras)
        p = self.params(k, spp, seed, flags, **kw)
        dev = self.device
        if out is None:
            out = dict(radiance=torch.empty((nr, 3), device=dev), depth=torch.empty(nr, device=dev),
                       normal=torch.empty((nr, 3), device=dev), alpha=torch.empty(nr, device=dev))
            if hit_idx:
                out["hit_idx"] = torch.empty((nr, k), dtype=torch.int32, device=dev)
            if sec_hit_idx:
                slots = spp * (2 if int(flags) & FLAG_NEE else 1)
                out["sec_hit_idx"] = torch.empty((nr, slots, k), dtype=torch.int32, device=dev)
        o = _lib.Outputs(_ptr(out["radiance"]), _ptr(out["depth"]), _ptr(out["normal"]), _ptr(out["alpha"]),
                         _ptr(out.get("hit_idx")), _ptr(out.get("sec_hit_idx")))
        self._chk(self.L.lf_render(self.ctx, C.byref(xf), C.byref(em), rp, cams, nc, C.byref(p), C.byref(o)))
        return out

    def render_backward(self, env, R=None, t=None, rays=None, cameras=None, k=32, spp=1, seed=0, flags=0,
                        d_radiance=None, d_depth=None, d_normal=None, d_alpha=None, grads=None, **kw) -> dict:
        import torch
        em, xf, rp, cams, nc, nr, keep = self._args(env, R, t, rays, cameras)
        p = self.params(k, spp, seed, flags, **kw)
        for g, nm, tail in ((d_radiance, "d_radiance", (3,)), (d_depth, "d_depth", ()),
                            (d_normal, "d_normal", (3,)), (d_alpha, "d_alpha", ())):
            if g is not None:
                _check_tensor(g, nm, tail, nr)
        if grads is None:
            grads = {k_: torch.empty_like(v) for k_, v in self.scene.items()}
            grads["env"] = torch.empty_like(env)
        go = _lib.GradOut(_ptr(d_radiance), _ptr(d_depth), _ptr(d_normal), _ptr(d_alpha))
        gi = _lib.GradIn(_ptr(grads["mu"]), _ptr(grads["q"]), _ptr(grads["scale"]), _ptr(grads["opacity"]),
                         _ptr(grads["albedo"]), _ptr(grads["roughness"]), _ptr(grads["metallic"]),
                         _ptr(grads["env"]))
        self._chk(self.L.lf_render_backward(self.ctx, C.byref(xf), C.byref(em), rp, cams, nc, C.byref(p),
                                            C.byref(go), C.byref(gi)))
        return grads

    def l1_loss(self, pred, target, want_grad=True):
        import torch
        if pred.shape != target.shape:
            raise ValueError("pred and target shapes differ")
        loss = torch.empty((), device=self.device)
        grad = torch.empty_like(pred) if want_grad else None
        self._chk(self.L.lf_l1_loss(self.ctx, _ptr(pred), _ptr(target), pred.numel(), _ptr(loss), _ptr(grad)))
        return loss, grad

    def l1_loss_noalloc(self, pred, target, loss, grad=None):
        """lf_l1_loss_noalloc: the L1 objective into caller-provided outputs
        (loss: device scalar, grad: like pred or None), no device allocation."""
        if pred.shape != target.shape or (grad is not None and grad.shape != pred.shape):
            raise ValueError("pred, target and grad shapes differ")
        self._chk(self.L.lf_l1_loss_noalloc(self.ctx, _ptr(pred), _ptr(target), pred.numel(), _ptr(loss),
                                            _ptr(grad)))
        return loss, grad

    # -- geometry-refinement objectives (Sec. 3.1, 3.2); each returns
    #    (loss device scalar, gradient w.r.t. the first map or None)
    def _loss_out(self, like, want_grad):
        import torch
        return torch.empty((), device=self.device), (torch.empty_like(like) if want_grad else None)

    def loss_alpha(self, alpha, want_grad=True):
        """L_alpha = mean |A - 1| over the accumulated-opacity map (Eq. alpha-coverage)."""
        _check_f32(alpha)
        loss, grad = self._loss_out(alpha, want_grad)
        self._chk(self.L.lf_loss_alpha(self.ctx, _ptr(alpha), alpha.numel(), _ptr(loss), _ptr(grad)))
        return loss, grad

    def loss_scale(self, scale, s_max, want_grad=True):
        """L_s over in-plane scales [N,2] (Eq. scale-regularization)."""
        _check_f32(scale)
        if scale.dim() != 2 or scale.shape[1] != 2:
            raise ValueError("scale must be [N,2]")
        loss, grad = self._loss_out(scale, want_grad)
        self._chk(self.L.lf_loss_scale(self.ctx, _ptr(scale), scale.shape[0], float(s_max), _ptr(loss), _ptr(grad)))
        return loss, grad

    def loss_depth(self, depth, ref, conf=None, eps=1e-6, want_grad=True):
        """L_D, confidence-weighted relative L1 on depth (Eq. reconstruction-depth); conf None means 1."""
        for t in (depth, ref) + ((conf,) if conf is not None else ()):
            _check_f32(t)
            if t.numel() != depth.numel():
                raise ValueError("depth, ref and conf sizes differ")
        loss, grad = self._loss_out(depth, want_grad)
        self._chk(self.L.lf_loss_depth(self.ctx, _ptr(depth), _ptr(ref), _ptr(conf), depth.numel(), float(eps),
                                       _ptr(loss), _ptr(grad)))
        return loss, grad

    def loss_normal(self, normal, ref, want_grad=True):
        """L_N = 1 - mean <N, N*> over [P,3] normal maps (Eq. reconstruction-normal)."""
        _check_f32(normal)
        _check_f32(ref)
        if normal.shape != ref.shape or normal.dim() != 2 or normal.shape[1] != 3:
            raise ValueError("normal and ref must both be [P,3]")
        loss, grad = self._loss_out(normal, want_grad)
        self._chk(self.L.lf_loss_normal(self.ctx, _ptr(normal), _ptr(ref), normal.shape[0], _ptr(loss), _ptr(grad)))
        return loss, grad

    def loss_tv(self, env, want_grad=True):
        """L_TV of a lat-long environment map [H,W,3] (Eq. training-objectives)."""
        _check_f32(env)
        if env.dim() != 3 or env.shape[2] != 3:
            raise ValueError("env must be [H,W,3]")
        loss, grad = self._loss_out(env, want_grad)
        self._chk(self.L.lf_loss_tv(self.ctx, _ptr(env), env.shape[0], env.shape[1], _ptr(loss), _ptr(grad)))
        return loss, grad

    def loss_depth_normal(self, camera, depth, ref, want_grad=True):
        """L_DN on the normals derived from the rendered depth of `camera` (Eq. reconstruction-normal)."""
        _check_f32(depth)
        _check_f32(ref)
        n = int(camera.w) * int(camera.h)
        if depth.numel() != n or ref.numel() != 3 * n:
            raise ValueError("depth must hold w*h values and ref w*h normals")
        c = camera_struct(camera)
        loss, grad = self._loss_out(depth, want_grad)
        self._chk(self.L.lf_loss_depth_normal(self.ctx, C.byref(c), _ptr(depth), _ptr(ref), _ptr(loss), _ptr(grad)))
        return loss, grad

    def raygen(self, camera):
        import torch
        n = int(camera.w) * int(camera.h)
        o = torch.empty((n, 3), device=self.device)
        d = torch.empty((n, 3), device=self.device)
        c = camera_struct(camera)
        self._chk(self.L.lf_raygen(self.ctx, C.byref(c), _ptr(o), _ptr(d)))
        return o, d

    def sync(self, timeout_ms=None):
        """Waits for the context's stream (lf_sync); with timeout_ms, a host
        watchdog cuts the traversal short after that long (lf_sync_timeout,
        LF_ETIMEOUT)."""
        if timeout_ms is None:
            self._chk(self.L.lf_sync(self.ctx))
        else:
            self._chk(self.L.lf_sync_timeout(self.ctx, float(timeout_ms)))

    def abort(self):
        """Raises the context's abort word (lf_abort; any thread): the work
        already enqueued drains without further traversal and the next sync
        raises LF_EABORTED."""
        self._chk(self.L.lf_abort(self.ctx))

    def stats(self) -> dict:
        st = _lib.RenderStats()
        self._chk(self.L.lf_stats_get(self.ctx, C.byref(st)))
        return dict(rays_primary=st.rays_primary, rays_secondary=st.rays_secondary)

    def trace_counters(self) -> dict:
        c = (C.c_uint64 * _lib.NUM_COUNTERS)()
        self._chk(self.L.lf_trace_counters(self.ctx, c))
        keys = ("rays", "nodes", "tests", "inserts")
        p, s_ = dict(zip(keys, c[:4])), dict(zip(keys, c[4:8]))
        for i, name in enumerate(("ties", "prefilter_pass", "valid_hits", "stack_pushes", "stack_deepest",
                                  "hinted", "hint_retries")):
            p[name], s_[name] = c[8 + 2 * i], c[9 + 2 * i]
        return {"primary": p, "secondary": s_}

    def profile(self, enable: bool = True):
        self._chk(self.L.lf_profile_enable(self.ctx, int(enable)))

    def profile_read(self) -> dict:
        ms = (C.c_double * _lib.NUM_PHASES)()
        n = (C.c_int64 * _lib.NUM_PHASES)()
        self._chk(self.L.lf_profile_read(self.ctx, ms, n))
        return {name: (ms[i], n[i]) for i, name in enumerate(_lib.PHASES)}


class Server:
    """Relight server over a Tracer's scene (lf_server_*): requests carry
    per-object transforms, an environment map, one camera, S and a seed; the
    library batches all admitted requests into shared wavefront passes.
    Request tensors are kept alive here until the request has completed."""

    def __init__(self, tracer: Tracer, max_slots=16, hbm_budget_bytes=16 << 30, tile_rays=65536,
                 batch_rays=1048576, max_spp=4, max_pending=4096, policy=_lib.SCHED_OLDEST_FIRST,
                 max_in_flight=2, k=32, flags=0, **kw):
        self.L = tracer.L
        self.tracer = tracer
        cfg = _lib.ServerConfig()
        self.L.lf_server_config_default(C.byref(cfg))
        cfg.max_slots, cfg.hbm_budget_bytes, cfg.tile_rays = int(max_slots), int(hbm_budget_bytes), int(tile_rays)
        cfg.batch_rays, cfg.max_spp, cfg.max_pending = int(batch_rays), int(max_spp), int(max_pending)
        cfg.policy, cfg.max_in_flight = int(policy), int(max_in_flight)
        cfg.params = Tracer.params(k, max_spp, 0, flags, **kw)
        srv = C.c_void_p()
        tracer._chk(self.L.lf_server_create(tracer.ctx, C.byref(cfg), C.byref(srv)))
        self.srv = srv
        self.cfg = cfg
        self._keep = {}

    def _chk(self, st):
        if st != 0:
            raise LFError(st, self.L.lf_server_last_error(self.srv).decode())

    def submit(self, env, camera, R=None, t=None, spp=1, seed=0, out=None) -> int:
        """Enqueues a request and returns its ticket; env, R, t are float32
        tensors (CUDA or CPU), outputs are allocated unless given."""
        import torch
        n = int(camera.w) * int(camera.h)
        dev = self.tracer.device
        if out is None:
            out = dict(radiance=torch.empty((n, 3), device=dev), depth=torch.empty(n, device=dev),
                       normal=torch.empty((n, 3), device=dev), alpha=torch.empty(n, device=dev))
        for key, tail in (("radiance", (3,)), ("depth", ()), ("normal", (3,)), ("alpha", ())):
            _check_tensor(out[key], key, tail, n)
        for x, nm in ((env, "env"), (R, "R"), (t, "t")):
            if x is not None and (x.dtype != torch.float32 or not x.is_contiguous()):
                raise ValueError(f"{nm} must be a contiguous float32 tensor")
        if env.dim() != 3 or env.shape[2] != 3:
            raise ValueError("env must be [H, W, 3]")
        m = self.tracer.n_objects
        if m > 0 and (R is None or t is None or tuple(R.shape) != (m, 3, 3) or tuple(t.shape) != (m, 3)):
            raise ValueError(f"R and t must be [{m},3,3] and [{m},3]")
        req = _lib.Request()
        req.xf = _lib.Transforms(_ptr(R) if m else None, _ptr(t) if m else None)
        req.env = _lib.EnvMap(_ptr(env), env.shape[0], env.shape[1])
        req.cam = camera_struct(camera)
        req.spp, req.seed = int(spp), int(seed)
        req.out = _lib.Outputs(_ptr(out["radiance"]), _ptr(out["depth"]), _ptr(out["normal"]), _ptr(out["alpha"]),
                               None, None)
        tk = C.c_uint64()
        self._chk(self.L.lf_server_submit(self.srv, C.byref(req), C.byref(tk)))
        self._keep[tk.value] = (env, R, t, out)
        return tk.value

    def poll(self, ticket: int) -> bool:
        done = C.c_int()
        self._chk(self.L.lf_server_poll(self.srv, int(ticket), C.byref(done)))
        return bool(done.value)

    def wait(self, ticket: int) -> dict:
        """Blocks until the request completes; returns its outputs."""
        self._chk(self.L.lf_server_wait(self.srv, int(ticket)))
        return self._keep.pop(int(ticket))[3]

    def result(self, ticket: int) -> dict:
        """Outputs of a completed request (after poll returned True)."""
        return self._keep.pop(int(ticket))[3]

    def latency_ms(self, ticket: int) -> float:
        ms = C.c_double()
        self._chk(self.L.lf_server_latency(self.srv, int(ticket), C.byref(ms)))
        return ms.value

    def stats(self) -> dict:
        st = _lib.ServerStats()
        self._chk(self.L.lf_server_stats_get(self.srv, C.byref(st)))
        return {f: getattr(st, f) for f, _ in _lib.ServerStats._fields_}

    def close(self):
        if getattr(self, "srv", None):
            self.L.lf_server_destroy(self.srv)
            self.srv = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _render_fn():
    import torch

    class RenderFn(torch.autograd.Function):
        """Differentiable render: forward -> lf_render, backward -> lf_render_backward
        (path replay; hit lists are recomputed, not saved).  The scene tensors must
        be the ones registered with tracer.set_scene; they are refit on entry."""

        @staticmethod
        def forward(ctx, tracer, cfg, mu, q, scale, opacity, albedo, roughness, metallic, env):
            for k_, v in zip(("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic"),
                             (mu, q, scale, opacity, albedo, roughness, metallic)):
                if tracer.scene is None or tracer.scene[k_].data_ptr() != v.data_ptr():
                    raise ValueError(f"{k_} is not the tensor registered with Tracer.set_scene")
            tracer.refit()
            out = tracer.render(env, **cfg)
            ctx.tracer, ctx.cfg = tracer, cfg
            ctx.save_for_backward(env)
            return out["radiance"], out["depth"], out["normal"], out["alpha"]

        @staticmethod
        def backward(ctx, g_rad, g_depth, g_normal, g_alpha):
            (env,) = ctx.saved_tensors
            cfg = {k_: v for k_, v in ctx.cfg.items() if k_ not in ("hit_idx", "sec_hit_idx")}
            cont = (lambda g: None if g is None else g.contiguous())
            g = ctx.tracer.render_backward(env, d_radiance=cont(g_rad), d_depth=cont(g_depth),
                                           d_normal=cont(g_normal), d_alpha=cont(g_alpha), **cfg)
            return (None, None, g["mu"], g["q"], g["scale"], g["opacity"], g["albedo"], g["roughness"],
                    g["metallic"], g["env"])

    return RenderFn


class _Lazy:
    _cls = None

    def __get__(self, obj, owner):
        if _Lazy._cls is None:
            _Lazy._cls = _render_fn()
        return _Lazy._cls


class _NS:
    RenderFn = _Lazy()


def __getattr__(name):
    if name == "RenderFn":
        return _NS.RenderFn
    raise AttributeError(name)
