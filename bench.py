"""Benchmark of the one-bounce surfel ray tracer on one MI355X.

Workload: the resident serving scene (1M surfels: 760k background surfels on
20 surface-like shapes plus 8 rigidly moved objects of 30k surfels), one
1024x1024 pinhole camera, k = 32, S = 4 secondary samples per primary hit,
256x512 lognormal environment map with a bright lobe.  One step is one pass
of the whole differentiable hot path: bottom-up refit of the hierarchies,
per-state instance records and environment tables, ray generation,
traversal + k-closest hit buffers, compositing, S sampled directions with
ballot-compacted secondary rays, secondary traces and shading, the
scene-linear L1 loss against a target rendered from perturbed parameters,
the replayed backward pass (hit lists recomputed), and an SGD update of all
parameters.  The metric counts traced rays (primary + live secondary rays)
per second of fwd+bwd steps; forward-only rays/s and per-phase timings are
reported alongside, and a serving run (Poisson stream of rearrange-and-relight
requests) gives p50/p99 latency of the continuous-batching server against the
plain tracer serving the same stream one request at a time.

python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


class Marker:
    """A roctx range around a timed region (rocprofv3 --marker-trace shows it,
    so a kernel trace can be cut to one leg); a no-op without the library."""
    _lib = None

    def __init__(self, name):
        self.name = name.encode()

    def __enter__(self):
        if Marker._lib is None:
            import ctypes
            try:
                Marker._lib = ctypes.CDLL("librocprofiler-sdk-roctx.so.1")
                Marker._lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
            except OSError:
                Marker._lib = False
        if Marker._lib:
            Marker._lib.roctxRangePushA(self.name)
        return self

    def __exit__(self, *exc):
        if Marker._lib:
            Marker._lib.roctxRangePop()
        return False


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--spp", type=int, default=4)
    ap.add_argument("--res", type=int, default=1024)
    ap.add_argument("--scale", type=float, default=1.0, help="surfel-count scale (1.0 = 1M surfels)")
    ap.add_argument("--cpu-sample", type=int, default=1024,
                    help="primary rays of the CPU-baseline sample on all cores (median of 3 runs)")
    ap.add_argument("--cpu-sample-1core", type=int, default=128,
                    help="primary rays of the single-core CPU-baseline sample (median of 3 runs; 0 = skip)")
    ap.add_argument("--s1-steps", type=int, default=3, help="timed steps of the S = 1 leg (0 = skip)")
    ap.add_argument("--config-rows", type=str, default="1,2,3,4",
                    help="comma-separated configurations C1-C4 timed as secondary rows (empty = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fwd-steps", type=int, default=5)
    ap.add_argument("--geo-steps", type=int, default=10, help="timed geometry-refinement steps (0 = skip)")
    ap.add_argument("--ir-steps", type=int, default=30,
                    help="iterations of the staged inverse-rendering loop (0 = skip)")
    ap.add_argument("--nee-spp", type=str, default="8,16,32",
                    help="comma-separated spp of the two-ray estimator's training steps (empty = skip)")
    ap.add_argument("--serve-requests", type=int, default=500, help="requests per serving run (0 = skip)")
    ap.add_argument("--serve-loads", type=str, default="0.5,0.8",
                    help="comma-separated arrival rates as fractions of the plain tracer's capacity")
    ap.add_argument("--serve-policies", type=str, default="1",
                    help="comma-separated pass-filling policies (0 shortest first, 1 oldest first, 2 round robin)")
    ap.add_argument("--serve-batch", type=int, default=1048576, help="primary rays per batched pass")
    ap.add_argument("--serve-in-flight", type=int, default=3, help="concurrent passes (one stream each)")
    ap.add_argument("--serve-only", action="store_true", help="skip the fwd+bwd and CPU legs")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB device to device (calibrates HBM byte counters)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (each GPU would hold its "
              "own copy of the scene and trace its share of the rays); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_probe:
        src = torch.ones(1 << 28, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 4}))
        return

    import paper_2608_29269_amd as lf
    import scenegen

    dev = torch.device("cuda", 0)
    wl = scenegen.make_workload(5, scale=args.scale, resolution=args.res)
    st = wl.states[0]
    cam = st.cameras[0]
    sc = wl.scene
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    params = dict(mu=T(sc.mu), q=T(sc.q), scale=T(sc.scale), opacity=T(sc.opacity), albedo=T(sc.albedo),
                  roughness=T(sc.roughness), metallic=T(sc.metallic))
    env = T(st.env)
    R, t = T(st.R), T(st.t)
    cfg = dict(cameras=[cam], k=wl.k, spp=args.spp, seed=wl.seed)

    # target from perturbed parameters (separate context, built once)
    tgt_scene = scenegen.perturb_scene(np.random.default_rng(2000), sc)
    ttr = lf.Tracer(0)
    tp = dict(mu=T(tgt_scene.mu), q=T(tgt_scene.q), scale=T(tgt_scene.scale), opacity=T(tgt_scene.opacity),
              albedo=T(tgt_scene.albedo), roughness=T(tgt_scene.roughness), metallic=T(tgt_scene.metallic))
    ttr.set_scene(**tp, object_offset=list(sc.object_offset))
    tgt = ttr.render(env, R, t, **cfg)
    target = tgt["radiance"].clone()
    # reference maps of the geometry objectives: depth, normals and a coverage-based confidence
    geo_ref = dict(depth=tgt["depth"].clone(), normal=tgt["normal"].clone(),
                   conf=(tgt["alpha"] > 0.5).float())
    ttr.sync()
    del ttr

    tr = lf.Tracer(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tr.set_scene(**params, object_offset=list(sc.object_offset))
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    info = tr.info()
    nr = cam.w * cam.h
    out = dict(radiance=torch.empty((nr, 3), device=dev), depth=torch.empty(nr, device=dev),
               normal=torch.empty((nr, 3), device=dev), alpha=torch.empty(nr, device=dev))
    grads = {k: torch.empty_like(v) for k, v in params.items()}
    grads["env"] = torch.empty_like(env)
    lr = 1e-5

    if args.serve_only:
        serving = serve_bench(tr, sc, args, [float(x) for x in args.serve_loads.split(",") if x],
                              [int(x) for x in args.serve_policies.split(",") if x])
        print(json.dumps({"serving": serving}))
        return

    def step():
        tr.refit()
        tr.render(env, R, t, out=out, **cfg)
        loss, g = tr.l1_loss(out["radiance"], target)
        tr.render_backward(env, R, t, d_radiance=g, grads=grads, **cfg)
        with torch.no_grad():
            for k_, v in params.items():
                v.sub_(lr * grads[k_])
            env.sub_(lr * grads["env"]).clamp_(min=0.0)
            params["scale"].clamp_(min=1e-4)
            params["opacity"].clamp_(1e-4, 1.0)
            for k_ in ("albedo", "roughness", "metallic"):
                params[k_].clamp_(0.0, 1.0)
        return loss

    log(f"scene {sc.n} surfels, hierarchy built in {build_ms:.1f} ms; warmup {args.warmup} steps")
    for _ in range(args.warmup):
        step()
    tr.sync()
    log(f"timing {args.steps} fwd+bwd steps")
    tr.stats()
    tr.profile(True)
    tr.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    phases = tr.profile_read()
    tr.profile(False)
    stats = tr.stats()
    tr.sync()
    rays = stats["rays_primary"] + stats["rays_secondary"]
    value = rays / dt
    ms_per_step = dt * 1e3 / args.steps

    log(f"fwd+bwd: {ms_per_step:.2f} ms/step, {value:.4g} rays/s; timing forward only")
    # forward only (M1)
    for _ in range(2):
        tr.refit()
        tr.render(env, R, t, out=out, **cfg)
    tr.sync()
    tr.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.fwd_steps):
        tr.refit()
        tr.render(env, R, t, out=out, **cfg)
    torch.cuda.synchronize()
    dtf = time.perf_counter() - t0
    sf = tr.stats()
    fwd_rays_s = (sf["rays_primary"] + sf["rays_secondary"]) / dtf

    # CPU baseline (the FP64 oracle as it stands) on a bounded sample of the same workload
    cpu = None
    counts = None
    if not args.no_cpu_baseline:
        log(f"forward: {fwd_rays_s:.4g} rays/s; CPU oracle on {args.cpu_sample} rays")
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        v, secs, counts = cpu_oracle_rate(sc, st, cam, wl, args.spp, args.cpu_sample, threads, nr, seed=0)
        cpu = {"value": v, "unit": "rays/s", "cores": int(threads), "kind": "oracle",
               "sample": f"{args.cpu_sample} random pixels of the 1024x1024 camera (plus their live secondary "
                         f"rays), fwd+bwd, 1M surfels brute force in FP64; median of 3 runs "
                         f"({', '.join(f'{x:.1f}' for x in secs)} s)"}
        if args.cpu_sample_1core > 0:
            log(f"CPU oracle on one core, {args.cpu_sample_1core} rays")
            v1, secs1, _ = cpu_oracle_rate(sc, st, cam, wl, args.spp, args.cpu_sample_1core, 1, nr, seed=1)
            cpu["single_core"] = {"value": v1, "cores": 1,
                                  "sample": f"{args.cpu_sample_1core} random pixels, same work; median of 3 "
                                            f"runs ({', '.join(f'{x:.1f}' for x in secs1)} s)"}

    s1 = None
    if args.s1_steps > 0:
        log("S = 1 leg")
        s1 = s1_bench(tr, env, R, t, cam, wl, params, grads, out, target, args.s1_steps)

    estimator = None
    nee_spp = [int(x) for x in args.nee_spp.split(",") if x]
    if nee_spp:
        log(f"two-ray estimator at spp {nee_spp}")
        estimator = estimator_bench(lf, tr, env, R, t, cam, wl, params, grads, out, target, nee_spp)

    geometry = None
    if args.geo_steps > 0:
        log("geometry-refinement step")
        geometry = geometry_bench(lf, tr, env, R, t, cam, wl, params, grads, out, geo_ref, args)

    inverse = None
    if args.ir_steps > 0:
        log(f"staged inverse rendering, {args.ir_steps} iterations")
        inverse = inverse_rendering_bench(lf, tr, sc, wl, params, grads, args)

    serving = None
    if args.serve_requests > 0:
        serving = serve_bench(tr, sc, args, [float(x) for x in args.serve_loads.split(",") if x],
                              [int(x) for x in args.serve_policies.split(",") if x])

    rows = None
    cfg_rows = [int(x) for x in args.config_rows.split(",") if x]
    if cfg_rows:
        log(f"configuration rows {cfg_rows}")
        del tr
        torch.cuda.empty_cache()
        rows = config_rows(lf, cfg_rows)

    copy_gbs = copy_bandwidth(torch)
    roof = roofline(phases, counts, stats, args, nr, copy_gbs)
    res = {
        "metric": "rays/s fwd+bwd at 1M surfels",
        "value": float(value),
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(ms_per_step),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 decisions / f32 values",
        "data": "synthetic",
        "config": {"workload": f"resident scene {sc.n} surfels (760k background + 8x30k objects), "
                               f"{cam.w}x{cam.h} camera, k={wl.k}, S={args.spp}, 256x512 env; "
                               "refit + forward + L1 + replayed backward + SGD per step",
                   "surfels": int(sc.n), "resolution": [cam.w, cam.h], "k": wl.k, "spp": args.spp},
        "fwd_rays_per_s": float(fwd_rays_s),
        "s1": s1,
        "config_rows": rows,
        "rays_per_step": {"primary": stats["rays_primary"] / args.steps,
                          "secondary": stats["rays_secondary"] / args.steps},
        "bvh_build_ms": build_ms,
        "bvh": info,
        "loss": float(loss),
        "phases_ms_per_step": {k_: v[0] / args.steps for k_, v in phases.items() if v[1]},
        "roofline": roof,
        "cpu_baseline": cpu,
        "geometry": geometry,
        "two_ray_estimator": estimator,
        "inverse_rendering": inverse,
        "serving": serving,
    }
    print(json.dumps(res))


def cpu_oracle_rate(sc, st, cam, wl, spp, n_pix, threads, nr, seed):
    """The FP64 oracle's fwd+bwd rays/s on n_pix random pixels of the camera
    (plus their live secondary rays) with `threads` OpenMP threads: median of
    3 runs.  Also returns the per-ray counts of the first run."""
    import oracle
    rng = np.random.default_rng(seed)
    pix = np.sort(rng.choice(nr, n_pix, replace=False))
    o, d, ids = oracle.raygen(cam, pix)
    sa = oracle.SceneArrays(sc, st.R, st.t, st.env)
    p = oracle.Params(k=wl.k, spp=spp, seed=wl.seed)
    rates, secs, counts = [], [], None
    for _ in range(3):
        c0 = time.perf_counter()
        ref = oracle.render(sa, o, d, ids, p, lists=False, threads=threads)
        oracle.backward(sa, o, d, ids, p, g_radiance=np.sign(ref["radiance"]) / (3.0 * nr), threads=threads)
        cdt = time.perf_counter() - c0
        if counts is None:
            counts = ref["counts"]
        rays = len(pix) + ref["counts"][:, oracle.C_SEC_RAYS].sum()
        rates.append(rays / cdt)
        secs.append(cdt)
    return float(np.median(rates)), secs, counts


def s1_bench(tr, env, R, t, cam, wl, params, grads, out, target, steps, lr=1e-5):
    """M1 (forward) and M2 (fwd+bwd) rays/s at S = 1 on the benchmark scene
    and camera: one warm-up, then `steps` timed steps of each."""
    import torch
    cfg = dict(cameras=[cam], k=wl.k, spp=1, seed=wl.seed)

    def step():
        tr.refit()
        tr.render(env, R, t, out=out, **cfg)
        loss, g = tr.l1_loss(out["radiance"], target)
        tr.render_backward(env, R, t, d_radiance=g, grads=grads, **cfg)
        with torch.no_grad():
            for k_, v in params.items():
                v.sub_(lr * grads[k_])
            params["scale"].clamp_(min=1e-4)
            params["opacity"].clamp_(1e-4, 1.0)
            for k_ in ("albedo", "roughness", "metallic"):
                params[k_].clamp_(0.0, 1.0)

    step()
    tr.sync()
    tr.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = tr.stats()
    fb = (st["rays_primary"] + st["rays_secondary"]) / dt
    tr.render(env, R, t, out=out, **cfg)
    tr.sync()
    tr.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tr.refit()
        tr.render(env, R, t, out=out, **cfg)
    torch.cuda.synchronize()
    dtf = time.perf_counter() - t0
    sf = tr.stats()
    res = {"fwd_bwd_rays_per_s": fb, "fwd_bwd_ms_per_step": dt * 1e3 / steps,
           "fwd_rays_per_s": (sf["rays_primary"] + sf["rays_secondary"]) / dtf,
           "fwd_ms": dtf * 1e3 / steps, "secondary_rays_per_step": sf["rays_secondary"] / steps}
    log(f"S=1: fwd+bwd {fb:.4g} rays/s, fwd {res['fwd_rays_per_s']:.4g} rays/s")
    return res


def config_rows(lf, which, steps=3):
    """Secondary rows: configurations C1-C4 at their full sizes, each in its
    own context.  C1 (4k volume surfels, 64x64, k=16, primary only) and C2
    (200k surface surfels, 800x800, S=1) forward; C3 (300k surfels, 4 x
    800x800, S=1) the training step against a render of the perturbed
    scene; C4 (500k + 8 x 20k instanced surfels, 4 states at 1024x1024, S=4)
    forward and backward of every state with its own transforms and map.
    One warm-up, then `steps` timed repetitions; rays are traced rays."""
    import torch
    import scenegen
    dev = torch.device("cuda", 0)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    rows = {}
    for i in which:
        wl = scenegen.make_workload(i)
        sc = wl.scene
        tr = lf.Tracer(0)
        p = dict(mu=T(sc.mu), q=T(sc.q), scale=T(sc.scale), opacity=T(sc.opacity), albedo=T(sc.albedo),
                 roughness=T(sc.roughness), metallic=T(sc.metallic))
        tr.set_scene(**p, object_offset=list(sc.object_offset))
        sts = [(T(s_.env), T(s_.R) if sc.n_objects else None, T(s_.t) if sc.n_objects else None, s_.cameras)
               for s_ in wl.states]
        flags = lf.FLAG_NO_SECONDARY if wl.no_secondary else 0
        targets = None
        if i == 3:  # L1 target rendered from the perturbed scene and map
            ttr = lf.Tracer(0)
            ts_ = wl.target_scene
            ttr.set_scene(T(ts_.mu), T(ts_.q), T(ts_.scale), T(ts_.opacity), T(ts_.albedo), T(ts_.roughness),
                          T(ts_.metallic), list(ts_.object_offset))
            targets = [ttr.render(T(wl.target_envs[0]), None, None, cameras=sts[0][3], k=wl.k, spp=wl.spp,
                                  seed=wl.seed)["radiance"].clone()]
            ttr.sync()
            del ttr

        def run():
            for j, (env, R, t, cams) in enumerate(sts):
                out = tr.render(env, R, t, cameras=cams, k=wl.k, spp=wl.spp, seed=wl.seed + j, flags=flags)
                if i in (3, 4):
                    tgt = targets[j] if targets else torch.zeros_like(out["radiance"])
                    _, g = tr.l1_loss(out["radiance"], tgt)
                    tr.render_backward(env, R, t, cameras=cams, k=wl.k, spp=wl.spp, seed=wl.seed + j, flags=flags,
                                       d_radiance=g)

        run()
        tr.sync()
        tr.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = tr.stats()
        rays = st["rays_primary"] + st["rays_secondary"]
        rows[f"C{i}"] = {"workload": wl.name, "surfels": int(sc.n), "pass": "fwd+bwd" if i in (3, 4) else "fwd",
                         "rays_per_s": rays / dt, "ms_per_step": dt * 1e3 / steps,
                         "rays_per_step": rays / steps}
        log(f"C{i}: {rows[f'C{i}']['rays_per_s']:.4g} rays/s, {dt * 1e3 / steps:.1f} ms per step")
        tr.sync()
        del tr
        torch.cuda.empty_cache()
    return rows


def copy_bandwidth(torch):
    """Device-to-device copy of 1 GiB: bytes read + written over the median
    of 5 timed copies (HIP events on torch's stream)."""
    src = torch.empty(1 << 28, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    times = []
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    gbs = 2.0 * src.numel() * 4 / (float(np.median(times)) * 1e-3) / 1e9
    del src, dst
    return gbs


def estimator_bench(lf, tr, env, R, t, cam, wl, params, grads, out, target, spps, lr=1e-5):
    """The paper's two-ray estimator (Sec. 4.2: per path sample one
    environment next-event ray and one cosine/GGX continuation) with the
    replayed Owen-scrambled Sobol samples (Sec. 3.3) on the same scene and camera, at the spp of its training schedule (8, 16, 32): one
    warm-up and one timed training step each (refit, forward, L1, replayed
    backward, SGD)."""
    import torch
    res = {}
    for spp in spps:
        cfg = dict(cameras=[cam], k=wl.k, spp=spp, seed=wl.seed, flags=lf.FLAG_NEE | lf.FLAG_SOBOL)

        def step():
            tr.refit()
            tr.render(env, R, t, out=out, **cfg)
            loss, g = tr.l1_loss(out["radiance"], target)
            tr.render_backward(env, R, t, d_radiance=g, grads=grads, **cfg)
            with torch.no_grad():
                for k_, v in params.items():
                    v.sub_(lr * grads[k_])
                params["scale"].clamp_(min=1e-4)
                params["opacity"].clamp_(1e-4, 1.0)
                for k_ in ("albedo", "roughness", "metallic"):
                    params[k_].clamp_(0.0, 1.0)
            return loss

        step()
        tr.sync()
        tr.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with Marker(f"bench:two_ray_spp{spp}"):
            step()
            torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = tr.stats()
        res[str(spp)] = {"ms_per_step": dt * 1e3, "rays_per_s": (st["rays_primary"] + st["rays_secondary"]) / dt,
                         "secondary_rays_per_step": st["rays_secondary"]}
        log(f"two-ray spp {spp}: {dt * 1e3:.0f} ms/step, {res[str(spp)]['rays_per_s']:.4g} rays/s")
    return res


def inverse_rendering_bench(lf, tr, sc, wl, params, grads, args, n_states=3, batch=16384, lam_tv=1e-2,
                            lr_env=1.0, lr_mat=1e-3):
    """The staged inverse-rendering loop (Sec. 4.2 implementation details,
    Eq. training-objectives) as a throughput workload on the resident scene
    with its geometry fixed: three states, each with its own rigid object
    transforms, camera and 128x256 environment map (the trainable E_k);
    targets rendered once from the reference materials and maps.  Every
    iteration takes one state's image, draws 16,384 of its pixels, traces them
    with the two-ray estimator and the Sobol sampler, and applies L1 + lambda_E L_TV(E_k) through
    the replayed backward.  The paper's 15,000-iteration schedule is scaled
    to the iteration count: lighting only for the first 2/15, then lighting
    and base colour until 9/15, then all materials; spp 8, 16 from half way,
    32 from 4/5."""
    import torch
    import scenegen
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(4000)
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)  # noqa: E731
    res = args.res
    states = []
    for k in range(n_states):
        R_, t_ = scenegen.random_rigid(rng, sc.n_objects)
        cam_k = scenegen.sphere_camera(rng, res, res)
        o, d = tr.raygen(cam_k)
        states.append(dict(R=T(R_), t=T(t_), env_true=T(scenegen.lognormal_env(rng, 128, 256)), o=o, d=d))
    # targets: the whole image of each state from the reference materials and maps
    for stt in states:
        o_all, d_all = stt["o"], stt["d"]
        stt["target"] = tr.render(stt["env_true"], stt["R"], stt["t"], rays=(o_all, d_all), k=wl.k, spp=8,
                                  seed=7, flags=lf.FLAG_NEE | lf.FLAG_SOBOL)["radiance"].clone()
        stt["env"] = torch.full_like(stt["env_true"], float(stt["env_true"].mean()))  # trainable E_k
        stt["g_env"] = torch.empty_like(stt["env"])
    mats = ("albedo", "roughness", "metallic")
    ref_mats = {k_: params[k_].clone() for k_ in mats}
    main_g_env = grads["env"]
    with torch.no_grad():  # the materials start from a perturbed copy
        params["albedo"].copy_((ref_mats["albedo"] * 0.5 + 0.25).clamp(0, 1))
        params["roughness"].fill_(0.5)
        params["metallic"].fill_(0.1)
    n_it = args.ir_steps
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    per_bucket = {}
    tr.sync()
    tr.stats()
    tr.profile(True)
    tr.profile_read()
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    with Marker("bench:inverse_rendering"):
        for it in range(n_it):
            frac = it / n_it
            spp = 8 if frac < 0.5 else (16 if frac < 0.8 else 32)
            unlocked = () if frac < 2 / 15 else (("albedo",) if frac < 0.6 else mats)
            stt = states[it % n_states]
            t0 = time.perf_counter()
            pix = torch.randint(0, res * res, (batch,), device=dev, generator=gen).sort().values
            o_b, d_b = stt["o"][pix].contiguous(), stt["d"][pix].contiguous()
            cfg = dict(rays=(o_b, d_b), k=wl.k, spp=spp, seed=100 + it, flags=lf.FLAG_NEE | lf.FLAG_SOBOL)
            out = tr.render(stt["env"], stt["R"], stt["t"], **cfg)
            loss, g = tr.l1_loss(out["radiance"], stt["target"][pix].contiguous())
            grads["env"] = stt["g_env"]
            tr.render_backward(stt["env"], stt["R"], stt["t"], d_radiance=g, grads=grads, **cfg)
            tv, g_tv = tr.loss_tv(stt["env"])
            with torch.no_grad():
                stt["env"].sub_(lr_env * (grads["env"] + lam_tv * g_tv)).clamp_(min=0.0)
                for k_ in unlocked:
                    params[k_].sub_(lr_mat * grads[k_]).clamp_(0.0, 1.0)
            torch.cuda.synchronize()
            key = f"spp{spp}_" + ("lighting" if not unlocked else ("lighting+albedo" if len(unlocked) == 1 else "all"))
            b = per_bucket.setdefault(key, [0, 0.0])
            b[0] += 1
            b[1] += time.perf_counter() - t0
    dt = time.perf_counter() - t_all
    phases = tr.profile_read()
    tr.profile(False)
    st = tr.stats()
    with torch.no_grad():  # restore the reference materials for the legs that follow
        for k_ in mats:
            params[k_].copy_(ref_mats[k_])
    grads["env"] = main_g_env
    return {"iterations": n_it, "batch_pixels": batch, "states": n_states, "env": [128, 256],
            "ms_per_iteration": dt * 1e3 / n_it, "iterations_per_s": n_it / dt,
            "rays_per_s": (st["rays_primary"] + st["rays_secondary"]) / dt, "last_l1": float(loss),
            "last_tv": float(tv),
            "ms_per_iteration_by_stage": {k_: v[1] * 1e3 / v[0] for k_, v in per_bucket.items()},
            "phases_ms_per_iteration": {k_: v[0] / n_it for k_, v in phases.items() if v[1]}}


# algorithmic HBM bytes per element of each geometry objective: maps read once, gradient written once
GEO_BYTES = {"alpha": 8, "scale": 16, "depth": 16, "normal": 36, "depth_normal": 20}


def geometry_bench(lf, tr, env, R, t, cam, wl, params, grads, out, ref, args, s_max=0.05, lr=1e-5):
    """Ray-tracing-oriented geometry refinement (Sec. 3.2, Eq. geometry-objective
    with unit weights): refit, primary render (depth, normal, alpha), the
    objectives L_alpha, L_s, L_D, L_N, L_DN, the replayed backward through the
    depth, normal and alpha maps, and an SGD update of the geometry (position,
    rotation, scale, opacity).  Also times each objective alone over the
    1024x1024 maps with the library's phase timers (whole call: zeroing, the
    streaming pass and the final scalar; camera upload excluded)."""
    import torch
    gcfg = dict(cameras=[cam], k=wl.k, spp=1, seed=wl.seed, flags=lf.FLAG_NO_SECONDARY)
    geo = ("mu", "q", "scale", "opacity")

    def gstep():
        tr.refit()
        tr.render(env, R, t, out=out, **gcfg)
        lD, gD = tr.loss_depth(out["depth"], ref["depth"], ref["conf"], eps=1e-6)
        lN, gN = tr.loss_normal(out["normal"], ref["normal"])
        lDN, gDN = tr.loss_depth_normal(cam, out["depth"], ref["normal"])
        lA, gA = tr.loss_alpha(out["alpha"])
        lS, gS = tr.loss_scale(params["scale"], s_max)
        gD.add_(gDN)
        tr.render_backward(env, R, t, d_depth=gD, d_normal=gN, d_alpha=gA, grads=grads, **gcfg)
        with torch.no_grad():
            grads["scale"].add_(gS)
            for k_ in geo:
                params[k_].sub_(lr * grads[k_])
            params["scale"].clamp_(min=1e-4)
            params["opacity"].clamp_(1e-4, 1.0)
        return lD + lN + lDN + lA + lS

    for _ in range(args.warmup):
        gstep()
    tr.sync()
    tr.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with Marker("bench:geometry"):
        for _ in range(args.geo_steps):
            loss = gstep()
        torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = tr.stats()
    res = {"ms_per_step": dt * 1e3 / args.geo_steps, "rays_per_s": (st["rays_primary"] + st["rays_secondary"]) / dt,
           "loss": float(loss), "objectives": {}}

    nr = cam.w * cam.h
    calls = {
        "alpha": (nr, lambda: tr.loss_alpha(out["alpha"])),
        "scale": (params["scale"].shape[0], lambda: tr.loss_scale(params["scale"], s_max)),
        "depth": (nr, lambda: tr.loss_depth(out["depth"], ref["depth"], ref["conf"], eps=1e-6)),
        "normal": (nr, lambda: tr.loss_normal(out["normal"], ref["normal"])),
        "depth_normal": (nr, lambda: tr.loss_depth_normal(cam, out["depth"], ref["normal"])),
    }
    reps = 50
    for name, (n, fn) in calls.items():
        fn()
        tr.sync()
        tr.profile(True)
        tr.profile_read()
        # a render ahead of the calls keeps the GPU busy while the host queues them, so the
        # phase timers see device time rather than host submission gaps
        tr.render(env, R, t, out=out, **gcfg)
        for _ in range(reps):
            fn()
        tr.sync()
        ms = tr.profile_read()["loss"][0] / reps
        tr.profile(False)
        gbs = GEO_BYTES[name] * n / (ms * 1e-3) / 1e9
        res["objectives"][name] = {"elements": int(n), "call_ms": ms, "bytes": GEO_BYTES[name] * n,
                                   "call_GB/s": gbs, "call_frac": gbs / HBM_PEAK_GBS}
    return res


def serve_bench(tr, sc, args, loads, policies=(0,)):
    """Relight latency (arrival to result) of a Poisson request stream on the
    resident scene: the continuous-batching server against the plain tracer
    serving the same stream FIFO, one request at a time.  Each request draws a
    rigid transform per object, a 256x512 lognormal env map, a resolution in
    {256, 512, 1024}^2 and S in {1, 4}; the rate is a fraction of the plain
    tracer's capacity measured on that mix."""
    import torch

    import paper_2608_29269_amd as lf
    import scenegen
    dev = torch.device("cuda", 0)
    M = sc.n_objects
    res_set, spp_set = (256, 512, 1024), (1, 4)
    # plain capacity on the request mix (each combination equally likely)
    cal = scenegen.request_stream(M, 6, 1.0, seed=99)
    svc = []
    for j, (res, spp) in enumerate([(r, s_) for r in res_set for s_ in spp_set]):
        q = cal[j]
        cam = scenegen.sphere_camera(np.random.default_rng(j), res, res)
        env, R, t = (torch.as_tensor(x, device=dev) for x in (q.env, q.R, q.t))
        times = []
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tr.render(env, R, t, cameras=[cam], k=32, spp=spp, seed=q.seed)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        svc.append(float(np.median(times[1:])))
    mean_svc = float(np.mean(svc))
    capacity = 1.0 / mean_svc
    log(f"serving: plain capacity {capacity:.2f} requests/s (mean service {mean_svc * 1e3:.1f} ms)")
    runs = []
    for load in loads:
        rate = load * capacity
        reqs = scenegen.request_stream(M, args.serve_requests, rate, seed=5, resolutions=res_set, spps=spp_set)
        dv = []
        for q in reqs:
            n = q.camera.w * q.camera.h
            dv.append(dict(env=torch.as_tensor(q.env, device=dev), R=torch.as_tensor(q.R, device=dev),
                           t=torch.as_tensor(q.t, device=dev),
                           out=dict(radiance=torch.empty((n, 3), device=dev), depth=torch.empty(n, device=dev),
                                    normal=torch.empty((n, 3), device=dev), alpha=torch.empty(n, device=dev))))
        torch.cuda.synchronize()
        # plain tracer, FIFO, one request at a time
        tr.stats()
        lat = []
        t_start = time.perf_counter()
        with Marker(f"bench:serve_plain_load{load}"):
            for q, d in zip(reqs, dv):
                now = time.perf_counter() - t_start
                if now < q.arrival_s:
                    time.sleep(q.arrival_s - now)
                tr.render(d["env"], d["R"], d["t"], cameras=[q.camera], k=32, spp=q.spp, seed=q.seed, out=d["out"])
                torch.cuda.synchronize()
                lat.append(time.perf_counter() - t_start - q.arrival_s)
        span = time.perf_counter() - t_start - reqs[0].arrival_s
        ps = tr.stats()
        plain = {"p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": float(np.mean(lat)) * 1e3,
                 "rays_per_s": (ps["rays_primary"] + ps["rays_secondary"]) / span}
        log(f"serving load {load}: plain p50 {plain['p50_ms']:.0f} ms p99 {plain['p99_ms']:.0f} ms")
        plain["by_class_p50_ms"] = by_class(reqs, lat)
        # continuous-batching server, per pass-filling policy
        for policy in policies:
            srv = lf.Server(tr, max_slots=16, hbm_budget_bytes=16 << 30, tile_rays=65536,
                            batch_rays=args.serve_batch, max_spp=4, policy=policy,
                            max_in_flight=args.serve_in_flight)
            tickets = []
            t_start = time.perf_counter()
            with Marker(f"bench:serve_{POLICY_NAMES[policy]}_load{load}"):
                for q, d in zip(reqs, dv):
                    now = time.perf_counter() - t_start
                    if now < q.arrival_s:
                        time.sleep(q.arrival_s - now)
                    tickets.append(srv.submit(d["env"], q.camera, R=d["R"], t=d["t"], spp=q.spp, seed=q.seed,
                                              out=d["out"]))
                for tk in tickets:
                    srv.wait(tk)
            slat = [srv.latency_ms(tk) / 1e3 for tk in tickets]
            st = srv.stats()
            srv.close()
            served = {"policy": POLICY_NAMES[policy], "p50_ms": pct(slat, 50), "p99_ms": pct(slat, 99),
                      "mean_ms": float(np.mean(slat)) * 1e3, "rays_per_s": st["rays_per_s"],
                      "passes": st["iterations"], "by_class_p50_ms": by_class(reqs, slat)}
            log(f"serving load {load}: server ({POLICY_NAMES[policy]}) p50 {served['p50_ms']:.0f} ms "
                f"p99 {served['p99_ms']:.0f} ms")
            runs.append({"load": load, "rate_req_per_s": rate, "requests": len(reqs), "server": served,
                         "plain": plain,
                         "p99_ratio_plain_over_server": plain["p99_ms"] / served["p99_ms"],
                         "p50_ratio_plain_over_server": plain["p50_ms"] / served["p50_ms"]})
    return {"capacity_req_per_s": capacity, "mean_service_ms": mean_svc * 1e3,
            "service_ms_alone": {f"{r}x{r} S={s_}": v * 1e3
                                 for (r, s_), v in zip([(r, s_) for r in res_set for s_ in spp_set], svc)},
            "mix": "resolution {256,512,1024}^2 x S {1,4}, 256x512 env, 8 rigid transforms per request",
            "server_config": {"max_slots": 16, "hbm_budget_gib": 16, "tile_rays": 65536,
                              "batch_rays": args.serve_batch, "max_in_flight": args.serve_in_flight},
            "runs": runs}


POLICY_NAMES = {0: "shortest_first", 1: "oldest_first", 2: "round_robin"}


def by_class(reqs, lat):
    """p50 latency (ms) per (resolution, S) class."""
    out = {}
    for key in sorted({(q.camera.w, q.spp) for q in reqs}):
        v = [l for q, l in zip(reqs, lat) if (q.camera.w, q.spp) == key]
        out[f"{key[0]} S={key[1]}"] = pct(v, 50)
    return out


def pct(v, q):
    """Nearest-rank percentile in milliseconds of a list of seconds."""
    a = np.sort(np.asarray(v, np.float64))
    i = min(max(int(np.ceil(q / 100.0 * len(a))), 1), len(a))
    return float(a[i - 1] * 1e3)


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2608_29269_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


# Kernels that each own one phase timer (one launch per call) and what they process.
KERNEL_OF_PHASE = {"trace1": "k_trace1p<32, false>", "trace2": "k_trace2<32, false>",
                   "composite1": "k_composite1<32, false>", "composite2": "k_composite2<32, false>",
                   "adj_hits": "k_adj_hits<32>"}


def kernel_bytes(counts, stats, steps):
    """Algorithmic HBM bytes per launch of each tracing kernel: per-ray
    figures times the rays one launch processes.  h_touch (supports crossed
    before the k-th hit) and h_comp (composited hits) are counted by the
    oracle on the CPU sample of the same workload."""
    import oracle
    c = counts
    sec = max(c[:, oracle.C_SEC_RAYS].sum(), 1.0)
    touch_p = c[:, oracle.C_TOUCH_PRI].mean()
    comp_p = c[:, oracle.C_COMP_PRI].mean()
    touch_s = c[:, oracle.C_TOUCH_SEC].sum() / sec
    comp_s = c[:, oracle.C_COMP_SEC].sum() / sec
    rays_pri = stats["rays_primary"] / max(steps, 1)
    rays_sec = stats["rays_secondary"] / max(steps, 1)
    per_ray = {
        # traversal: 40 B of geometry per crossed support (primary rays come from the camera on the device)
        "trace1": 40 * touch_p,
        # compositing: 20 B of material per composited hit, 60 B surface record and 20 B depth/normal/alpha out
        "composite1": 20 * comp_p + 60 + 20,
        # 44 B queued ray in (origin, direction, id, sample, throughput), geometry per crossed support
        "trace2": 44 + 40 * touch_s,
        "composite2": 20 * comp_s + 60,
        # 44 B of adjoint seeds in, material per composited hit, 120 B gradient read-modify-write per hit
        "adj_hits": 44 + 20 * comp_p + 120 * comp_p,
    }
    rays = {"trace1": rays_pri, "composite1": rays_pri, "trace2": rays_sec, "composite2": rays_sec,
            "adj_hits": rays_pri}
    return {k: per_ray[k] * rays[k] for k in per_ray}, per_ray, rays


def roofline(phases, counts, stats, args, nr, copy_gbs=None):
    """Roofline of the dominant kernel: algorithmic bytes per launch over its
    average launch duration, measured with HIP events on the library's stream
    (each of these phases holds exactly one launch per call).  Also against
    the measured device-to-device copy bandwidth, and with the counter
    evidence (HBM traffic, L2 hit rate, VALU issue) taken at the current
    kernel sources."""
    cand = {k: v for k, v in phases.items() if k in KERNEL_OF_PHASE and v[1]}
    name, (ms, n) = max(cand.items(), key=lambda kv: kv[1][0])
    avg_ms = ms / n
    out = {"bound": "hbm", "kernel": KERNEL_OF_PHASE[name], "phase": name, "avg_ms": avg_ms, "achieved": None,
           "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None, "traffic": None, "l2_hit_rate": None,
           "copy_GBs": copy_gbs}
    if counts is None:
        return out
    per_launch, per_ray, rays = kernel_bytes(counts, stats, args.steps)
    if name not in per_launch:
        return out
    achieved = per_launch[name] / (avg_ms * 1e-3) / 1e9
    out.update(achieved=float(achieved), frac=float(achieved / HBM_PEAK_GBS),
               alg_bytes_per_launch=float(per_launch[name]), alg_bytes_per_ray=float(per_ray[name]),
               rays_per_launch=float(rays[name]))
    if copy_gbs:
        out["frac_of_copy"] = float(achieved / copy_gbs)
    lf_ = os.path.join(ROOT, "profiles", "l2.json")
    if os.path.exists(lf_):
        try:
            lj = json.load(open(lf_))
            e = lj.get("kernels", {}).get(out["kernel"])
            if e and lj.get("source_digest") == source_digest():
                out["l2_hit_rate"] = e["hit_rate"]
        except (OSError, ValueError, KeyError):
            out["l2_hit_rate"] = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        try:
            tj = json.load(open(tf))
            e = tj.get("kernels", {}).get(out["kernel"])
            if e and tj.get("source_digest") == source_digest():
                out["traffic"] = e.get("hbm_bytes_per_launch")
        except (OSError, ValueError):
            out["traffic"] = None
    # the kernel is latency- and ALU-bound: its VALU issue fraction from the SQ counters (same digest rule)
    sf = os.path.join(ROOT, "profiles", "sq.json")
    if os.path.exists(sf):
        try:
            sj = json.load(open(sf))
            e = sj.get("kernels", {}).get(out["kernel"])
            if e and sj.get("source_digest") == source_digest():
                out["valu_issue_per_wave"] = e["valu_issue_per_wave"]
                out["valu_issue_per_simd"] = e["valu_issue_per_wave"] * e["waves_per_simd"]
        except (OSError, ValueError, KeyError):
            pass
    return out


if __name__ == "__main__":
    main()
