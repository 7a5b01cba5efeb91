"""Parity at the full workload sizes (200k to 1M surfels, 800^2 to 1024^2
images, S up to 4), in the launch configuration the benchmark times: whole
images in one call.  The oracle computes sampled pixels one by one; forward
outputs are compared on those pixels, and gradients are compared with an
upstream gradient that is non-zero only on them (every other ray then adds
exactly nothing).  Requires an MI355X."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_common import grad_check, ambiguous, dev, rel_close, run_oracle, state_args, upload_scene

pytestmark = pytest.mark.gpu

RTOL = 1e-4
GTOL = 1e-3
N_SAMPLE = 256


@pytest.fixture(scope="module")
def tracer():
    import paper_2608_29269_amd as lf
    return lf.Tracer()


def _sampled_rays(cams, m, seed):
    """m random ray ids over the cameras of one call, with their rays."""
    rng = np.random.default_rng(seed)
    sizes = [c.w * c.h for c in cams]
    off = np.concatenate([[0], np.cumsum(sizes)])
    ids = np.sort(rng.choice(off[-1], m, replace=False))
    o, d = [], []
    for i in ids:
        c = int(np.searchsorted(off, i, side="right") - 1)
        oo, dd, _ = oracle.raygen(cams[c], np.array([i - off[c]]))
        o.append(oo[0])
        d.append(dd[0])
    return ids, np.array(o, np.float32), np.array(d, np.float32)


@pytest.mark.parametrize("which,state", [(2, 0), (3, 0), (4, 0), (4, 3), (5, 0)])
def test_full_size_forward_on_sampled_pixels(tracer, which, state):
    wl = scenegen.make_workload(which)
    st = wl.states[state]
    print(f"workload {which} state {state}: {wl.scene.n} surfels, {len(st.cameras)} x "
          f"{st.cameras[0].w}x{st.cameras[0].h}, S={wl.spp}", flush=True)
    upload_scene(tracer, wl.scene)
    out = tracer.render(**state_args(tracer, wl.scene, st), cameras=st.cameras, k=wl.k, spp=wl.spp,
                        seed=wl.seed + state, hit_idx=True, sec_hit_idx=True)
    tracer.sync()
    ids, o, d = _sampled_rays(st.cameras, N_SAMPLE, which * 10 + state)
    ref = run_oracle(wl.scene, st, o, d, ids, wl.k, wl.spp, wl.seed + state, 0)
    amb = ambiguous(ref["margins"])
    ok = ~amb
    print(f"ambiguous {int(amb.sum())} of {N_SAMPLE}", flush=True)
    assert amb.sum() <= 2, amb.sum()
    # primary and per-slot secondary hit lists of the sampled rays, as the benchmark launches them
    np.testing.assert_array_equal(out["hit_idx"].cpu().numpy()[ids][ok], ref["hit_idx"][ok])
    np.testing.assert_array_equal(out["sec_hit_idx"].cpu().numpy()[ids][ok], ref["sec_hit_idx"][ok])
    for key in ("radiance", "depth", "normal", "alpha"):
        g = out[key].cpu().numpy()[ids]
        assert rel_close(g[ok], ref[key][ok], RTOL) < RTOL, key


def _grad_check(g_gpu, g_ref, name):
    grad_check(g_gpu, g_ref, name)


@pytest.mark.parametrize("which,det", [(3, False), (5, False), (5, True)])
def test_full_size_gradients_from_sampled_pixels(tracer, which, det):
    """The training-step configuration (300k surfels, 4 x 800^2, S=1) and the
    benchmark configuration (1M surfels, 1024^2, S=4), the latter also with
    order-fixed gradient sums (LF_FLAG_DETERMINISTIC)."""
    import paper_2608_29269_amd as lf
    flags = lf.FLAG_DETERMINISTIC if det else 0
    wl = scenegen.make_workload(which)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cams = st.cameras
    n = sum(c.w * c.h for c in cams)
    ids, o, d = _sampled_rays(cams, N_SAMPLE, 100 + which)
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    p = oracle.Params(k=wl.k, spp=wl.spp, seed=wl.seed)
    fwd = oracle.render(sa, o, d, ids, p, lists=False)
    amb = ambiguous(fwd["margins"])
    rng = np.random.default_rng(which)
    up = dict(radiance=rng.standard_normal((N_SAMPLE, 3)), depth=rng.standard_normal(N_SAMPLE),
              normal=rng.standard_normal((N_SAMPLE, 3)), alpha=rng.standard_normal(N_SAMPLE))
    full = {}
    for k_, v in up.items():
        v[amb] = 0.0
        up[k_] = v.astype(np.float32)
        f = np.zeros((n,) + v.shape[1:], np.float32)
        f[ids] = up[k_]
        full[k_] = dev(f)
    g_ref = oracle.backward(sa, o, d, ids, p, g_radiance=up["radiance"], g_depth=up["depth"],
                            g_normal=up["normal"], g_alpha=up["alpha"])
    g = tracer.render_backward(**state_args(tracer, wl.scene, st), cameras=cams, k=wl.k, spp=wl.spp,
                               seed=wl.seed, flags=flags, d_radiance=full["radiance"], d_depth=full["depth"],
                               d_normal=full["normal"], d_alpha=full["alpha"])
    tracer.sync()
    for name in ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic", "env"):
        _grad_check(g[name].cpu().numpy(), g_ref[name], name)


def test_full_size_two_ray_sobol_step_on_sampled_pixels(tracer):
    """The benchmark's two-ray leg at its first spp: 1M surfels, 1024^2,
    next-event + continuation per sample with Owen-scrambled Sobol samples
    (LF_FLAG_NEE | LF_FLAG_SOBOL), spp 8 (16 secondary slots per ray):
    forward outputs and gradients from an upstream on sampled pixels."""
    wl = scenegen.make_workload(5)
    st = wl.states[0]
    cams = st.cameras
    spp, flags = 8, oracle.NEE | oracle.SOBOL
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    out = tracer.render(**args, cameras=cams, k=wl.k, spp=spp, seed=wl.seed, flags=flags)
    tracer.sync()
    ids, o, d = _sampled_rays(cams, N_SAMPLE, 7)
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    p = oracle.Params(k=wl.k, spp=spp, seed=wl.seed, flags=flags)
    ref = oracle.render(sa, o, d, ids, p, lists=False)
    amb = ambiguous(ref["margins"])
    ok = ~amb
    print(f"ambiguous {int(amb.sum())} of {N_SAMPLE}", flush=True)
    assert amb.sum() <= 2, amb.sum()
    for key in ("radiance", "depth", "normal", "alpha"):
        g = out[key].cpu().numpy()[ids]
        assert rel_close(g[ok], ref[key][ok], RTOL) < RTOL, key
    n = cams[0].w * cams[0].h
    rng = np.random.default_rng(8)
    up = rng.standard_normal((N_SAMPLE, 3))
    up[amb] = 0.0
    up = up.astype(np.float32)
    full = np.zeros((n, 3), np.float32)
    full[ids] = up
    g_ref = oracle.backward(sa, o, d, ids, p, g_radiance=up)
    g = tracer.render_backward(**args, cameras=cams, k=wl.k, spp=spp, seed=wl.seed, flags=flags,
                               d_radiance=dev(full))
    tracer.sync()
    for name in ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic", "env"):
        _grad_check(g[name].cpu().numpy(), g_ref[name], name)
