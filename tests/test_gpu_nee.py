"""GPU parity of the two-ray estimator (LF_FLAG_NEE: per path sample one
environment next-event ray and one cosine/GGX continuation with
power-heuristic MIS; Sec. 3.3 Eq. path-estimator, Sec. 4.2) against the FP64
oracle, forward and replayed backward, through the C ABI.  Requires an
MI355X."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_common import grad_check, ambiguous, dev, rel_close, run_oracle, state_args, upload_scene

pytestmark = pytest.mark.gpu

RTOL = 1e-4
NEE = oracle.NEE


@pytest.fixture(scope="module")
def tracer():
    import paper_2608_29269_amd as lf
    return lf.Tracer()


@pytest.fixture(scope="module")
def c2_small():
    return scenegen.make_workload(2, scale=0.1, resolution=96)  # 20k surfels, 96x96


def _check(out, ref, amb, pix=None):
    g = {k: v.cpu().numpy() for k, v in out.items()}
    if pix is not None:
        g = {k: v[pix] for k, v in g.items()}
    ok = ~amb
    assert ok.mean() >= 0.99, f"ambiguous fraction {amb.mean():.4f}"
    np.testing.assert_array_equal(g["hit_idx"][ok], ref["hit_idx"][ok])
    np.testing.assert_array_equal(g["sec_hit_idx"][ok], ref["sec_hit_idx"][ok])
    for key in ("radiance", "depth", "normal", "alpha"):
        e = rel_close(g[key][ok], ref[key][ok], RTOL)
        assert e < RTOL, (key, e)


@pytest.mark.parametrize("spp", [1, 3])
def test_c2_two_ray_parity(tracer, c2_small, spp):
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cam = st.cameras[0]
    out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=32, spp=spp, seed=wl.seed, flags=NEE,
                        hit_idx=True, sec_hit_idx=True)
    assert tuple(out["sec_hit_idx"].shape) == (cam.w * cam.h, 2 * spp, 32)
    pix = np.arange(0, cam.w * cam.h, 3)
    o, d, ids = oracle.raygen(cam, pix)
    ref = run_oracle(wl.scene, st, o, d, ids, 32, spp, wl.seed, NEE)
    _check(out, ref, ambiguous(ref["margins"]), pix)
    traced = ref["sec_alpha"] >= 0
    assert traced[:, 0::2].mean() > 0.2 and traced[:, 1::2].mean() > 0.2  # both kinds of slot are traced


def test_two_ray_without_env_sampling_is_the_one_ray_form(tracer, c2_small):
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    kw = dict(cameras=st.cameras[:1], k=32, spp=2, seed=5, hit_idx=True, sec_hit_idx=True)
    a = tracer.render(**args, flags=oracle.BSDF_ONLY, **kw)
    b = tracer.render(**args, flags=oracle.BSDF_ONLY | NEE, **kw)
    ra, rb = a["radiance"].cpu().numpy(), b["radiance"].cpu().numpy()
    assert np.abs(ra - rb).max() <= 1e-6 * max(np.abs(ra).max(), 1e-30)
    sa, sb = a["sec_hit_idx"].cpu().numpy(), b["sec_hit_idx"].cpu().numpy()
    assert np.all(sb[:, 0::2] == -1) and np.array_equal(sb[:, 1::2], sa)


def test_two_ray_unshadowed_and_instanced_parity(tracer):
    wl = scenegen.make_workload(4, scale=0.01, resolution=48)
    st = wl.states[1]
    upload_scene(tracer, wl.scene)
    cam = st.cameras[0]
    for flags in (NEE, NEE | oracle.NO_SECONDARY):
        out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=wl.k, spp=2, seed=4, flags=flags,
                            hit_idx=True, sec_hit_idx=True)
        o, d, ids = oracle.raygen(cam)
        ref = run_oracle(wl.scene, st, o, d, ids, wl.k, 2, 4, flags)
        _check(out, ref, ambiguous(ref["margins"], include_secondary=not flags & oracle.NO_SECONDARY))


@pytest.mark.parametrize("which,scale,res,spp,flags", [
    (3, 0.02, 40, 2, NEE),                          # surface-like training step, two rays per sample
    (4, 0.01, 32, 1, NEE),                          # instanced objects
    (1, 1.0, 32, 2, NEE | oracle.NO_SECONDARY),     # unshadowed two-technique form
])
def test_two_ray_adjoint_matches_oracle(tracer, which, scale, res, spp, flags):
    wl = scenegen.make_workload(which, scale=scale, resolution=res)
    st = wl.states[0]
    env = scenegen.lognormal_env(np.random.default_rng(5), 32, 64)
    st = scenegen.State(R=st.R, t=st.t, env=env, cameras=st.cameras)
    cam = st.cameras[0]
    o, d, ids = oracle.raygen(cam)
    n = len(ids)
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    p = oracle.Params(k=wl.k, spp=spp, seed=wl.seed, flags=flags)
    fwd = oracle.render(sa, o, d, ids, p, lists=False)
    amb = ambiguous(fwd["margins"])
    rng = np.random.default_rng(which)
    up = dict(radiance=rng.standard_normal((n, 3)), depth=rng.standard_normal(n), normal=rng.standard_normal((n, 3)),
              alpha=rng.standard_normal(n))
    for k in up:
        up[k][amb] = 0.0
        up[k] = up[k].astype(np.float32)
    g_ref = oracle.backward(sa, o, d, ids, p, g_radiance=up["radiance"], g_depth=up["depth"],
                            g_normal=up["normal"], g_alpha=up["alpha"])
    upload_scene(tracer, wl.scene)
    g = tracer.render_backward(**state_args(tracer, wl.scene, st), cameras=[cam], k=wl.k, spp=spp, seed=wl.seed,
                               flags=flags, d_radiance=dev(up["radiance"]), d_depth=dev(up["depth"]),
                               d_normal=dev(up["normal"]), d_alpha=dev(up["alpha"]))
    tracer.sync()
    for name in ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic", "env"):
        grad_check(g[name].cpu().numpy(), g_ref[name], name, nonzero=True)


def test_server_rejects_the_two_ray_form(tracer, c2_small):
    import paper_2608_29269_amd as lf
    upload_scene(tracer, c2_small.scene)
    with pytest.raises(lf.LFError):
        lf.Server(tracer, flags=NEE)
