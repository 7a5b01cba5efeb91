"""Pins of the oracle's two-ray estimator (Sec. 3.3 "differentiable one-bounce
path tracing" and Eq. path-estimator; Sec. 4.2: per path one environment
next-event sample, one cosine/GGX continuation, at most one secondary hit and
two environment samples there; power-heuristic MIS between the two primary
techniques): exact reduction to the one-ray form when environment sampling
is off, unbiasedness against quadrature (unshadowed and under a grey roof),
the slot layout of the outputs, and central finite differences of its
replayed adjoint.  CPU only."""
import numpy as np
import pytest
from scipy import integrate

import oracle
import scenegen
from tests.helpers import make_scene, no_transforms

P = oracle.Params
GROUPS = ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic", "env")


def _render_same_ray(scene, env, n, o, d, **kw):
    R, t = no_transforms(scene)
    sa = oracle.SceneArrays(scene, R, t, env)
    p = P(**{**dict(k=8, spp=1, seed=123), **kw})
    oo = np.tile(np.asarray(o, dtype=np.float64), (n, 1))
    dd = np.tile(np.asarray(d, dtype=np.float64) / np.linalg.norm(d), (n, 1))
    return oracle.render(sa, oo, dd, np.arange(n), p, lists=True)


@pytest.fixture(scope="module")
def small_env():
    rng = np.random.default_rng(9)
    return scenegen.lognormal_env(rng, 8, 16, lobe_gain=50.0, lobe_width=0.3)


def _workload(which=2, scale=0.02, res=16, spp=2, flags=0):
    wl = scenegen.make_workload(which, scale=scale, resolution=res)
    st = wl.states[0]
    env = scenegen.lognormal_env(np.random.default_rng(5), 16, 32)
    o, d, ids = oracle.raygen(st.cameras[0])
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, env)
    return wl, sa, o, d, ids, P(k=wl.k, spp=spp, seed=31, flags=flags)


def test_without_environment_sampling_it_is_the_one_ray_form():
    """With environment sampling off the next-event slot is dead and the
    continuation carries K = 1/p_b and full weight, which is the one-ray form
    with c_env = 0 drawing the same uniforms: same radiance, and the odd slots
    hold the one-ray form's secondary hit lists."""
    wl, sa, o, d, ids, p1 = _workload(flags=oracle.BSDF_ONLY)
    p2 = P(k=p1.k, spp=p1.spp, seed=p1.seed, flags=oracle.BSDF_ONLY | oracle.NEE)
    a = oracle.render(sa, o, d, ids, p1)
    b = oracle.render(sa, o, d, ids, p2)
    np.testing.assert_allclose(b["radiance"], a["radiance"], rtol=1e-12, atol=1e-15)
    assert b["sec_hit_idx"].shape[1] == 2 * p1.spp
    assert np.all(b["sec_hit_idx"][:, 0::2] == -1)
    assert np.array_equal(b["sec_hit_idx"][:, 1::2], a["sec_hit_idx"])
    assert np.all(b["sec_alpha"][:, 0::2] == -1.0)
    assert a["counts"][:, oracle.C_SEC_RAYS].sum() == b["counts"][:, oracle.C_SEC_RAYS].sum() > 0


def test_next_event_slots_trace_one_ray_per_live_sample():
    wl, sa, o, d, ids, p = _workload(flags=oracle.NEE)
    out = oracle.render(sa, o, d, ids, p)
    hit = out["hit_idx"][:, 0] >= 0
    traced = out["sec_alpha"] >= 0  # -1 marks a slot without a secondary ray
    # both kinds of slot are traced on rays with a surface, none on misses
    assert traced[hit][:, 0::2].mean() > 0.3 and traced[hit][:, 1::2].mean() > 0.3
    assert not traced[~hit].any()
    assert out["counts"][:, oracle.C_SEC_RAYS].sum() == traced.sum()


@pytest.mark.parametrize("m,r,flags", [(0.0, 0.5, oracle.DIFFUSE_ONLY), (1.0, 0.4, 0), (0.4, 0.25, 0)])
def test_two_ray_estimator_unbiased_against_quadrature(m, r, flags, small_env):
    """Unshadowed (no secondary ray): next-event + continuation with
    multi-sample power MIS has the mean of int f cos E dw."""
    a = np.array([0.9, 0.6, 0.3])
    sc = make_scene([[0, 0, 0]], scale=[[10, 10]], opacity=[1.0], albedo=[a], metallic=[m], roughness=[r])
    d = np.array([0.3, -0.2, -1.0])
    d /= np.linalg.norm(d)
    N = 40000
    out = _render_same_ray(sc, small_env, N, -3 * d, d, spp=1, flags=flags | oracle.NO_SECONDARY | oracle.NEE)
    a32, m32, r32 = a.astype(np.float32).astype(np.float64), float(np.float32(m)), float(np.float32(r))
    n = np.array([0, 0, 1.0])
    wo = -d
    H, W = small_env.shape[:2]
    sub = 12
    acc = np.zeros(3)
    for i in range(H * sub):
        th = (i + 0.5) * np.pi / (H * sub)
        for j in range(W * sub):
            ph = (j + 0.5) * 2 * np.pi / (W * sub)
            w = np.array([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)])
            if w[2] <= 0:
                continue
            acc += oracle.brdf(n, w, wo, a32, m32, r32, flags) * w[2] * oracle.env_lookup(small_env, w) * np.sin(th)
    acc *= (np.pi / (H * sub)) * (2 * np.pi / (W * sub))
    want = 0.99 * acc + 0.01 * oracle.env_lookup(small_env, d)
    L = out["radiance"]
    se = L.std(0) / np.sqrt(N)
    assert np.all(np.abs(L.mean(0) - want) < 4 * se + 2e-3 * np.abs(want)), (L.mean(0), want, se)


def test_grey_roof_matches_quadrature_with_next_event_rays():
    """White Lambert floor under a roof of albedo 0.5 in a constant
    environment: L = c (1 - 0.5 E_cos[A2]).  The next-event rays see the roof
    only as transmittance; counting the roof's radiance on them as well
    would raise the mean."""
    s_roof, h_roof, off = 10.0, 0.5, 1e-3
    sc = make_scene([[0, 0, 0], [0, 0, h_roof]], scale=[[10, 10], [s_roof, s_roof]], opacity=[1, 1],
                    albedo=[[1, 1, 1], [0.5, 0.5, 0.5]], metallic=[0, 0])
    N = 20000
    out = _render_same_ray(sc, scenegen.constant_env(1.0, 8, 16), N, [0, 0, 0.25], [0, 0, -1], spp=1,
                           flags=oracle.DIFFUSE_ONLY | oracle.NEE)
    h = h_roof - off

    def a2(th):
        rho2 = (h * np.tan(th) / s_roof) ** 2
        if rho2 > min(9.0, 2 * np.log(255.0)):
            return 0.0
        return min(0.99, np.exp(-0.5 * rho2))

    EA2, _ = integrate.quad(lambda th: a2(th) * 2 * np.cos(th) * np.sin(th), 0, np.pi / 2, limit=200)
    want = 0.99 * (1 - 0.5 * EA2) + 0.01
    L = out["radiance"][:, 0]
    assert abs(L.mean() - want) < 4 * L.std() / np.sqrt(N) + 1e-12, (L.mean(), want)
    assert np.mean(out["sec_alpha"][:, 0] > 0.9) > 0.3  # next-event rays do meet the roof


@pytest.mark.parametrize("which,scale,spp,flags", [
    (2, 0.02, 2, oracle.NEE),                          # surface-like, one bounce, two rays per sample
    (4, 0.005, 1, oracle.NEE | oracle.NO_SECONDARY),   # instanced, unshadowed two-technique form
])
def test_two_ray_adjoint_matches_central_fd(which, scale, spp, flags):
    wl = scenegen.make_workload(which, scale=scale, resolution=16)
    st = wl.states[0]
    o, d, ids = oracle.raygen(st.cameras[0])
    env = scenegen.lognormal_env(np.random.default_rng(77), 16, 32)
    p = P(k=wl.k, spp=spp, seed=77, flags=flags)
    rng = np.random.default_rng(which)
    n = len(ids)
    up = {"radiance": rng.standard_normal((n, 3)), "alpha": rng.standard_normal(n)}
    sa0 = oracle.SceneArrays(wl.scene, st.R, st.t, env)
    g = oracle.backward(sa0, o, d, ids, p, g_radiance=up["radiance"], g_alpha=up["alpha"])
    sc = wl.scene
    th0 = {"mu": sc.mu, "q": sc.q, "scale": sc.scale, "opacity": sc.opacity, "albedo": sc.albedo,
           "roughness": sc.roughness, "metallic": sc.metallic, "env": env}
    th0 = {k: np.asarray(v, np.float64) for k, v in th0.items()}
    for grp in GROUPS:
        v = rng.standard_normal(th0[grp].shape)
        h = 1e-6 * max(1.0, float(np.abs(th0[grp]).max()))
        vals = {}
        for sgn in (+2, +1, -1, -2):
            ov = dict(th0)
            ov[grp] = th0[grp] + sgn * h * v
            sa = oracle.SceneArrays(wl.scene, st.R, st.t, env, overrides=ov)
            out = oracle.frozen_eval(sa0, sa, o, d, ids, p)
            vals[sgn] = sum(float((out[k] * up[k]).sum()) for k in up)
        fd = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
        ad = float((g[grp] * v).sum())
        assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3 * abs(vals[1])), (grp, fd, ad)
