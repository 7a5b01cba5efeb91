"""Pins of the oracle's sampler, BRDF, environment sampling and one-bounce
estimator (Sec. 3.3, Eq. rendering-equation, Eq. path-estimator) against
published test vectors, closed forms, quadrature and unbiasedness.  CPU only."""
import json
import os

import numpy as np
import pytest
from scipy import integrate, stats

import oracle
import scenegen
from tests.helpers import make_scene, no_transforms

P = oracle.Params
GOLD = os.path.join(os.path.dirname(__file__), "golden")


# --- sampler ---------------------------------------------------------------------------

def test_splitmix64_published_vector():
    g = json.load(open(os.path.join(GOLD, "splitmix64.json")))
    gamma = int(g["gamma"], 16)
    got = [oracle.splitmix64((g["seed"] + i * gamma) % 2 ** 64) for i in range(len(g["outputs"]))]
    assert got == [int(x) for x in g["outputs"]]


def test_uniform_is_24_bit_and_uniform():
    u = np.array([oracle.uniform(3, r, s, d) for r in range(200) for s in range(5) for d in range(9)])
    assert np.all(u >= 0) and np.all(u < 1)
    assert np.all(np.floor(u * 2 ** 24) == u * 2 ** 24)
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    # every coordinate of (seed, ray, sample, dim) changes the value
    base = oracle.uniform(1, 2, 3, 4)
    assert len({base, oracle.uniform(2, 2, 3, 4), oracle.uniform(1, 3, 3, 4), oracle.uniform(1, 2, 4, 4),
                oracle.uniform(1, 2, 3, 5)}) == 5


# --- frames ------------------------------------------------------------------------------

def test_quaternion_frame_closed_form():
    for th in (0.3, 1.7, -2.5):
        q = [np.cos(th / 2), 0, 0, np.sin(th / 2)]  # rotation about z
        tu, tv, n = oracle.quat_to_frame(q)
        np.testing.assert_allclose(tu, [np.cos(th), np.sin(th), 0], atol=1e-15)
        np.testing.assert_allclose(tv, [-np.sin(th), np.cos(th), 0], atol=1e-15)
        np.testing.assert_allclose(n, [0, 0, 1], atol=1e-15)
    rng = np.random.default_rng(0)
    for q in rng.standard_normal((50, 4)):
        tu, tv, n = oracle.quat_to_frame(q)
        F = np.stack([tu, tv, n], 1)
        np.testing.assert_allclose(F.T @ F, np.eye(3), atol=1e-14)
        assert np.linalg.det(F) == pytest.approx(1.0, abs=1e-14)
        np.testing.assert_allclose(oracle.quat_to_frame(3.7 * q)[2], n, atol=1e-15)


def test_onb_orthonormal_right_handed():
    rng = np.random.default_rng(1)
    ns = list(scenegen.unit_vectors(rng, 200)) + [np.array([0, 0, 1.0]), np.array([0, 0, -1.0])]
    for n in ns:
        b1, b2 = oracle.onb(n)
        F = np.stack([b1, b2, n], 1)
        np.testing.assert_allclose(F.T @ F, np.eye(3), atol=1e-13)
        np.testing.assert_allclose(np.cross(b1, b2), n, atol=1e-13)


# --- BRDF ---------------------------------------------------------------------------------

@pytest.mark.parametrize("r", [0.08, 0.2, 0.5, 1.0])
def test_ggx_normalisation(r):
    val, _ = integrate.quad(lambda th: oracle.ggx_D(np.cos(th), r) * np.cos(th) * np.sin(th) * 2 * np.pi,
                            0, np.pi / 2, limit=400, points=[1e-3, 1e-2, 0.1])
    assert val == pytest.approx(1.0, abs=2e-7)


def test_smith_g1_bounds():
    for r in (0.1, 0.5, 1.0):
        assert oracle.smith_G1(1.0, r) == pytest.approx(1.0, abs=1e-15)
        cs = np.linspace(1e-3, 1, 50)
        g = np.array([oracle.smith_G1(c, r) for c in cs])
        assert np.all(g > 0) and np.all(g <= 1 + 1e-15) and np.all(np.diff(g) > 0)
    # alpha_g = 1 reduces the Smith term to 2c / (1 + c)
    assert oracle.smith_G1(0.3, 1.0) == pytest.approx(0.6 / 1.3, rel=1e-14)


def test_brdf_normal_incidence_and_lambert():
    n = np.array([0, 0, 1.0])
    a, m, r = np.array([0.8, 0.4, 0.2]), 0.3, 0.5
    f = oracle.brdf(n, n, n, a, m, r)
    F0 = 0.04 * (1 - m) + a * m
    D1 = 1.0 / (np.pi * r ** 4)  # D(n.h = 1) = 1 / (pi alpha_g^2), alpha_g = r^2
    np.testing.assert_allclose(f, (1 - m) * a / np.pi + D1 * F0 / 4, rtol=1e-13)
    fd = oracle.brdf(n, np.array([0.6, 0, 0.8]), n, a, m, r, oracle.DIFFUSE_ONLY)
    np.testing.assert_allclose(fd, (1 - m) * a / np.pi, rtol=1e-15)
    # below the surface: zero
    assert np.all(oracle.brdf(n, np.array([0.6, 0, -0.8]), n, a, m, r) == 0)


def test_brdf_reciprocity():
    rng = np.random.default_rng(2)
    n = np.array([0, 0, 1.0])
    for _ in range(100):
        wi, wo = scenegen.unit_vectors(rng, 2)
        wi[2], wo[2] = abs(wi[2]), abs(wo[2])
        a, m, r = rng.random(3), rng.random(), rng.random()
        np.testing.assert_allclose(oracle.brdf(n, wi, wo, a, m, r), oracle.brdf(n, wo, wi, a, m, r), rtol=1e-12)


def test_grazing_fresnel_tends_to_one():
    n = np.array([0, 0, 1.0])
    # near-grazing mirror configuration: v.h -> 0, F -> 1 whatever F0
    th = np.pi / 2 - 1e-4
    wo = np.array([np.sin(th), 0, np.cos(th)])
    wi = np.array([-np.sin(th), 0, np.cos(th)])
    f_hi = oracle.brdf(n, wi, wo, np.array([1.0, 1, 1]), 1.0, 0.3)
    f_lo = oracle.brdf(n, wi, wo, np.array([0.0, 0, 0]), 1.0, 0.3)  # F0 = 0
    np.testing.assert_allclose(f_lo / f_hi, 1.0, rtol=1e-3)


def _hemi_quad(fun, n_th=256, n_ph=256):
    """Midpoint quadrature over the upper hemisphere of +z."""
    th = (np.arange(n_th) + 0.5) * (np.pi / 2) / n_th
    ph = (np.arange(n_ph) + 0.5) * 2 * np.pi / n_ph
    tot = 0.0
    for t in th:
        for p in ph:
            w = np.array([np.sin(t) * np.cos(p), np.sin(t) * np.sin(p), np.cos(t)])
            tot += fun(w) * np.sin(t)
    return tot * (np.pi / 2 / n_th) * (2 * np.pi / n_ph)


def test_bsdf_pdf_integrates_to_one_for_cosine():
    n = np.array([0, 0, 1.0])
    wo = np.array([0.3, 0.1, 0.95])
    wo /= np.linalg.norm(wo)
    v = _hemi_quad(lambda w: oracle.pdf_bsdf(n, w, wo, np.array([0.5] * 3), 0.0, 0.5, oracle.DIFFUSE_ONLY), 64, 64)
    assert v == pytest.approx(1.0, abs=1e-3)
    # the mixture loses only the GGX mass that reflects below the horizon
    v2 = _hemi_quad(lambda w: oracle.pdf_bsdf(n, w, wo, np.array([0.5] * 3), 1.0, 0.3), 128, 128)
    assert 0.97 < v2 <= 1.0 + 1e-3


@pytest.mark.parametrize("m,r", [(0.0, 0.5), (1.0, 0.3), (0.5, 0.15)])
def test_bsdf_sampling_matches_pdf_chi2(m, r):
    rng = np.random.default_rng(4)
    n = np.array([0, 0, 1.0])
    wo = np.array([0.5, 0.0, 0.8660254037844386])
    a = np.array([0.7, 0.5, 0.3])
    N = 40000
    nb_t, nb_p = 8, 8
    counts = np.zeros((nb_t, nb_p))
    below = 0
    for _ in range(N):
        ok, w = oracle.sample_bsdf(n, wo, a, m, r, 0, *rng.random(3))
        if not ok:
            below += 1
            continue
        ct = w[2]
        ph = np.arctan2(w[1], w[0]) % (2 * np.pi)
        counts[min(int((1 - ct) * nb_t), nb_t - 1), min(int(ph / (2 * np.pi) * nb_p), nb_p - 1)] += 1
    # expected bin masses by quadrature of the pdf in (cos theta, phi)
    exp = np.zeros_like(counts)
    sub = 40
    for i in range(nb_t):
        for j in range(nb_p):
            acc = 0.0
            for si in range(sub):
                for sj in range(sub):
                    ct = 1 - (i + (si + 0.5) / sub) / nb_t
                    ph = (j + (sj + 0.5) / sub) / nb_p * 2 * np.pi
                    st = np.sqrt(max(0.0, 1 - ct * ct))
                    w = np.array([st * np.cos(ph), st * np.sin(ph), ct])
                    acc += oracle.pdf_bsdf(n, w, wo, a, m, r)
            exp[i, j] = acc / sub ** 2 * (1.0 / nb_t) * (2 * np.pi / nb_p) * N
    mask = exp > 20
    chi2 = ((counts[mask] - exp[mask]) ** 2 / exp[mask]).sum()
    dof = mask.sum() - 1
    assert stats.chi2.sf(chi2, dof) > 1e-4, (chi2, dof)


# --- environment ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def small_env():
    rng = np.random.default_rng(9)
    return scenegen.lognormal_env(rng, 8, 16, lobe_gain=50.0, lobe_width=0.3)


def test_env_pdf_integrates_to_one(small_env):
    H, W = small_env.shape[:2]
    sub = 8
    tot = 0.0
    for i in range(H * sub):
        th = (i + 0.5) * np.pi / (H * sub)
        for j in range(W * sub):
            ph = (j + 0.5) * 2 * np.pi / (W * sub)
            w = np.array([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)])
            tot += oracle.env_pdf(small_env, w) * np.sin(th)
    tot *= (np.pi / (H * sub)) * (2 * np.pi / (W * sub))
    assert tot == pytest.approx(1.0, abs=2e-3)


def test_env_sampling_chi2_and_pdf_consistency(small_env):
    H, W = small_env.shape[:2]
    rng = np.random.default_rng(5)
    lum = small_env @ np.array([0.2126, 0.7152, 0.0722])
    rw = lum.sum(1) * np.sin((np.arange(H) + 0.5) * np.pi / H)
    prob = (rw / rw.sum())[:, None] * lum / lum.sum(1, keepdims=True)
    N = 60000
    counts = np.zeros((H, W))
    for _ in range(N):
        pdf, w = oracle.env_sample(small_env, *rng.random(2))
        th = np.arccos(np.clip(w[1], -1, 1))
        ph = np.arctan2(w[2], w[0]) % (2 * np.pi)
        r, c = min(int(th / np.pi * H), H - 1), min(int(ph / (2 * np.pi) * W), W - 1)
        counts[r, c] += 1
        assert pdf == pytest.approx(oracle.env_pdf(small_env, w), rel=1e-6)  # acos near the poles
    exp = prob * N
    mask = exp > 10
    chi2 = ((counts[mask] - exp[mask]) ** 2 / exp[mask]).sum()
    assert stats.chi2.sf(chi2, mask.sum() - 1) > 1e-4


def test_env_single_hot_texel_direction():
    H, W = 8, 16
    env = np.zeros((H, W, 3), dtype=np.float32)
    env[3, 11] = 5.0
    rng = np.random.default_rng(6)
    for ua, ub in rng.random((50, 2)):
        pdf, w = oracle.env_sample(env, ua, ub)
        th = np.arccos(w[1])
        ph = np.arctan2(w[2], w[0]) % (2 * np.pi)
        assert 3 * np.pi / H - 1e-12 <= th <= 4 * np.pi / H + 1e-12
        assert 11 * 2 * np.pi / W - 1e-12 <= ph <= 12 * 2 * np.pi / W + 1e-12
        # all mass on one texel: pdf = H W / (2 pi^2 sin theta)
        assert pdf == pytest.approx(H * W / (2 * np.pi ** 2 * np.sin(th)), rel=1e-12)


def test_env_lookup_constant_and_texel_centres(small_env):
    c = scenegen.constant_env(2.5, 8, 16)
    for w in scenegen.unit_vectors(np.random.default_rng(7), 30):
        np.testing.assert_allclose(oracle.env_lookup(c, w), 2.5, rtol=1e-15)
    H, W = small_env.shape[:2]
    for r, col in [(2, 3), (5, 0), (4, 15)]:
        th, ph = (r + 0.5) * np.pi / H, (col + 0.5) * 2 * np.pi / W
        w = np.array([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)])
        np.testing.assert_allclose(oracle.env_lookup(small_env, w), small_env[r, col], rtol=1e-9)


# --- estimator ----------------------------------------------------------------------------

def _render_same_ray(scene, env, n, o, d, **kw):
    R, t = no_transforms(scene)
    sa = oracle.SceneArrays(scene, R, t, env)
    p = P(**{**dict(k=8, spp=1, seed=123), **kw})
    oo = np.tile(np.asarray(o, dtype=np.float64), (n, 1))
    dd = np.tile(np.asarray(d, dtype=np.float64) / np.linalg.norm(d), (n, 1))
    return oracle.render(sa, oo, dd, np.arange(n), p, lists=False)


def test_furnace_empty_scene():
    sc = make_scene(np.zeros((0, 3)))
    out = _render_same_ray(sc, scenegen.constant_env(1.7, 8, 16), 50, [0, 0, 3], [0.1, 0.2, -1], spp=4)
    assert np.all(out["radiance"] == np.float32(1.7))


@pytest.mark.parametrize("opacity", [1.0, 0.5])
def test_furnace_zero_variance_lambert(opacity):
    sc = make_scene([[0, 0, 0]], scale=[[10, 10]], opacity=[opacity], albedo=[[1, 1, 1]], metallic=[0])
    out = _render_same_ray(sc, scenegen.constant_env(1.0, 8, 16), 400, [0.1, 0, 2], [0, 0.2, -1], spp=4,
                           flags=oracle.DIFFUSE_ONLY | oracle.BSDF_ONLY)
    # every sample returns a_bar * c with a_bar = A/(A+eps) (Eq. surface-record's epsilon):
    # L = A * A/(A+eps) * c + T * c, with zero variance
    A = out["alpha"][:, None]
    np.testing.assert_allclose(out["radiance"], np.repeat(A * A / (A + 1e-6) + (1 - A), 3, 1), rtol=0, atol=1e-12)
    assert np.all(np.abs(out["radiance"] - 1.0) < 2e-6)
    assert np.all(out["sec_alpha"] == 0.0)  # secondaries escape


def test_furnace_zero_variance_with_occluding_roof():
    sc = make_scene([[0, 0, 0], [0, 0, 0.5]], scale=[[10, 10]] * 2, opacity=[1, 1], albedo=[[1, 1, 1]] * 2,
                    metallic=[0, 0])
    out = _render_same_ray(sc, scenegen.constant_env(1.0, 8, 16), 400, [0, 0, 0.25], [0, 0, -1], spp=2,
                           flags=oracle.DIFFUSE_ONLY | oracle.BSDF_ONLY)
    A2 = out["sec_alpha"]
    assert np.mean(A2 > 0.9) > 0.9  # the roof really occludes
    # L_in = T2 c + A2 * (a2_bar c) with a2_bar = A2/(A2+eps); every sample is a_bar * L_in
    Lin = (1 - A2) + A2 * A2 / (A2 + 1e-6)
    A = out["alpha"]
    want = A * A / (A + 1e-6) * Lin.mean(1) + (1 - A)
    np.testing.assert_allclose(out["radiance"], np.repeat(want[:, None], 3, 1), rtol=0, atol=1e-12)
    assert np.all(np.abs(out["radiance"] - 1.0) < 3e-6)


def test_grey_roof_matches_quadrature():
    """Floor (white Lambert) under a roof of albedo 0.5: L = c (1 - 0.5 E_cos[A2])."""
    s_roof, h_roof, off = 10.0, 0.5, 1e-3
    sc = make_scene([[0, 0, 0], [0, 0, h_roof]], scale=[[10, 10], [s_roof, s_roof]], opacity=[1, 1],
                    albedo=[[1, 1, 1], [0.5, 0.5, 0.5]], metallic=[0, 0])
    N = 20000
    out = _render_same_ray(sc, scenegen.constant_env(1.0, 8, 16), N, [0, 0, 0.25], [0, 0, -1], spp=1,
                           flags=oracle.DIFFUSE_ONLY | oracle.BSDF_ONLY)
    h = h_roof - off

    def a2(th):
        rho2 = (h * np.tan(th) / s_roof) ** 2
        if rho2 > min(9.0, 2 * np.log(255.0)):
            return 0.0
        return min(0.99, np.exp(-0.5 * rho2))

    EA2, _ = integrate.quad(lambda th: a2(th) * 2 * np.cos(th) * np.sin(th), 0, np.pi / 2, limit=200)
    A, T = 0.99, 0.01
    want = A * (1 - 0.5 * EA2) + T
    L = out["radiance"][:, 0]
    assert abs(L.mean() - want) < 4 * L.std() / np.sqrt(N) + 1e-12


@pytest.mark.parametrize("m,r,flags", [(0.0, 0.5, oracle.DIFFUSE_ONLY), (1.0, 0.4, 0), (0.4, 0.25, 0)])
def test_mis_estimator_unbiased_against_quadrature(m, r, flags, small_env):
    """Unshadowed one-sample MIS over {env IS, BSDF mixture} has the mean of
    the reflectance integral int f cos E dw (Eq. rendering-equation)."""
    a = np.array([0.9, 0.6, 0.3])
    sc = make_scene([[0, 0, 0]], scale=[[10, 10]], opacity=[1.0], albedo=[a], metallic=[m], roughness=[r])
    d = np.array([0.3, -0.2, -1.0])
    d /= np.linalg.norm(d)
    N = 60000
    out = _render_same_ray(sc, small_env, N, -3 * d, d, spp=1, flags=flags | oracle.NO_SECONDARY)
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
    Ed = oracle.env_lookup(small_env, d)
    want = 0.99 * acc + 0.01 * Ed
    L = out["radiance"]
    se = L.std(0) / np.sqrt(N)
    assert np.all(np.abs(L.mean(0) - want) < 4 * se + 2e-3 * np.abs(want)), (L.mean(0), want, se)


def test_metallic_furnace_loses_energy():
    sc = make_scene([[0, 0, 0]], scale=[[10, 10]], opacity=[1.0], albedo=[[1, 1, 1]], metallic=[1.0],
                    roughness=[0.6])
    N = 20000
    out = _render_same_ray(sc, scenegen.constant_env(1.0, 8, 16), N, [0.3, 0, 2], [-0.1, 0, -1], spp=1,
                           flags=oracle.NO_SECONDARY)
    L = out["radiance"][:, 0]
    assert L.mean() <= 1.0 + 4 * L.std() / np.sqrt(N)
    assert L.mean() > 0.8
