"""Pins of the oracle's tracing and compositing (Sec. 3.2, Eq. gaussian-response,
Eq. surface-record) against closed forms, invariants and an independent NumPy
brute force.  CPU only."""
import numpy as np
import pytest

import oracle
import scenegen
from tests import ref_numpy
from tests.helpers import axis_angle_quat, make_scene, no_transforms, rays_single

P = oracle.Params


def run(scene, o, d, ids, env=None, R=None, t=None, **kw):
    if R is None:
        R, t = no_transforms(scene)
    if env is None:
        env = scenegen.constant_env(1.0, 8, 16)
    sa = oracle.SceneArrays(scene, R, t, env)
    p = P(**{**dict(k=16, spp=1, seed=7, flags=oracle.NO_SECONDARY), **kw})
    return oracle.render(sa, o, d, ids, p)


# --- single surfel at a known depth and normal -------------------------------------------

@pytest.mark.parametrize("tilt", [0.0, 0.4, -1.1])
def test_single_surfel_depth_normal(tilt):
    # normal n = R_x(tilt) e_z; ray straight down the z axis through the centre
    q = axis_angle_quat([1, 0, 0], tilt).astype(np.float32)
    sc = make_scene([[0, 0, 0]], q=[q], opacity=[0.7], scale=[[0.2, 0.3]])
    out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]))
    at = float(np.float32(0.7))  # rho = 0 at the centre
    assert out["alpha"][0] == pytest.approx(at, rel=1e-15)
    assert out["depth"][0] == pytest.approx(at * 5.0 / (at + 1e-6), rel=1e-14)
    th = 2.0 * np.arctan2(float(q[1]), float(q[0]))  # angle of the stored (float32) quaternion
    n = np.array([0.0, -np.sin(th), np.cos(th)])  # R_x(th) e_z
    np.testing.assert_allclose(out["normal"][0], n, atol=1e-14)  # already faces +z viewer
    # the same surfel seen from below: same depth, normal flipped towards the viewer
    out2 = run(sc, *rays_single([0, 0, -5], [0, 0, 1]))
    assert out2["depth"][0] == pytest.approx(out["depth"][0], rel=1e-14)
    np.testing.assert_allclose(out2["normal"][0], -n, atol=1e-14)


@pytest.mark.parametrize("x0,y0", [(0.05, 0.0), (0.0, 0.1), (0.13, -0.21), (-0.3, 0.2)])
def test_single_surfel_effective_opacity(x0, y0):
    su, sv, a = 0.2, 0.35, 0.8
    sc = make_scene([[0, 0, 0]], scale=[[su, sv]], opacity=[a])
    out = run(sc, *rays_single([x0, y0, 3], [0, 0, -1]))
    su, sv, a = float(np.float32(su)), float(np.float32(sv)), float(np.float32(a))
    want = a * np.exp(-0.5 * ((x0 / su) ** 2 + (y0 / sv) ** 2))
    assert out["alpha"][0] == pytest.approx(want, rel=1e-12)
    assert out["transmittance"][0] == pytest.approx(1 - want, rel=1e-12)


def test_support_radius_three_sigma():
    # alpha = 1 -> opacity threshold radius sqrt(2 ln 255) = 3.33 > 3: the 3-sigma support binds
    s = 0.25
    sc = make_scene([[0, 0, 0]], scale=[[s, s]], opacity=[1.0])
    s = float(np.float32(s))
    inside = run(sc, *rays_single([2.999 * s, 0, 1], [0, 0, -1]))
    outside = run(sc, *rays_single([3.001 * s, 0, 1], [0, 0, -1]))
    assert inside["hit_idx"][0, 0] == 0 and inside["alpha"][0] > 0
    assert outside["hit_idx"][0, 0] == -1 and outside["alpha"][0] == 0.0


def test_opacity_threshold_before_cap():
    a, s = float(np.float32(0.1)), float(np.float32(0.25))
    rho_thr = np.sqrt(2.0 * np.log(float(a) * 255.0))  # alpha exp(-rho^2/2) = 1/255
    assert rho_thr < 3.0
    sc = make_scene([[0, 0, 0]], scale=[[s, s]], opacity=[a])
    inside = run(sc, *rays_single([(rho_thr - 1e-6) * s, 0, 1], [0, 0, -1]))
    outside = run(sc, *rays_single([(rho_thr + 1e-6) * s, 0, 1], [0, 0, -1]))
    assert inside["hit_idx"][0, 0] == 0
    assert inside["alpha"][0] == pytest.approx(1 / 255, rel=1e-5)
    assert outside["hit_idx"][0, 0] == -1


def test_cap_at_099():
    sc = make_scene([[0, 0, 0], [0, 0, -1]], opacity=[1.0, 1.0])
    out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]))
    # each layer: alpha_t = min(0.99, 1) -> T = 0.01 per layer
    assert out["transmittance"][0] == pytest.approx(0.01 * 0.01, rel=1e-12)
    assert out["alpha"][0] == pytest.approx(1 - 1e-4, rel=1e-12)


def test_transmittance_product_and_order_independence():
    rng = np.random.default_rng(3)
    n = 9
    ts = 1.0 + 0.1 * np.arange(n)
    a = rng.uniform(0.05, 0.9, n).astype(np.float32).astype(np.float64)
    mu = np.stack([np.zeros(n), np.zeros(n), 5.0 - ts], 1)
    perm = rng.permutation(n)
    for order in (np.arange(n), perm):
        sc = make_scene(mu[order], opacity=a[order], scale=np.full((n, 2), 1.0))
        out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]), k=16)
        tj = 5.0 - mu[:, 2].astype(np.float32).astype(np.float64)  # centres are stored in float32
        Tj = np.concatenate([[1.0], np.cumprod(1 - a)])
        w = Tj[:-1] * a
        A = 1 - Tj[-1]
        assert out["transmittance"][0] == pytest.approx(Tj[-1], rel=1e-13)
        assert out["alpha"][0] == pytest.approx(A, rel=1e-13)
        assert out["depth"][0] == pytest.approx((w * tj).sum() / (A + 1e-6), rel=1e-13)
        assert list(out["hit_idx"][0, :n]) == list(np.argsort(order))


def test_exact_tie_lower_index_first():
    # surfel 1 and surfel 2 are identical: the lower index must come first
    sc = make_scene([[0, 0, -1], [0, 0, 0], [0, 0, 0]], opacity=[0.5, 0.3, 0.6])
    out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]))
    assert list(out["hit_idx"][0, :3]) == [1, 2, 0]
    a1, a2, a0 = (float(np.float32(v)) for v in (0.3, 0.6, 0.5))
    A = a1 + (1 - a1) * a2 + (1 - a1) * (1 - a2) * a0
    assert out["alpha"][0] == pytest.approx(A, rel=1e-14)


def test_truncation_to_k():
    n, k = 12, 5
    mu = np.stack([np.zeros(n), np.zeros(n), -0.1 * np.arange(n)], 1)
    a = np.full(n, 0.3, dtype=np.float32).astype(np.float64)
    sc = make_scene(mu, opacity=a, scale=np.ones((n, 2)))
    out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]), k=k)
    assert list(out["hit_idx"][0]) == list(range(k))
    assert out["alpha"][0] == pytest.approx(1 - 0.7 ** k, rel=1e-6)
    assert out["transmittance"][0] == pytest.approx(float(np.prod(1 - a[:k])), rel=1e-14)


def test_below_threshold_hits_do_not_count_toward_k():
    # a faint surfel (alpha < 1/255) in front never occupies a slot
    sc = make_scene([[0, 0, 1], [0, 0, 0]], opacity=[0.003, 0.5])
    out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]), k=1)
    assert out["hit_idx"][0, 0] == 1


def test_t_min_culls_hits_behind_the_origin():
    sc = make_scene([[0, 0, 0], [0, 0, 6], [0, 0, 5 - 5e-5]])
    out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]))
    assert list(out["hit_idx"][0, :2]) == [0, -1]


# --- invariants on the C1 workload ----------------------------------------------------

@pytest.fixture(scope="module")
def c1():
    wl = scenegen.make_workload(1)
    st = wl.states[0]
    o, d, ids = oracle.raygen(st.cameras[0])
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    out = oracle.render(sa, o, d, ids, P(k=wl.k, spp=1, seed=wl.seed, flags=oracle.NO_SECONDARY))
    return wl, o, d, ids, out


def test_c1_invariants(c1):
    wl, o, d, ids, out = c1
    A, T = out["alpha"], out["transmittance"]
    nh = (out["hit_idx"] >= 0).sum(1)
    np.testing.assert_allclose(A + T, 1.0, atol=1e-12)
    assert np.all(A >= 0) and np.all(A <= 1 - 0.01 ** nh + 1e-15)
    hit = nh > 0
    assert hit.mean() > 0.5
    # composited normal faces the viewer on every hit ray
    assert np.all(np.einsum("ij,ij->i", out["normal"][hit], -d[hit].astype(np.float64)) > 0)
    np.testing.assert_allclose(np.linalg.norm(out["normal"][hit], axis=1), 1.0, atol=1e-12)
    assert np.all(out["normal"][~hit] == 0) and np.all(out["depth"][~hit] == 0)
    # hit lists are strictly index-unique and sorted by (t, index)
    for r in np.nonzero(hit)[0][:200]:
        h = out["hit_idx"][r, :nh[r]]
        assert len(set(h.tolist())) == len(h)


def test_c1_matches_independent_numpy(c1):
    wl, o, d, ids, out = c1
    sel = np.random.default_rng(0).choice(len(ids), 300, replace=False)
    hits, A, T, depth, normal = ref_numpy.trace(wl.scene, wl.states[0].R, wl.states[0].t, o[sel], d[sel], wl.k)
    assert np.array_equal(hits, out["hit_idx"][sel].astype(np.int64))
    np.testing.assert_allclose(A, out["alpha"][sel], rtol=0, atol=1e-12)
    np.testing.assert_allclose(T, out["transmittance"][sel], rtol=0, atol=1e-12)
    np.testing.assert_allclose(depth, out["depth"][sel], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(normal, out["normal"][sel], atol=1e-10)


def test_instanced_objects_match_numpy_and_flattened():
    rng = np.random.default_rng(11)
    wl = scenegen.make_workload(4, scale=0.004, resolution=24)  # 2000 + 8x80 surfels
    st = wl.states[0]
    o, d, ids = oracle.raygen(st.cameras[0])
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    out = oracle.render(sa, o, d, ids, P(k=32, spp=1, seed=1, flags=oracle.NO_SECONDARY))
    sel = rng.choice(len(ids), 120, replace=False)
    hits, A, T, depth, normal = ref_numpy.trace(wl.scene, st.R, st.t, o[sel], d[sel], 32)
    assert np.array_equal(hits, out["hit_idx"][sel].astype(np.int64))
    np.testing.assert_allclose(A, out["alpha"][sel], atol=1e-12)
    np.testing.assert_allclose(depth, out["depth"][sel], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(normal, out["normal"][sel], atol=1e-9)


def test_rigid_motion_equivariance():
    """Moving every surfel and the rays by one rigid motion leaves depth, A and
    (under a constant env) radiance unchanged and rotates the normals."""
    wl = scenegen.make_workload(1, scale=0.5)
    st = wl.states[0]
    o, d, ids = oracle.raygen(st.cameras[0])
    sel = np.arange(0, len(ids), 7)
    o, d, ids = o[sel].astype(np.float64), d[sel].astype(np.float64), ids[sel]
    p = P(k=16, spp=2, seed=5, flags=oracle.NO_SECONDARY)
    base = oracle.render(oracle.SceneArrays(wl.scene, st.R, st.t, st.env), o, d, ids, p)
    # express the same motion as an object instance over the whole scene
    qR = axis_angle_quat([0.3, -0.5, 0.8], 1.1)
    Rm = scenegen.quat_to_matrix_np(qR[None])[0]
    tm = np.array([0.4, -0.2, 0.7])
    sc = wl.scene.copy()
    sc.object_offset = np.array([0, 0, sc.n], dtype=np.int64)
    sa = oracle.SceneArrays(sc, Rm[None], tm[None], st.env)
    o2 = o @ Rm.T + tm
    d2 = d @ Rm.T
    # feed the oracle's own orthonormalisation of an exact rotation: R is exact here
    out = oracle.render(sa, o2, d2, ids, p)
    assert np.array_equal(out["hit_idx"], base["hit_idx"])
    np.testing.assert_allclose(out["depth"], base["depth"], rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(out["alpha"], base["alpha"], atol=1e-11)
    np.testing.assert_allclose(out["normal"], base["normal"] @ Rm.T, atol=1e-9)
    # constant env: the estimator is rotation invariant sample by sample only
    # when the local frames rotate too, so compare the pixel means
    assert abs(out["radiance"].mean() - base["radiance"].mean()) < 0.02


def test_identity_object_equals_background():
    wl = scenegen.make_workload(1, scale=0.5)
    st = wl.states[0]
    o, d, ids = oracle.raygen(st.cameras[0])
    p = P(k=16, spp=1, seed=5, flags=oracle.NO_SECONDARY)
    base = oracle.render(oracle.SceneArrays(wl.scene, st.R, st.t, st.env), o, d, ids, p)
    sc = wl.scene.copy()
    h = sc.n // 2
    sc.object_offset = np.array([0, h, sc.n], dtype=np.int64)
    out = oracle.render(oracle.SceneArrays(sc, np.eye(3)[None], np.zeros((1, 3)), st.env), o, d, ids, p)
    for k in ("hit_idx", "depth", "alpha", "normal", "radiance"):
        assert np.array_equal(out[k], base[k]), k


def test_raygen_matches_fp64_pinhole():
    rng = np.random.default_rng(8)
    cam = scenegen.sphere_camera(rng, 37, 23, fov_y_deg=50.0)
    o, d, pix = oracle.raygen(cam)
    pose = cam.pose.astype(np.float64).reshape(3, 4)
    th = np.tan(np.deg2rad(50.0) / 2)
    x, y = pix % 37 + 0.5, pix // 37 + 0.5
    dc = np.stack([(2 * x / 37 - 1) * th * 37 / 23, (1 - 2 * y / 23) * th, -np.ones_like(x)], 1)
    dw = dc @ pose[:, :3].T
    dw /= np.linalg.norm(dw, axis=1, keepdims=True)
    np.testing.assert_allclose(d, dw, atol=2e-6)
    np.testing.assert_allclose(np.linalg.norm(d.astype(np.float64), axis=1), 1.0, atol=1e-6)
    assert np.all(o == cam.pose.reshape(3, 4)[:, 3])
    # the camera looks at the origin: the central pixel's ray passes within one pixel of it
    c = (23 // 2) * 37 + 37 // 2
    closest = np.linalg.norm(np.cross(d[c].astype(np.float64), -o[c].astype(np.float64)))
    assert closest < 3.0 * 2 * th / 23
