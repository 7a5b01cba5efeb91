"""Pins of the FP64 geometry-objective reference (oracle/losses.py) against
closed forms, exact geometric facts and finite differences: coverage and
scale terms (Sec. 3.1, Eq. alpha-coverage, Eq. scale-regularization), depth
and normal terms (Sec. 3.2, Eq. reconstruction-depth,
Eq. reconstruction-normal)."""
import numpy as np
import pytest

from oracle import losses as OL


def _fd(f, x, idx, h=1e-6):
    xp, xm = x.copy(), x.copy()
    xp.flat[idx] += h
    xm.flat[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


def _pinhole(h, w, fov_deg=50.0, eye=(0.3, -0.2, 4.0)):
    """FP64 unit rays of a camera at `eye` looking down -z (row y = 0 on top)
    and the unnormalised directions r(x, y), which are affine in (x, y)."""
    th = np.tan(np.radians(fov_deg) / 2)
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    rx = (2 * (xs + 0.5) / w - 1) * th * w / h
    ry = (1 - 2 * (ys + 0.5) / h) * th
    r = np.stack([rx, ry, -np.ones_like(rx)], axis=-1)
    o = np.broadcast_to(np.asarray(eye, np.float64), r.shape).copy()
    d = r / np.linalg.norm(r, axis=-1, keepdims=True)
    return o.reshape(-1, 3), d.reshape(-1, 3), r, (2 * th * w / h / w, -2 * th / h)


# -- scene-linear L1 data term (Sec. 3.4, Eq. training-objectives) ------------

def test_l1_closed_forms():
    # a constant offset c on every value: loss |c|, gradient sign(c)/n
    t = np.random.default_rng(1).uniform(0, 5, (10, 3))
    for c in (0.75, -2.5):
        loss, g = OL.l1_loss(t + c, t)
        assert loss == pytest.approx(abs(c), rel=1e-13)
        assert np.array_equal(g, np.full(30, np.sign(c) / 30))
    # the mean runs over pixels x channels: one channel of one pixel off by d
    p = t.copy()
    p[4, 1] += 3.0
    loss, g = OL.l1_loss(p, t)
    assert loss == pytest.approx(3.0 / 30, rel=1e-13)
    assert g[4 * 3 + 1] == 1.0 / 30 and np.count_nonzero(g) == 1
    # exact ties: sign(0) = 0
    loss, g = OL.l1_loss(t, t)
    assert loss == 0.0 and not g.any()
    assert OL.l1_loss(np.zeros(0), np.zeros(0))[0] == 0.0
    # HDR values are not tonemapped: the loss is linear in a common scale
    q = np.random.default_rng(2).uniform(0, 1, 30)
    assert OL.l1_loss(1e3 * q, 1e3 * t)[0] == pytest.approx(1e3 * OL.l1_loss(q, t)[0], rel=1e-13)
    with pytest.raises(ValueError):
        OL.l1_loss(np.zeros(3), np.zeros(4))


def test_l1_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    t = rng.uniform(0, 4, 50)
    p = t + rng.choice([-1.0, 1.0], 50) * rng.uniform(0.1, 1.0, 50)  # every residual away from the kink
    _, g = OL.l1_loss(p, t)
    for i in (0, 17, 49):
        assert g[i] == pytest.approx(_fd(lambda v: OL.l1_loss(v, t)[0], p, i), rel=1e-7)


# -- coverage (Eq. alpha-coverage) -------------------------------------------

def test_coverage_closed_forms():
    assert OL.coverage_loss(np.ones(100))[0] == 0.0
    assert OL.coverage_loss(np.zeros(100))[0] == 1.0
    loss, g = OL.coverage_loss(np.full(64, 0.25))
    assert loss == pytest.approx(0.75, abs=1e-15)
    assert np.allclose(g, -1.0 / 64)
    assert OL.coverage_loss(np.zeros(0))[0] == 0.0


def test_coverage_gradient_matches_finite_differences():
    a = np.random.default_rng(0).uniform(0.05, 0.95, 40)
    _, g = OL.coverage_loss(a)
    for i in (0, 7, 39):
        assert g[i] == pytest.approx(_fd(lambda v: OL.coverage_loss(v)[0], a, i), rel=1e-7)


# -- scale regulariser (Eq. scale-regularization) -----------------------------

def test_scale_closed_forms():
    s_max = 0.1
    s = np.full((5, 2), 0.05)
    assert OL.scale_loss(s, s_max)[0] == 0.0
    s[2] = (0.01, 0.2)  # infinity norm 2 s_max -> term (2-1)^2 = 1
    loss, g = OL.scale_loss(s, s_max)
    assert loss == pytest.approx(1.0 / 5, abs=1e-15)
    assert g[2, 0] == 0.0 and g[2, 1] == pytest.approx(2 * 1.0 / (5 * s_max))
    assert not np.any(g[[0, 1, 3, 4]])
    s[2] = (0.3, 0.01)  # the other component is the maximum -> (3-1)^2 = 4
    assert OL.scale_loss(s, s_max)[0] == pytest.approx(4.0 / 5)


def test_scale_gradient_matches_finite_differences():
    s = np.random.default_rng(1).uniform(0.01, 0.3, (30, 2))
    _, g = OL.scale_loss(s, 0.1)
    for i in range(0, 60, 7):
        assert g.flat[i] == pytest.approx(_fd(lambda v: OL.scale_loss(v, 0.1)[0], s, i), rel=1e-6, abs=1e-12)


# -- depth (Eq. reconstruction-depth) ------------------------------------------

def test_depth_closed_forms():
    rng = np.random.default_rng(2)
    ref = rng.uniform(1, 3, 50)
    conf = rng.uniform(0, 1, 50)
    assert OL.depth_loss(ref, ref, conf, 1e-6)[0] == 0.0
    # D = 2 D*, C = 1: the relative error is exactly ||D*|| / (||D*|| + eps)
    s = ref.sum()
    assert OL.depth_loss(2 * ref, ref, np.ones(50), 0.5)[0] == pytest.approx(s / (s + 0.5), rel=1e-14)
    # zero confidence removes a pixel from numerator and denominator
    c = np.ones(50)
    c[:25] = 0
    d = ref.copy()
    d[:25] += 10
    assert OL.depth_loss(d, ref, c, 1e-6)[0] == 0.0


def test_depth_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    ref = rng.uniform(1, 3, 30)
    d = ref + rng.choice([-1, 1], 30) * rng.uniform(0.05, 0.5, 30)
    conf = rng.uniform(0.1, 1, 30)
    _, g = OL.depth_loss(d, ref, conf, 1e-3)
    for i in (0, 11, 29):
        assert g[i] == pytest.approx(_fd(lambda v: OL.depth_loss(v, ref, conf, 1e-3)[0], d, i), rel=1e-6)


# -- rendered normal (Eq. reconstruction-normal, L_N) --------------------------

def test_normal_closed_forms():
    rng = np.random.default_rng(4)
    n = rng.normal(size=(20, 3))
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    assert OL.normal_loss(n, n)[0] == pytest.approx(0.0, abs=1e-15)
    assert OL.normal_loss(-n, n)[0] == pytest.approx(2.0, abs=1e-15)
    ortho = np.cross(n, rng.normal(size=(20, 3)))
    ortho /= np.linalg.norm(ortho, axis=1, keepdims=True)
    assert OL.normal_loss(ortho, n)[0] == pytest.approx(1.0, abs=1e-14)
    assert OL.normal_loss(np.zeros((20, 3)), n)[0] == 1.0


def test_normal_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    a, r = rng.normal(size=(12, 3)), rng.normal(size=(12, 3))
    _, g = OL.normal_loss(a, r)
    for i in (0, 17, 35):
        assert g.flat[i] == pytest.approx(_fd(lambda v: OL.normal_loss(v, r)[0], a, i), rel=1e-8)


# -- depth-derived normal ------------------------------------------------------

def test_planar_depth_gives_the_plane_normal_facing_the_camera():
    h, w = 9, 13
    o, d, _, _ = _pinhole(h, w)
    for nrm, c in (((0.0, 0.0, 1.0), 0.0), ((0.3, -0.5, 0.8), -0.2), ((-0.6, 0.1, 0.5), 0.4)):
        n = np.asarray(nrm) / np.linalg.norm(nrm)
        depth = (c - o @ n) / (d @ n)  # ray parameter of the plane n.X = c
        assert np.all(depth > 0)
        N = OL.depth_normals(o, d, depth, h, w).reshape(h, w, 3)
        inner = N[1:-1, 1:-1].reshape(-1, 3)
        facing = n if (d @ n).mean() < 0 else -n
        assert np.abs(inner - facing).max() < 1e-12
        assert not N[0].any() and not N[-1].any() and not N[:, 0].any() and not N[:, -1].any()


def test_quadratic_surface_normals_are_the_exact_tangent_cross_product():
    # P(x, y) = o + f(x, y) r(x, y) with f and r affine in the pixel
    # coordinates is quadratic, so central differences equal twice the exact
    # derivatives; a forward difference or a swapped operand would not match.
    h, w = 11, 15
    o, d, r, (rx_x, ry_y) = _pinhole(h, w)
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float64)
    al, be, ga = 3.0, 0.09, -0.07
    f = al + be * xs + ga * ys
    depth = (f * np.linalg.norm(r, axis=-1)).reshape(-1)
    Px = be * r + f[..., None] * np.array([rx_x, 0.0, 0.0])
    Py = ga * r + f[..., None] * np.array([0.0, ry_y, 0.0])
    want = -np.cross(Px, Py)
    want /= np.linalg.norm(want, axis=-1, keepdims=True)
    N = OL.depth_normals(o, d, depth, h, w).reshape(h, w, 3)
    assert np.abs(N[1:-1, 1:-1] - want[1:-1, 1:-1]).max() < 1e-12
    assert np.all((N[1:-1, 1:-1] * d.reshape(h, w, 3)[1:-1, 1:-1]).sum(-1) < 0)  # faces the camera


def test_depth_normals_of_a_sphere_converge_to_the_radial_normal():
    errs = []
    for h in (24, 48):
        w = h
        o, d, _, _ = _pinhole(h, w, fov_deg=20.0, eye=(0.0, 0.0, 4.0))
        # unit sphere at the origin: nearest root of |o + t d|^2 = 1
        b = (o * d).sum(1)
        disc = b * b - ((o * o).sum(1) - 1)
        hit = disc > 0
        depth = np.where(hit, -b - np.sqrt(np.maximum(disc, 0)), 0.0)
        N = OL.depth_normals(o, d, depth, h, w)
        X = o + depth[:, None] * d
        ok = np.linalg.norm(N, axis=1) > 0
        assert ok.sum() > 0.4 * hit.sum()
        assert not np.any(ok & ~hit)  # no normal where there is no surface
        # stay away from the silhouette, where the finite differences straddle it
        core = ok & ((X * d).sum(1) < -0.5)
        errs.append(np.abs(N[core] - X[core]).max())
    assert errs[0] < 2e-2 and errs[1] < errs[0] / 3  # second order in the pixel pitch


def test_depth_normal_loss_of_a_plane_against_its_own_normal():
    h, w = 7, 10
    o, d, _, _ = _pinhole(h, w)
    n = np.array([0.2, 0.1, 1.0])
    n /= np.linalg.norm(n)
    depth = (0.0 - o @ n) / (d @ n)
    loss, _ = OL.depth_normal_loss(o, d, depth, np.tile(n, (h * w, 1)), h, w)
    assert loss == pytest.approx(1.0 - (h - 2) * (w - 2) / (h * w), abs=1e-12)


def test_depth_normal_gradient_matches_finite_differences():
    h, w = 8, 9
    o, d, _, _ = _pinhole(h, w)
    rng = np.random.default_rng(6)
    depth = 3.5 + 0.2 * rng.normal(size=h * w)
    depth[5] = 0.0  # a pixel without surface: its neighbours get no normal
    ref = rng.normal(size=(h * w, 3))
    ref /= np.linalg.norm(ref, axis=1, keepdims=True)
    _, g = OL.depth_normal_loss(o, d, depth, ref, h, w)
    f = lambda v: OL.depth_normal_loss(o, d, v, ref, h, w)[0]  # noqa: E731
    for i in (0, 10, 14, 31, 40, 55, 71):
        assert g[i] == pytest.approx(_fd(f, depth, i, h=1e-7), rel=1e-5, abs=1e-10)
    assert g[5] == 0.0  # every normal that would use it is undefined
    assert np.all(np.isfinite(g))


# -- total variation of the environment map (Eq. training-objectives) ------------------

def test_tv_closed_forms():
    H, W = 6, 10
    assert OL.tv_loss(np.full((H, W, 3), 2.5))[0] == 0.0
    E = np.zeros((H, W, 3))
    E[2, 4, 1] = 3.0  # one hot texel in one channel: two horizontal and two vertical jumps of 3
    loss, g = OL.tv_loss(E)
    assert loss == pytest.approx(4 * 3.0 / (3 * H * W), abs=1e-15)
    assert g[2, 4, 1] == pytest.approx(4 / (3 * H * W)) and g[2, 3, 1] == pytest.approx(-1 / (3 * H * W))
    # azimuth wraps: a ramp 0..W-1 along x jumps back by W-1 between the last and the first column
    R = np.tile(np.arange(W, dtype=np.float64)[None, :, None], (H, 1, 3))
    assert OL.tv_loss(R)[0] == pytest.approx(H * 3 * (2 * (W - 1)) / (3 * H * W))
    # no wrap over the poles: a ramp along y costs (H-1) per column
    V = np.tile(np.arange(H, dtype=np.float64)[:, None, None], (1, W, 3))
    assert OL.tv_loss(V)[0] == pytest.approx(W * 3 * (H - 1) / (3 * H * W))
    assert OL.tv_loss(np.zeros((1, 1, 3)))[0] == 0.0


def test_tv_gradient_matches_finite_differences():
    E = np.random.default_rng(12).uniform(0, 5, (5, 7, 3))
    _, g = OL.tv_loss(E)
    for i in (0, 17, 40, 104):
        assert g.flat[i] == pytest.approx(_fd(lambda v: OL.tv_loss(v)[0], E, i), rel=1e-6, abs=1e-12)
