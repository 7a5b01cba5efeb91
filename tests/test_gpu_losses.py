"""GPU parity of the geometry-refinement objectives (Sec. 3.1, Eq. alpha-coverage,
Eq. scale-regularization; Sec. 3.2, Eq. reconstruction-depth,
Eq. reconstruction-normal) against the FP64 reference in oracle/losses.py,
through the C ABI; and the objectives driving the replayed backward through
the tracer's depth, normal and alpha outputs.  Requires an MI355X.

Tolerances: the GPU sums in binary64 and writes binary32, so losses agree
to a few float ulps (rel 1e-6) and gradients elementwise to float rounding
(rel 1e-6 of each value, floored at 1e-6 of the largest)."""
import numpy as np
import pytest

import oracle
import scenegen
from oracle import losses as OL
from tests.gpu_common import ambiguous, dev, grad_check, state_args, upload_scene

pytestmark = pytest.mark.gpu

SIZES = (0, 1, 255, 257, 2048 * 256 + 37)  # empty, one, ragged blocks, past the grid-stride span


@pytest.fixture(scope="module")
def tracer():
    import paper_2608_29269_amd as lf
    return lf.Tracer()


def _close_loss(gpu, ref, rtol=1e-6, atol=1e-7):
    assert abs(float(gpu) - ref) <= rtol * abs(ref) + atol, (float(gpu), ref)


def _close_grad(gpu, ref, rtol=1e-6):
    a = gpu.detach().cpu().numpy().astype(np.float64).reshape(ref.shape)
    floor = 1e-6 * (np.abs(ref).max() if ref.size else 0.0)
    assert np.all(np.abs(a - ref) <= rtol * np.abs(ref) + floor + 1e-30), np.abs(a - ref).max()


@pytest.mark.parametrize("n", SIZES + (3 * 1024 * 1024,))
def test_l1_loss(tracer, n):
    # the scene-linear data term (Sec. 3.4, Eq. training-objectives) at the
    # sizes of a ragged launch and of a 1024x1024 RGB image, with exact ties
    rng = np.random.default_rng(400 + n)
    t = np.exp(rng.normal(0, 1.5, n)).astype(np.float32)  # HDR magnitudes
    p = (t * np.exp(rng.normal(0, 0.2, n))).astype(np.float32)
    p[: n // 9] = t[: n // 9]  # exact pixels: sign(0) = 0
    loss, g = tracer.l1_loss(dev(p), dev(t))
    ref, gref = OL.l1_loss(p, t)
    _close_loss(loss, ref)
    a = g.cpu().numpy().astype(np.float64)
    # sign(r)/n rounded once to binary32: equal to the reference within half an ulp
    assert np.array_equal(np.sign(a), np.sign(gref))
    assert np.all(np.abs(a - gref) <= 2.0 ** -24 * np.abs(gref)), np.abs(a - gref).max()
    lossonly, none = tracer.l1_loss(dev(p), dev(t), want_grad=False)
    assert none is None and float(lossonly) == float(loss)


@pytest.mark.parametrize("n", SIZES)
def test_coverage_loss(tracer, n):
    rng = np.random.default_rng(n)
    a = rng.uniform(0, 1, n).astype(np.float32)
    a[: n // 10] = 1.0  # fully covered pixels: sign(0) = 0
    loss, g = tracer.loss_alpha(dev(a))
    ref, gref = OL.coverage_loss(a)
    _close_loss(loss, ref)
    _close_grad(g, gref)


@pytest.mark.parametrize("n", SIZES)
def test_scale_loss(tracer, n):
    rng = np.random.default_rng(100 + n)
    s = np.exp(rng.uniform(np.log(0.01), np.log(0.3), (n, 2))).astype(np.float32)
    if n > 3:
        s[1] = (0.2, 0.2)  # tie: the first component takes the gradient
        s[2] = (0.05, 0.05)  # below the limit
    loss, g = tracer.loss_scale(dev(s), 0.1)
    ref, gref = OL.scale_loss(s, np.float64(np.float32(0.1)))
    _close_loss(loss, ref)
    _close_grad(g, gref)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("with_conf", [False, True])
def test_depth_loss(tracer, n, with_conf):
    rng = np.random.default_rng(200 + n)
    ref = rng.uniform(1, 5, n).astype(np.float32)
    d = (ref + rng.normal(0, 0.3, n)).astype(np.float32)
    d[: n // 7] = ref[: n // 7]  # exact pixels: sign(0) = 0
    conf = rng.uniform(0, 1, n).astype(np.float32) if with_conf else None
    loss, g = tracer.loss_depth(dev(d), dev(ref), dev(conf) if with_conf else None, eps=1e-3)
    want, gref = OL.depth_loss(d, ref, conf if with_conf else np.ones(n), np.float64(np.float32(1e-3)))
    _close_loss(loss, want)
    _close_grad(g, gref)


@pytest.mark.parametrize("n", SIZES)
def test_normal_loss(tracer, n):
    rng = np.random.default_rng(300 + n)
    nm = rng.normal(size=(n, 3))
    nm /= np.maximum(np.linalg.norm(nm, axis=1, keepdims=True), 1e-12)
    r = rng.normal(size=(n, 3))
    r /= np.maximum(np.linalg.norm(r, axis=1, keepdims=True), 1e-12)
    nm, r = nm.astype(np.float32), r.astype(np.float32)
    loss, g = tracer.loss_normal(dev(nm), dev(r))
    want, gref = OL.normal_loss(nm, r)
    _close_loss(loss, want)
    _close_grad(g, gref)


@pytest.mark.parametrize("h,w", [(1, 1), (1, 7), (5, 1), (17, 33), (128, 256), (256, 512)])
def test_tv_loss(tracer, h, w):
    rng = np.random.default_rng(h * 1000 + w)
    E = np.exp(rng.normal(0, 1, (h, w, 3))).astype(np.float32)
    if h * w > 4:
        E[h // 2, :, 1] = E[h // 2, 0, 1]  # a constant run: sign(0) = 0 in the gradient
    loss, g = tracer.loss_tv(dev(E))
    want, gref = OL.tv_loss(E)
    _close_loss(loss, want)
    _close_grad(g, gref)


def _depth_scene(cam, rng, holes=True):
    """Smooth depth of a tilted, gently curved surface seen by `cam`, with a
    few pixels without surface (depth 0)."""
    o, d, _ = oracle.raygen(cam)
    h, w = cam.h, cam.w
    ys, xs = np.mgrid[0:h, 0:w]
    depth = 3.0 + 0.4 * np.sin(xs / max(w, 1) * 3.1) * np.cos(ys / max(h, 1) * 2.3) + 0.1 * xs / max(w, 1)
    depth = depth.reshape(-1) + rng.normal(0, 1e-3, h * w)
    if holes:
        depth[rng.choice(h * w, max(1, h * w // 50), replace=False)] = 0.0
    ref = rng.normal(size=(h * w, 3))
    ref /= np.linalg.norm(ref, axis=1, keepdims=True)
    return o, d, depth.astype(np.float32), ref.astype(np.float32)


@pytest.mark.parametrize("w,h", [(1, 1), (3, 3), (37, 23), (64, 48), (130, 71)])
def test_depth_normal_loss(tracer, w, h):
    cam = scenegen.look_at_camera(np.array([0.4, -0.3, 3.0]), w, h, fov_y_deg=50.0)
    rng = np.random.default_rng(w * 1000 + h)
    o, d, depth, ref = _depth_scene(cam, rng)
    loss, g = tracer.loss_depth_normal(cam, dev(depth), dev(ref))
    want, gref = OL.depth_normal_loss(o, d, depth, ref, h, w)
    _close_loss(loss, want)
    _close_grad(g, gref, rtol=1e-5)


def test_depth_normal_loss_without_gradient_and_repeated(tracer):
    cam = scenegen.look_at_camera(np.array([0.0, 0.5, 3.0]), 40, 30, fov_y_deg=40.0)
    o, d, depth, ref = _depth_scene(cam, np.random.default_rng(7))
    want, _ = OL.depth_normal_loss(o, d, depth, ref, cam.h, cam.w)
    for _ in range(2):  # the accumulator is cleared by every call
        loss, g = tracer.loss_depth_normal(cam, dev(depth), dev(ref), want_grad=False)
        assert g is None
        _close_loss(loss, want)


def test_depth_normal_full_size_plane_and_sampled_gradients(tracer):
    """1024 x 1024, the benchmark's image size: the loss of a planar depth map
    against its own normal is the closed form 1 - (h-2)(w-2)/(hw) (up to the
    binary32 rounding of the depth), and sampled gradient entries match the
    reference evaluated on 7 x 7 crops (a pixel's gradient only reads depths
    within two pixels)."""
    import torch
    w = h = 1024
    cam = scenegen.look_at_camera(np.array([0.3, -2.0, 2.0]), w, h, fov_y_deg=60.0)
    o, d, _ = oracle.raygen(cam)
    n = np.array([0.1, 0.2, 1.0])
    n /= np.linalg.norm(n)
    depth = ((-0.5 - o.astype(np.float64) @ n) / (d.astype(np.float64) @ n))
    assert np.all(depth > 0)
    ref = np.tile(n if (d[0] @ n) < 0 else -n, (w * h, 1)).astype(np.float32)
    loss, _ = tracer.loss_depth_normal(cam, dev(depth.astype(np.float32)), dev(ref), want_grad=False)
    assert abs(float(loss) - (1.0 - (h - 2) * (w - 2) / (h * w))) < 1e-6

    rng = np.random.default_rng(11)
    o, d, depth, ref = _depth_scene(cam, rng)
    loss, g = tracer.loss_depth_normal(cam, dev(depth), dev(ref))
    torch.cuda.synchronize()
    g = g.cpu().numpy().astype(np.float64)
    ys = np.concatenate([[0, 1, 2, h - 1, h - 2], rng.integers(0, h, 40)])
    xs = np.concatenate([[0, 1, 2, w - 1, w - 2], rng.integers(0, w, 40)])
    for y, x in zip(ys, xs):
        y0, x0 = max(0, y - 3), max(0, x - 3)
        y1, x1 = min(h, y + 4), min(w, x + 4)
        cy, cx = y1 - y0, x1 - x0
        sel = (np.arange(y0, y1)[:, None] * w + np.arange(x0, x1)[None, :]).reshape(-1)
        # the crop reaches 3 pixels past the sample or stops at the image border
        _, gc = OL.depth_normal_loss(o[sel], d[sel], depth[sel], ref[sel], cy, cx)
        want = gc[(y - y0) * cx + (x - x0)] * (cy * cx) / (w * h)
        assert abs(g[y * w + x] - want) <= 1e-5 * abs(want) + 1e-12, (y, x, g[y * w + x], want)


def test_invalid_arguments_raise(tracer):
    import paper_2608_29269_amd as lf
    x = dev(np.ones(8, np.float32))
    with pytest.raises(lf.LFError):
        tracer.loss_scale(dev(np.ones((4, 2), np.float32)), 0.0)
    with pytest.raises(lf.LFError):
        tracer.loss_depth(x, x, None, eps=0.0)
    bad = scenegen.Camera(pose=np.eye(3, 4).reshape(-1), fov_y_deg=200.0, w=2, h=4)
    with pytest.raises(lf.LFError):
        tracer.loss_depth_normal(bad, x, dev(np.ones((8, 3), np.float32)))


def test_geometry_objectives_through_the_tracer(tracer):
    """Sec. 3.2 geometry refinement: L_D + L_N + L_DN + L_alpha on the rendered
    depth, normal and alpha maps.  The objectives on the GPU maps match the
    reference objectives on the oracle's maps, and the replayed backward
    driven by the reference objectives' map gradients matches the oracle's
    FP64 backward driven by the same upstream values."""
    wl = scenegen.make_workload(3, scale=0.02, resolution=40)
    st = wl.states[0]
    env = scenegen.lognormal_env(np.random.default_rng(5), 32, 64)
    st = scenegen.State(R=st.R, t=st.t, env=env, cameras=st.cameras)
    cam = st.cameras[0]
    o, d, ids = oracle.raygen(cam)
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    p = oracle.Params(k=wl.k, spp=1, seed=wl.seed, flags=1)
    fwd = oracle.render(sa, o, d, ids, p, lists=False)
    amb = ambiguous(fwd["margins"])
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    out = tracer.render(**args, cameras=[cam], k=wl.k, spp=1, seed=wl.seed, flags=1)
    rng = np.random.default_rng(9)
    n, h, w = len(ids), cam.h, cam.w
    d_ref = (fwd["depth"] * (1 + rng.normal(0, 0.05, n))).astype(np.float32)
    conf = (~amb).astype(np.float32) * rng.uniform(0.2, 1.0, n).astype(np.float32)
    n_ref = rng.normal(size=(n, 3))
    n_ref = (n_ref / np.linalg.norm(n_ref, axis=1, keepdims=True)).astype(np.float32)

    # objective values: GPU maps vs oracle maps (maps agree to float rounding off ambiguous rays)
    lg = [float(tracer.loss_depth(out["depth"], dev(d_ref), dev(conf), eps=1e-6)[0]),
          float(tracer.loss_normal(out["normal"], dev(n_ref))[0]),
          float(tracer.loss_depth_normal(cam, out["depth"], dev(n_ref))[0]),
          float(tracer.loss_alpha(out["alpha"])[0])]
    LD, gD = OL.depth_loss(fwd["depth"], d_ref, conf, np.float64(np.float32(1e-6)))
    LN, gN = OL.normal_loss(fwd["normal"], n_ref)
    LDN, gDN = OL.depth_normal_loss(o, d, fwd["depth"], n_ref, h, w)
    LA, gA = OL.coverage_loss(fwd["alpha"])
    # the maps agree with the oracle's off the ambiguous rays, to binary32 rounding of FP64 values
    ok = ~amb
    dg, ng, ag = (out[k].cpu().numpy().astype(np.float64) for k in ("depth", "normal", "alpha"))
    assert np.all(np.abs(dg - fwd["depth"])[ok] <= 1e-6 * np.abs(fwd["depth"][ok]) + 1e-7)
    assert np.all(np.abs(ng - fwd["normal"])[ok] <= 1e-6)
    assert np.all(np.abs(ag - fwd["alpha"])[ok] <= 1e-6)
    # the objectives on the GPU maps equal the reference objectives on those same maps
    mine = (OL.depth_loss(dg, d_ref, conf, np.float64(np.float32(1e-6)))[0], OL.normal_loss(ng, n_ref)[0],
            OL.depth_normal_loss(o, d, dg, n_ref, h, w)[0], OL.coverage_loss(ag)[0])
    for a, b in zip(lg, mine):
        assert abs(a - b) <= 1e-6 * abs(b) + 1e-7, (lg, mine)
    # and those on the oracle's maps differ only through the ambiguous rays
    for a, b in zip(lg, (LD, LN, LDN, LA)):
        assert abs(a - b) <= 2e-3 * abs(b) + 1e-6, (lg, (LD, LN, LDN, LA))

    # backward: same upstream on both sides, ambiguous rays (and their normal-difference neighbourhood) excluded
    bad = amb.reshape(h, w).copy()
    grow = bad.copy()
    for dy in (-2, -1, 0, 1, 2):
        for dx in (-2, -1, 0, 1, 2):
            grow |= np.roll(np.roll(bad, dy, 0), dx, 1)
    keep = ~grow.reshape(-1)
    up_depth = np.where(keep, gD + gDN, 0.0).astype(np.float32)
    up_normal = np.where(keep[:, None], gN, 0.0).astype(np.float32)
    up_alpha = np.where(keep, gA, 0.0).astype(np.float32)
    g_ref = oracle.backward(sa, o, d, ids, p, g_depth=up_depth, g_normal=up_normal, g_alpha=up_alpha)
    g = tracer.render_backward(**args, cameras=[cam], k=wl.k, spp=1, seed=wl.seed, flags=1,
                               d_depth=dev(up_depth), d_normal=dev(up_normal), d_alpha=dev(up_alpha))
    tracer.sync()
    for name in ("mu", "q", "scale", "opacity"):
        grad_check(g[name].cpu().numpy(), g_ref[name], name)
