"""GPU parity of the path-replay adjoint against the oracle's FP64 adjoint
(Sec. 3.3 PRB paragraph; geometry gradients through compositing, Sec. 3.2),
through the C ABI.  Requires an MI355X."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_common import grad_check, ambiguous, dev, state_args, upload_scene

pytestmark = pytest.mark.gpu

GROUPS = ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic", "env")
TOL = 1e-3


@pytest.fixture(scope="module")
def tracer():
    import paper_2608_29269_amd as lf
    return lf.Tracer()


def _grad_check(g_gpu, g_ref, name):
    grad_check(g_gpu, g_ref, name)


CASES = [
    (3, 0.02, 40, 1, 0, None),    # surface-like training step (6k surfels)
    (1, 1.0, 32, 2, 1, None),     # volume, primary-only shading
    (4, 0.01, 32, 2, 0, None),    # instanced objects, one bounce
    (3, 0.02, 40, 2, 0, 8),       # the k-buffer instantiations below and above 32
    (3, 0.02, 40, 2, 0, 64),
]


def _adjoint_case(which, scale, res, spp, flags, k):
    """A small workload, a random upstream gradient (zero on legitimately
    ambiguous rays, on both sides) and the oracle's FP64 adjoint."""
    wl = scenegen.make_workload(which, scale=scale, resolution=res)
    if k is not None:
        wl.k = k
    st = wl.states[0]
    env = st.env if st.env.shape[0] <= 64 else scenegen.lognormal_env(np.random.default_rng(5), 32, 64)
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
    for key in up:
        up[key][amb] = 0.0
        up[key] = up[key].astype(np.float32)
    g_ref = oracle.backward(sa, o, d, ids, p, g_radiance=up["radiance"], g_depth=up["depth"],
                            g_normal=up["normal"], g_alpha=up["alpha"])
    return wl, st, cam, up, g_ref


def _gpu_adjoint(tracer, wl, st, cam, up, spp, flags):
    g = tracer.render_backward(**state_args(tracer, wl.scene, st), cameras=[cam], k=wl.k, spp=spp, seed=wl.seed,
                               flags=flags, d_radiance=dev(up["radiance"]), d_depth=dev(up["depth"]),
                               d_normal=dev(up["normal"]), d_alpha=dev(up["alpha"]))
    tracer.sync()
    return {key: v.cpu().numpy() for key, v in g.items()}


@pytest.mark.parametrize("which,scale,res,spp,flags,k", CASES)
def test_adjoint_matches_oracle(tracer, which, scale, res, spp, flags, k):
    wl, st, cam, up, g_ref = _adjoint_case(which, scale, res, spp, flags, k)
    upload_scene(tracer, wl.scene)
    g = _gpu_adjoint(tracer, wl, st, cam, up, spp, flags)
    for name in GROUPS:
        _grad_check(g[name], g_ref[name], name)


@pytest.mark.parametrize("which,scale,res,spp,flags,k", CASES)
def test_deterministic_adjoint_matches_oracle_and_repeats_bitwise(tracer, which, scale, res, spp, flags, k):
    """With LF_FLAG_DETERMINISTIC every gradient is a binary64 sum in a fixed
    order rounded once: within 1e-3 of the oracle element by element, and
    bitwise the same on a second run (and after an atomic-path run in
    between, which leaves no state behind)."""
    import paper_2608_29269_amd as lf
    wl, st, cam, up, g_ref = _adjoint_case(which, scale, res, spp, flags, k)
    upload_scene(tracer, wl.scene)
    det = flags | lf.FLAG_DETERMINISTIC
    g1 = _gpu_adjoint(tracer, wl, st, cam, up, spp, det)
    for name in GROUPS:
        _grad_check(g1[name], g_ref[name], name)
    ga = _gpu_adjoint(tracer, wl, st, cam, up, spp, flags)
    g2 = _gpu_adjoint(tracer, wl, st, cam, up, spp, det)
    for name in GROUPS:
        assert np.array_equal(g1[name].view(np.uint32), g2[name].view(np.uint32)), name
        # the float-atomic path sums the same contributions in another order
        grad_check(ga[name], g1[name], name)


def torch_equal(x, y):
    """Bitwise equality of two float32 tensors."""
    import torch
    return bool(torch.equal(x.reshape(-1).view(torch.int32), y.reshape(-1).view(torch.int32)))


def test_gradients_overwrite(tracer):
    wl = scenegen.make_workload(1, scale=0.5, resolution=16)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    n = 256
    up = dev(np.ones((n, 3), np.float32))
    g1 = tracer.render_backward(**args, cameras=st.cameras, k=16, spp=1, seed=1, flags=1, d_radiance=up)
    a = {k: v.clone() for k, v in g1.items()}
    g2 = tracer.render_backward(**args, cameras=st.cameras, k=16, spp=1, seed=1, flags=1, d_radiance=up,
                                grads=g1)
    for k in a:
        np.testing.assert_allclose(g2[k].cpu().numpy(), a[k].cpu().numpy(), rtol=1e-5, atol=1e-6)
    # order-fixed sums: the overwritten gradients are bitwise those of a fresh call
    import paper_2608_29269_amd as lf
    g3 = tracer.render_backward(**args, cameras=st.cameras, k=16, spp=1, seed=1, flags=1 | lf.FLAG_DETERMINISTIC,
                                d_radiance=up)
    b = {k: v.clone() for k, v in g3.items()}
    g4 = tracer.render_backward(**args, cameras=st.cameras, k=16, spp=1, seed=1, flags=1 | lf.FLAG_DETERMINISTIC,
                                d_radiance=up, grads=g3)
    for k in b:
        assert torch_equal(g4[k], b[k]), k


def test_autograd_function_and_l1(tracer):
    import torch
    import paper_2608_29269_amd as lf
    wl = scenegen.make_workload(3, scale=0.01, resolution=24)
    st = wl.states[0]
    env_np = scenegen.lognormal_env(np.random.default_rng(2), 16, 32)
    ts = upload_scene(tracer, wl.scene)
    env = dev(env_np).requires_grad_(True)
    params = {k: v.requires_grad_(True) for k, v in ts.items()}
    cfg = dict(cameras=[st.cameras[0]], k=32, spp=1, seed=3)
    rad, depth, normal, alpha = lf.RenderFn.apply(tracer, cfg, params["mu"], params["q"], params["scale"],
                                                  params["opacity"], params["albedo"], params["roughness"],
                                                  params["metallic"], env)
    target = torch.zeros_like(rad)
    loss, g_l1 = tracer.l1_loss(rad.detach(), target)
    assert abs(float(loss) - float(rad.detach().abs().mean())) <= 1e-5 * float(loss)
    rad.backward(g_l1)
    assert params["albedo"].grad is not None and torch.isfinite(params["albedo"].grad).all()
    assert env.grad is not None and float(env.grad.abs().sum()) > 0


@pytest.mark.parametrize("k,extra", [(32, 0), (12, 0), (64, 0), (32, "nee_sobol")])
def test_replay_from_the_forward_k_th_distances_is_exact(tracer, k, extra):
    """The replay of a backward that follows a forward with the same
    arguments starts each ray from the k-th distance the forward found (a
    culling bound; a ray with fewer than k hits below it is traced again
    without it).  Its gradients equal, bit for bit, those of a backward that
    has no forward before it, with order-fixed sums; also when the
    environment was changed in place in between, so that the secondary rays
    differ and the bounds are wrong for many of them.  Also at k-buffer
    buckets whose first slots hold -inf sentinels (k = 12 of 16), at k = 64,
    and for the two-ray estimator with Sobol samples (two slots per sample)."""
    import paper_2608_29269_amd as lf
    wl = scenegen.make_workload(2, scale=0.1, resolution=96)  # 20k surface surfels
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    cam = st.cameras[0]
    n = cam.w * cam.h
    up = dev(np.random.default_rng(3).standard_normal((n, 3)).astype(np.float32))
    fl = (lf.FLAG_NEE | lf.FLAG_SOBOL) if extra == "nee_sobol" else 0
    cfg = dict(cameras=[cam], k=k, spp=2, seed=5)
    det = lf.FLAG_DETERMINISTIC | lf.FLAG_COUNT | fl

    def fresh_backward():
        tracer.refit()  # a new scene generation: nothing carried over
        g = tracer.render_backward(**args, **cfg, flags=det, d_radiance=up)
        return {k: v.clone() for k, v in g.items()}

    g_ref = fresh_backward()
    tracer.trace_counters()
    tracer.render(**args, **cfg, flags=lf.FLAG_COUNT | fl)
    g = tracer.render_backward(**args, **cfg, flags=det, d_radiance=up)
    cnt = tracer.trace_counters()
    # only rays whose forward filled all k slots carry a finite bound (at
    # k = 64 few secondary rays of this scene have that many hits)
    assert 0 < cnt["primary"]["hinted"] <= n, cnt
    assert k > 32 or cnt["secondary"]["hinted"] > 0, cnt
    for key in g_ref:
        assert torch_equal(g[key], g_ref[key]), key
    # stale bounds: the map changes in place between forward and backward
    tracer.render(**args, **cfg, flags=fl)
    args["env"].mul_(1.7).add_(0.3 * dev(np.random.default_rng(4).random(st.env.shape).astype(np.float32)))
    g_ref2 = fresh_backward()
    tracer.render(**args, **cfg, flags=fl)
    args["env"].mul_(1.0)  # same pointer, same contents
    g2 = tracer.render_backward(**args, **cfg, flags=det, d_radiance=up)
    for key in g_ref2:
        assert torch_equal(g2[key], g_ref2[key]), key
    tracer.render(**args, **cfg, flags=fl)
    args["env"].pow_(1.5)  # same pointer, new contents: the importance sampling and the secondary rays change
    tracer.trace_counters()
    g3 = tracer.render_backward(**args, **cfg, flags=det, d_radiance=up)
    cnt = tracer.trace_counters()
    assert k > 32 or cnt["secondary"]["hint_retries"] > 0, cnt  # wrong bounds are caught and retraced
    g_ref3 = fresh_backward()
    for key in g_ref3:
        assert torch_equal(g3[key], g_ref3[key]), key


@pytest.mark.parametrize("flags_name", ["nee_sobol", "no_background"])
def test_adjoint_with_explicit_rays_matches_oracle(tracer, flags_name):
    """The inverse-rendering loop's form: explicit rays of a random pixel
    subset (ray ids are positions in the batch), with the two-ray estimator
    and Sobol samples; and the one-ray form without the background term.
    All eight gradient groups against the oracle's FP64 adjoint."""
    import paper_2608_29269_amd as lf
    wl = scenegen.make_workload(3, scale=0.02, resolution=40)
    st = wl.states[0]
    env = scenegen.lognormal_env(np.random.default_rng(5), 32, 64)
    st = scenegen.State(R=st.R, t=st.t, env=env, cameras=st.cameras)
    o, d, _ = oracle.raygen(st.cameras[0])
    rng = np.random.default_rng(17)
    pick = np.sort(rng.choice(len(o), 700, replace=False))
    o2, d2 = np.ascontiguousarray(o[pick]), np.ascontiguousarray(d[pick])
    ids = np.arange(len(pick))
    flags = (lf.FLAG_NEE | lf.FLAG_SOBOL) if flags_name == "nee_sobol" else lf.FLAG_NO_BACKGROUND
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    p = oracle.Params(k=wl.k, spp=2, seed=9, flags=flags)
    fwd = oracle.render(sa, o2, d2, ids, p, lists=False)
    amb = ambiguous(fwd["margins"])
    n = len(ids)
    up = dict(radiance=rng.standard_normal((n, 3)), alpha=rng.standard_normal(n))
    for key in up:
        up[key][amb] = 0.0
        up[key] = up[key].astype(np.float32)
    g_ref = oracle.backward(sa, o2, d2, ids, p, g_radiance=up["radiance"], g_alpha=up["alpha"])
    upload_scene(tracer, wl.scene)
    g = tracer.render_backward(**state_args(tracer, wl.scene, st), rays=(dev(o2), dev(d2)), k=wl.k, spp=2, seed=9,
                               flags=flags, d_radiance=dev(up["radiance"]), d_alpha=dev(up["alpha"]))
    tracer.sync()
    for name in GROUPS:
        grad_check(g[name].cpu().numpy(), g_ref[name], name)


@pytest.mark.parametrize("det", [False, True])
def test_adjoint_on_degenerate_surfels_matches_oracle(tracer, det):
    """The replayed adjoint on the degenerate-surfel scene (opacity below
    alpha_min, unnormalised quaternion, needle, edge-on, on-plane origins,
    huge, opaque, identical pair), with and without LF_FLAG_DETERMINISTIC:
    all eight gradient groups against the oracle's FP64 adjoint.  Surfels no
    ray hits get exact zeros."""
    import paper_2608_29269_amd as lf
    from tests.helpers import degenerate_scene, degenerate_rays
    sc = degenerate_scene()
    o, d = degenerate_rays()
    env = scenegen.lognormal_env(np.random.default_rng(7), 16, 32)
    st = scenegen.State(R=np.zeros((0, 3, 3), np.float32), t=np.zeros((0, 3), np.float32), env=env, cameras=[])
    ids = np.arange(len(o))
    sa = oracle.SceneArrays(sc, st.R, st.t, st.env)
    p = oracle.Params(k=16, spp=2, seed=3, flags=0)
    fwd = oracle.render(sa, o, d, ids, p, lists=False)
    amb = ambiguous(fwd["margins"])
    n = len(o)
    rng = np.random.default_rng(23)
    up = dict(radiance=rng.standard_normal((n, 3)), depth=rng.standard_normal(n), normal=rng.standard_normal((n, 3)),
              alpha=rng.standard_normal(n))
    for key in up:
        up[key][amb] = 0.0
        up[key] = up[key].astype(np.float32)
    g_ref = oracle.backward(sa, o, d, ids, p, g_radiance=up["radiance"], g_depth=up["depth"], g_normal=up["normal"],
                            g_alpha=up["alpha"])
    upload_scene(tracer, sc)
    g = tracer.render_backward(env=dev(env), rays=(dev(o), dev(d)), k=16, spp=2, seed=3,
                               flags=lf.FLAG_DETERMINISTIC if det else 0, d_radiance=dev(up["radiance"]),
                               d_depth=dev(up["depth"]), d_normal=dev(up["normal"]), d_alpha=dev(up["alpha"]))
    tracer.sync()
    g = {key: v.cpu().numpy() for key, v in g.items()}
    for name in GROUPS:
        _grad_check(g[name], g_ref[name], name)
    for i in (0, 2, 3):  # never hit
        for name in ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic"):
            assert not np.any(g[name][i]), (name, i)
    assert np.any(g["mu"][1]) and np.any(g["albedo"][7]) and np.any(g["albedo"][8])
