"""Pins of the oracle's hand-written adjoint (path replay, Sec. 3.3 PRB
paragraph; geometry gradients through the compositing rules, Sec. 3.2)
against closed forms, exact linearity in the environment map, and central
finite differences of the frozen objective in FP64.  CPU only."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.helpers import make_scene, no_transforms, rays_single

P = oracle.Params
GROUPS = ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic")


def test_single_surfel_closed_form_gradients():
    su, sv, a = 0.2, 0.3, 0.6
    sc = make_scene([[0, 0, 0]], scale=[[su, sv]], opacity=[a])
    su, sv, a = (float(np.float32(v)) for v in (su, sv, a))
    x0, y0 = 0.07, -0.11
    o, d, ids = rays_single([x0, y0, 2], [0, 0, -1])
    R, t = no_transforms(sc)
    sa = oracle.SceneArrays(sc, R, t, scenegen.constant_env(1.0, 8, 16))
    p = P(k=4, spp=1, seed=3, flags=oracle.NO_SECONDARY)
    g = oracle.backward(sa, o, d, ids, p, g_alpha=np.ones(1))
    xu, xv = x0 / su, y0 / sv
    e = np.exp(-0.5 * (xu ** 2 + xv ** 2))
    assert g["opacity"][0] == pytest.approx(e, rel=1e-13)  # dA/dalpha
    assert g["scale"][0, 0] == pytest.approx(a * e * xu ** 2 / su, rel=1e-12)  # dA/ds_u
    assert g["scale"][0, 1] == pytest.approx(a * e * xv ** 2 / sv, rel=1e-12)
    # moving the centre by +dx along x moves the local coordinate by -dx/su
    assert g["mu"][0, 0] == pytest.approx(a * e * xu / su, rel=1e-12)
    assert g["mu"][0, 1] == pytest.approx(a * e * xv / sv, rel=1e-12)
    assert g["mu"][0, 2] == pytest.approx(0.0, abs=1e-14)  # a plane shift along the ray changes nothing
    # capped surfel: no opacity gradient
    sc2 = make_scene([[0, 0, 0]], scale=[[su, sv]], opacity=[1.0])
    sa2 = oracle.SceneArrays(sc2, R, t, scenegen.constant_env(1.0, 8, 16))
    g2 = oracle.backward(sa2, *rays_single([0, 0, 2], [0, 0, -1]), p, g_alpha=np.ones(1))
    assert g2["opacity"][0] == 0.0 and np.all(g2["scale"][0] == 0.0)


def _setup(which, scale, res, spp, flags=0, seed=77):
    wl = scenegen.make_workload(which, scale=scale, resolution=res)
    st = wl.states[0]
    o, d, ids = oracle.raygen(st.cameras[0])
    env = st.env
    if env.shape[0] > 32:  # coarse env keeps the FD test cheap; same recipe
        env = scenegen.lognormal_env(np.random.default_rng(seed), 16, 32)
    p = P(k=wl.k, spp=spp, seed=seed, flags=flags)
    return wl, st, env, o, d, ids, p


def _objective(out, up):
    return sum(float((out[k] * up[k]).sum()) for k in up)


def _theta(wl, env):
    sc = wl.scene
    return {"mu": sc.mu.astype(np.float64), "q": sc.q.astype(np.float64), "scale": sc.scale.astype(np.float64),
            "opacity": sc.opacity.astype(np.float64), "albedo": sc.albedo.astype(np.float64),
            "roughness": sc.roughness.astype(np.float64), "metallic": sc.metallic.astype(np.float64),
            "env": env.astype(np.float64)}


@pytest.mark.parametrize("which,scale,res,spp,flags", [
    (2, 0.02, 16, 2, 0),                       # surface-like, one bounce
    (1, 0.5, 16, 2, oracle.NO_SECONDARY),      # volume, primary-only shading
    (4, 0.005, 16, 2, 0),                      # background + 8 rigidly moved objects
])
def test_adjoint_matches_central_fd_of_frozen_objective(which, scale, res, spp, flags):
    wl, st, env, o, d, ids, p = _setup(which, scale, res, spp, flags)
    rng = np.random.default_rng(which)
    n = len(ids)
    up = {"radiance": rng.standard_normal((n, 3)), "depth": rng.standard_normal(n),
          "normal": rng.standard_normal((n, 3)), "alpha": rng.standard_normal(n)}
    sa0 = oracle.SceneArrays(wl.scene, st.R, st.t, env)
    g = oracle.backward(sa0, o, d, ids, p, g_radiance=up["radiance"], g_depth=up["depth"],
                        g_normal=up["normal"], g_alpha=up["alpha"])
    th0 = _theta(wl, env)
    for grp in GROUPS + ("env",):
        for trial in range(2):
            v = rng.standard_normal(th0[grp].shape)
            h = 1e-6 * max(1.0, float(np.abs(th0[grp]).max()))
            vals = {}
            for sgn in (+2, +1, -1, -2):
                ov = dict(th0)
                ov[grp] = th0[grp] + sgn * h * v
                sa = oracle.SceneArrays(wl.scene, st.R, st.t, env, overrides=ov)
                vals[sgn] = _objective(oracle.frozen_eval(sa0, sa, o, d, ids, p), up)
            # fourth-order central difference: small surfels make the objective
            # sharply curved, so the plain central difference carries O(h^2) bias
            fd = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
            ad = float((g[grp] * v).sum())
            assert abs(fd - ad) <= 1e-6 * max(abs(ad), 1e-3 * abs(vals[1])), (grp, fd, ad)


def test_env_gradient_is_exact_by_linearity():
    wl, st, env, o, d, ids, p = _setup(2, 0.02, 12, 2)
    rng = np.random.default_rng(1)
    n = len(ids)
    gL = rng.standard_normal((n, 3))
    sa0 = oracle.SceneArrays(wl.scene, st.R, st.t, env)
    g = oracle.backward(sa0, o, d, ids, p, g_radiance=gL)
    V = rng.standard_normal(env.shape)
    base = oracle.frozen_eval(sa0, sa0, o, d, ids, p)["radiance"]
    ov = _theta(wl, env)
    ov["env"] = env.astype(np.float64) + V
    plus = oracle.frozen_eval(sa0, oracle.SceneArrays(wl.scene, st.R, st.t, env, overrides=ov), o, d, ids, p)
    lhs = float(((plus["radiance"] - base) * gL).sum())
    assert lhs == pytest.approx(float((g["env"] * V).sum()), rel=1e-10)


def test_frozen_eval_equals_render_at_theta0():
    wl, st, env, o, d, ids, p = _setup(2, 0.02, 12, 2)
    sa0 = oracle.SceneArrays(wl.scene, st.R, st.t, env)
    a = oracle.render(sa0, o, d, ids, p, lists=False)
    b = oracle.frozen_eval(sa0, oracle.SceneArrays(wl.scene, st.R, st.t, env), o, d, ids, p)
    for k in ("radiance", "depth", "normal", "alpha"):
        assert np.array_equal(a[k], b[k])


def test_gradients_are_overwritten_not_accumulated():
    wl, st, env, o, d, ids, p = _setup(1, 0.25, 8, 1, oracle.NO_SECONDARY)
    sa0 = oracle.SceneArrays(wl.scene, st.R, st.t, env)
    up = np.ones((len(ids), 3))
    g1 = oracle.backward(sa0, o, d, ids, p, g_radiance=up)
    g2 = oracle.backward(sa0, o, d, ids, p, g_radiance=up)
    for k in GROUPS:
        np.testing.assert_allclose(g1[k], g2[k], rtol=1e-12, atol=1e-15)
