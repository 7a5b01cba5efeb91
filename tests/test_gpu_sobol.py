"""GPU parity of the Owen-scrambled Sobol sampler (LF_FLAG_SOBOL; Sec. 3.3 PRB
paragraph) against the FP64 oracle: the samplers must agree bit for bit,
which shows as identical sampled directions, hence identical secondary hit
lists, in both estimator forms, and as matching replayed gradients.
Requires an MI355X."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_common import grad_check, ambiguous, dev, rel_close, run_oracle, state_args, upload_scene

pytestmark = pytest.mark.gpu

RTOL = 1e-4
SOBOL = oracle.SOBOL


@pytest.fixture(scope="module")
def tracer():
    import paper_2608_29269_amd as lf
    return lf.Tracer()


@pytest.fixture(scope="module")
def c2_small():
    return scenegen.make_workload(2, scale=0.1, resolution=96)  # 20k surfels, 96x96


@pytest.mark.parametrize("spp,flags", [(4, SOBOL), (2, SOBOL | oracle.NEE), (8, SOBOL | oracle.NO_SECONDARY)])
def test_c2_sobol_parity(tracer, c2_small, spp, flags):
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cam = st.cameras[0]
    out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=32, spp=spp, seed=wl.seed, flags=flags,
                        hit_idx=True, sec_hit_idx=True)
    pix = np.arange(0, cam.w * cam.h, 5)
    o, d, ids = oracle.raygen(cam, pix)
    ref = run_oracle(wl.scene, st, o, d, ids, 32, spp, wl.seed, flags)
    amb = ambiguous(ref["margins"], include_secondary=not flags & oracle.NO_SECONDARY)
    g = {k: v.cpu().numpy()[pix] for k, v in out.items()}
    ok = ~amb
    assert ok.mean() >= 0.99
    np.testing.assert_array_equal(g["hit_idx"][ok], ref["hit_idx"][ok])
    np.testing.assert_array_equal(g["sec_hit_idx"][ok], ref["sec_hit_idx"][ok])
    for key in ("radiance", "depth", "normal", "alpha"):
        e = rel_close(g[key][ok], ref[key][ok], RTOL)
        assert e < RTOL, (key, e)
    if not flags & oracle.NO_SECONDARY:
        h = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=32, spp=spp, seed=wl.seed,
                          flags=flags & ~SOBOL, sec_hit_idx=True)
        assert not np.array_equal(h["sec_hit_idx"].cpu().numpy(), out["sec_hit_idx"].cpu().numpy())


def test_sobol_adjoint_matches_oracle(tracer):
    wl = scenegen.make_workload(3, scale=0.02, resolution=40)
    st = wl.states[0]
    env = scenegen.lognormal_env(np.random.default_rng(5), 32, 64)
    st = scenegen.State(R=st.R, t=st.t, env=env, cameras=st.cameras)
    cam = st.cameras[0]
    o, d, ids = oracle.raygen(cam)
    n = len(ids)
    flags = SOBOL | oracle.NEE
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    p = oracle.Params(k=wl.k, spp=4, seed=wl.seed, flags=flags)
    amb = ambiguous(oracle.render(sa, o, d, ids, p, lists=False)["margins"])
    rng = np.random.default_rng(3)
    up = rng.standard_normal((n, 3))
    up[amb] = 0.0
    up = up.astype(np.float32)
    g_ref = oracle.backward(sa, o, d, ids, p, g_radiance=up)
    upload_scene(tracer, wl.scene)
    g = tracer.render_backward(**state_args(tracer, wl.scene, st), cameras=[cam], k=wl.k, spp=4, seed=wl.seed,
                               flags=flags, d_radiance=dev(up))
    tracer.sync()
    for name in ("mu", "q", "scale", "opacity", "albedo", "roughness", "metallic", "env"):
        grad_check(g[name].cpu().numpy(), g_ref[name], name, nonzero=True)
