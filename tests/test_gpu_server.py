"""Relight server on the GPU: requests served in a mix with others (small
tiles, few slots, so every request spans many batched passes and shares them)
equal, bit for bit, the same request rendered alone by lf_render; one served
request is also checked against the FP64 oracle.  Requires an MI355X."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_common import ambiguous, dev, rel_close, run_oracle, upload_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import paper_2608_29269_amd as lf
    tr = lf.Tracer()
    wl = scenegen.make_workload(4, scale=0.02, resolution=64)  # 10k background + 8 x 400
    upload_scene(tr, wl.scene)
    return tr, wl


def _requests(n, seed, resolutions=((48, 40), (64, 64), (33, 17), (96, 72), (5, 3)), env_hw=((16, 32), (32, 64))):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        R, t = scenegen.random_rigid(rng, 8)
        h, w = env_hw[j % len(env_hw)]
        env = scenegen.lognormal_env(rng, h, w)
        wd, ht = resolutions[j % len(resolutions)]
        cam = scenegen.sphere_camera(rng, wd, ht)
        out.append(scenegen.Request(arrival_s=0.0, R=R, t=t, env=env, camera=cam, spp=(1, 4, 2)[j % 3],
                                    seed=500 + j))
    return out


def _alone(tr, q):
    return tr.render(dev(q.env), R=dev(q.R), t=dev(q.t), cameras=[q.camera], k=32, spp=q.spp, seed=q.seed)


@pytest.mark.parametrize("policy,lanes", [(0, 2), (1, 1), (2, 3)])
def test_served_in_a_mix_equals_rendered_alone(setup, policy, lanes):
    """Several passes run at once (one per lane); a request's tiles land in
    passes on different lanes, after its slot was staged on one of them."""
    import paper_2608_29269_amd as lf
    tr, wl = setup
    reqs = _requests(9, seed=1)
    srv = lf.Server(tr, max_slots=3, tile_rays=256, batch_rays=1024, max_spp=4, policy=policy,
                    max_in_flight=lanes)
    try:
        tickets = [srv.submit(dev(q.env), q.camera, R=dev(q.R), t=dev(q.t), spp=q.spp, seed=q.seed) for q in reqs]
        outs = [srv.wait(t) for t in tickets]
        st = srv.stats()
    finally:
        srv.close()
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["rays_primary"] == sum(q.camera.w * q.camera.h for q in reqs)
    assert st["iterations"] >= sum(q.camera.w * q.camera.h for q in reqs) // 1024
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    for q, got in zip(reqs, outs):
        ref = _alone(tr, q)
        for key in ("radiance", "depth", "normal", "alpha"):
            a, b = got[key].cpu().numpy(), ref[key].cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (key, q.camera.w, q.camera.h, q.spp)


def test_host_buffers_and_budget_limited_admission(setup):
    """Host-resident transforms and env maps are copied on admission; a budget
    that admits one request at a time serialises them without changing results."""
    import paper_2608_29269_amd as lf
    import torch
    tr, wl = setup
    reqs = _requests(4, seed=2, resolutions=((40, 40),), env_hw=((16, 32),))
    for q in reqs:
        q.spp = 4
    # working set of one request (40x40 rays, S = 4, 16x32 env): any two exceed 1.5 of it
    one = 40 * 40 * (32 + 44 * 4) + 16 * 32 * 12 + 8 * (17 + 16 * 33 + 16 * 32 + 2 * 16 + 2)
    srv = lf.Server(tr, max_slots=4, hbm_budget_bytes=int(1.5 * one), tile_rays=128, batch_rays=512, max_spp=4)
    try:
        tickets = [srv.submit(torch.from_numpy(q.env), q.camera, R=torch.from_numpy(q.R), t=torch.from_numpy(q.t),
                              spp=q.spp, seed=q.seed) for q in reqs]
        outs = [srv.wait(t) for t in tickets]
        lat = [srv.latency_ms(t) for t in tickets]
    finally:
        srv.close()
    assert lat == sorted(lat)  # FIFO, one at a time
    for q, got in zip(reqs, outs):
        ref = _alone(tr, q)
        for key in ("radiance", "depth", "normal", "alpha"):
            assert torch.equal(got[key], ref[key]), key


def test_served_request_matches_the_oracle(setup):
    import paper_2608_29269_amd as lf
    tr, wl = setup
    q = _requests(1, seed=3, resolutions=((64, 48),))[0]
    q.spp = 4
    srv = lf.Server(tr, max_slots=2, tile_rays=512, batch_rays=1024, max_spp=4)
    try:
        out = srv.wait(srv.submit(dev(q.env), q.camera, R=dev(q.R), t=dev(q.t), spp=q.spp, seed=q.seed))
    finally:
        srv.close()
    pix = np.arange(0, 64 * 48, 3)
    o, d, ids = oracle.raygen(q.camera, pix)
    st = scenegen.State(R=q.R, t=q.t, env=q.env, cameras=[q.camera])
    ref = run_oracle(wl.scene, st, o, d, ids, 32, q.spp, q.seed, 0)
    amb = ambiguous(ref["margins"])
    assert amb.mean() < 0.01
    ok = ~amb
    for key in ("radiance", "depth", "normal", "alpha"):
        g = out[key].cpu().numpy()[pix]
        assert rel_close(g[ok], ref[key][ok], 1e-4) < 1e-4, key


def test_bad_request_fails_alone_and_errors_are_reported(setup):
    import paper_2608_29269_amd as lf
    tr, wl = setup
    good, bad = _requests(2, seed=4, resolutions=((32, 32),))
    bad.R = np.zeros_like(bad.R)  # degenerate rotation: the instance kernel flags it, nothing faults
    srv = lf.Server(tr, max_slots=4, tile_rays=128, batch_rays=4096, max_spp=4)
    try:
        tb = srv.submit(dev(bad.env), bad.camera, R=dev(bad.R), t=dev(bad.t), spp=1, seed=1)
        tg = srv.submit(dev(good.env), good.camera, R=dev(good.R), t=dev(good.t), spp=good.spp, seed=good.seed)
        with pytest.raises(lf.LFError) as ei:
            srv.wait(tb)
        assert ei.value.status == 1  # LF_EINVAL
        got = srv.wait(tg)
        with pytest.raises(lf.LFError):
            srv.submit(dev(good.env), good.camera, R=dev(good.R), t=dev(good.t), spp=5)  # above max_spp
        with pytest.raises(lf.LFError) as ei:
            tr.refit()  # the scene is being served
        assert ei.value.status == 4  # LF_EBUSY
        assert srv.stats()["rejected"] == 0  # invalid arguments are refused before admission
    finally:
        srv.close()
    tr.refit()  # allowed again once the server is gone
    ref = _alone(tr, good)
    assert np.array_equal(got["radiance"].cpu().numpy(), ref["radiance"].cpu().numpy())


def test_served_with_sobol_samples_equals_rendered_alone(setup):
    """The server takes the Owen-scrambled Sobol sampler (LF_FLAG_SOBOL) from
    its configuration; a request served in a mix still equals, bit for bit,
    the same request rendered alone with that sampler."""
    import paper_2608_29269_amd as lf
    tr, wl = setup
    reqs = _requests(5, seed=3)
    srv = lf.Server(tr, max_slots=2, tile_rays=256, batch_rays=1024, max_spp=4, max_in_flight=2,
                    flags=lf.FLAG_SOBOL)
    try:
        tickets = [srv.submit(dev(q.env), q.camera, R=dev(q.R), t=dev(q.t), spp=q.spp, seed=q.seed) for q in reqs]
        outs = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for q, got in zip(reqs, outs):
        ref = tr.render(dev(q.env), R=dev(q.R), t=dev(q.t), cameras=[q.camera], k=32, spp=q.spp, seed=q.seed,
                        flags=lf.FLAG_SOBOL)
        plain = _alone(tr, q)
        for key in ("radiance", "depth", "normal", "alpha"):
            a, b = got[key].cpu().numpy(), ref[key].cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (key, q.camera.w, q.camera.h, q.spp)
        if q.spp > 1:  # the sampler is in effect
            assert not np.array_equal(got["radiance"].cpu().numpy(), plain["radiance"].cpu().numpy())


@pytest.mark.parametrize("lanes", [1, 3])
def test_lone_whole_requests_equal_rendered_alone(setup, lanes):
    """A pass that holds one whole request runs the single-request kernels
    with the request's slot data; served one at a time (each its own pass),
    every request equals lf_render of it bit for bit, also with several lanes
    staging and running in turn."""
    import paper_2608_29269_amd as lf
    tr, wl = setup
    reqs = _requests(6, seed=7)
    srv = lf.Server(tr, max_slots=2, tile_rays=65536, batch_rays=1 << 20, max_spp=4, policy=1, max_in_flight=lanes)
    outs = []
    try:
        for q in reqs:
            outs.append(srv.wait(srv.submit(dev(q.env), q.camera, R=dev(q.R), t=dev(q.t), spp=q.spp, seed=q.seed)))
        st = srv.stats()
    finally:
        srv.close()
    assert st["completed"] == len(reqs) and st["iterations"] == len(reqs)
    for q, got in zip(reqs, outs):
        ref = _alone(tr, q)
        for key in ("radiance", "depth", "normal", "alpha"):
            a, b = got[key].cpu().numpy(), ref[key].cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (key, q.camera.w, q.camera.h, q.spp)


@pytest.mark.parametrize("k", [6, 12, 48])
def test_served_at_other_k_buckets_equals_rendered_alone(setup, k):
    """The batched kernels at the other k-buffer instantiations (8, 16 and 64
    slots: k = 6, 12 and 48 leave sentinel slots in front), in a mix of
    requests that share passes, equal lf_render of each request at the same k,
    bit for bit."""
    import paper_2608_29269_amd as lf
    tr, wl = setup
    reqs = _requests(5, seed=20 + k)
    srv = lf.Server(tr, max_slots=3, tile_rays=256, batch_rays=1024, max_spp=4, policy=1, max_in_flight=2, k=k)
    try:
        tickets = [srv.submit(dev(q.env), q.camera, R=dev(q.R), t=dev(q.t), spp=q.spp, seed=q.seed) for q in reqs]
        outs = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for q, got in zip(reqs, outs):
        ref = tr.render(dev(q.env), R=dev(q.R), t=dev(q.t), cameras=[q.camera], k=k, spp=q.spp, seed=q.seed)
        for key in ("radiance", "depth", "normal", "alpha"):
            a, b = got[key].cpu().numpy(), ref[key].cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (key, k, q.camera.w, q.camera.h, q.spp)
