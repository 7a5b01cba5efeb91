"""Contexts are independent: two contexts on two streams, each with its own
copy of the scene, render and differentiate at the same time, and each
result equals the same call made alone on one context, bit for bit (the
forward always; the backward with LF_FLAG_DETERMINISTIC).  Requires an
MI355X."""
import numpy as np
import pytest

import scenegen
from tests.gpu_common import dev

pytestmark = pytest.mark.gpu


def _upload(wl, st):
    sc = wl.scene
    ts = dict(mu=dev(sc.mu), q=dev(sc.q), scale=dev(sc.scale), opacity=dev(sc.opacity), albedo=dev(sc.albedo),
              roughness=dev(sc.roughness), metallic=dev(sc.metallic))
    M = sc.n_objects
    args = dict(env=dev(st.env), R=dev(st.R.reshape(M, 3, 3)) if M else None, t=dev(st.t.reshape(M, 3)) if M else None)
    return ts, args


def test_two_contexts_on_two_streams_equal_lone_calls():
    import torch
    import paper_2608_29269_amd as lf
    wl = scenegen.make_workload(4, scale=0.02, resolution=48)  # instanced objects, 4 cameras
    st = wl.states[1]
    ts, args = _upload(wl, st)
    cams = st.cameras[:2]
    n = sum(c.w * c.h for c in cams)
    rng = np.random.default_rng(31)
    ups = [dev(rng.standard_normal((n, 3)).astype(np.float32)) for _ in range(2)]
    torch.cuda.synchronize()
    calls = [dict(cameras=cams, k=32, spp=2, seed=5), dict(cameras=cams, k=16, spp=3, seed=8, flags=int(lf.FLAG_NEE))]

    def run(tr, i):
        flags = calls[i].get("flags", 0)
        kw = {key: v for key, v in calls[i].items() if key != "flags"}
        out = tr.render(**args, **kw, flags=flags)
        g = tr.render_backward(**args, **kw, flags=flags | int(lf.FLAG_DETERMINISTIC), d_radiance=ups[i])
        return out, g

    # each call alone, one after the other, on a context of the current stream
    lone = lf.Tracer()
    lone.set_scene(**ts, object_offset=list(wl.scene.object_offset))
    ref = []
    for i in range(2):
        out, g = run(lone, i)
        lone.sync()
        ref.append(({key: v.cpu().numpy() for key, v in out.items()}, {key: v.cpu().numpy() for key, v in g.items()}))
    # both at once on two contexts and two streams
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    trs = [lf.Tracer(stream=s) for s in streams]
    for tr in trs:
        tr.set_scene(**ts, object_offset=list(wl.scene.object_offset))
    torch.cuda.synchronize()
    for rep in range(2):
        res = [run(trs[i], i) for i in range(2)]  # enqueued back to back, no wait in between
        for tr in trs:
            tr.sync()
        torch.cuda.synchronize()
        for i in range(2):
            out, g = res[i]
            for key, v in out.items():
                assert np.array_equal(v.cpu().numpy(), ref[i][0][key]), (rep, i, key)
            for key, v in g.items():
                assert np.array_equal(v.cpu().numpy(), ref[i][1][key]), (rep, i, key)
