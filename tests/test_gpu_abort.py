"""Failure detection of the persistent traversal pools: the host's abort
word (lf_abort) and the watchdog of lf_sync_timeout, through the C ABI.
Each condition is raised from the host, so every kernel still exits
normally.  Requires an MI355X."""
import time

import numpy as np
import pytest

import scenegen
from tests.gpu_common import state_args, upload_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tracer():
    import paper_2608_29269_amd as lf
    return lf.Tracer()


def _status(exc):
    return exc.value.status


def _outputs(out):
    return {k: v.cpu().numpy().copy() for k, v in out.items()}


def test_abort_before_a_render_cuts_it_short_and_the_next_render_is_whole(tracer):
    import paper_2608_29269_amd as lf
    from paper_2608_29269_amd import _lib
    wl = scenegen.make_workload(2, scale=0.05, resolution=64)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    cfg = dict(cameras=st.cameras, k=32, spp=2, seed=3)
    ref = _outputs(tracer.render(**args, **cfg))
    tracer.sync()
    tracer.abort()
    tracer.render(**args, **cfg)
    with pytest.raises(lf.LFError) as e:
        tracer.sync()
    assert _status(e) == _lib.LF_EABORTED
    # the request is cleared once the stream drained: the next render is whole
    again = _outputs(tracer.render(**args, **cfg))
    tracer.sync()
    for k in ref:
        assert np.array_equal(ref[k], again[k]), k
    # an abort with nothing enqueued affects nothing
    tracer.abort()
    tracer.sync()
    again = _outputs(tracer.render(**args, **cfg))
    tracer.sync()
    for k in ref:
        assert np.array_equal(ref[k], again[k]), k


def test_aborted_backward_drains_and_the_next_one_is_exact(tracer):
    import paper_2608_29269_amd as lf
    from paper_2608_29269_amd import _lib
    from tests.gpu_common import dev
    wl = scenegen.make_workload(2, scale=0.05, resolution=64)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    n = st.cameras[0].w * st.cameras[0].h
    up = dev(np.random.default_rng(1).standard_normal((n, 3)).astype(np.float32))
    cfg = dict(cameras=st.cameras, k=32, spp=2, seed=3, flags=lf.FLAG_DETERMINISTIC)
    ref = {k: v.clone() for k, v in tracer.render_backward(**args, **cfg, d_radiance=up).items()}
    tracer.sync()
    tracer.abort()
    tracer.render_backward(**args, **cfg, d_radiance=up)
    with pytest.raises(lf.LFError) as e:
        tracer.sync()
    assert _status(e) == _lib.LF_EABORTED
    g = tracer.render_backward(**args, **cfg, d_radiance=up)
    tracer.sync()
    for k in ref:
        assert np.array_equal(ref[k].cpu().numpy(), g[k].cpu().numpy()), k


def test_watchdog_cuts_a_long_render_short(tracer):
    """A 1M-surfel 1024x1024 S=4 render takes tens of milliseconds; a zero
    timeout fires at the first poll, the traversal drains without further
    work, and the context is usable afterwards."""
    import paper_2608_29269_amd as lf
    from paper_2608_29269_amd import _lib
    wl = scenegen.make_workload(5)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    cfg = dict(cameras=st.cameras, k=32, spp=4, seed=wl.seed)
    tracer.render(**args, **cfg)
    tracer.sync()
    t0 = time.perf_counter()
    tracer.render(**args, **cfg)
    tracer.sync()
    whole = time.perf_counter() - t0
    t0 = time.perf_counter()
    tracer.render(**args, **cfg)
    with pytest.raises(lf.LFError) as e:
        tracer.sync(timeout_ms=0.0)
    cut = time.perf_counter() - t0
    assert _status(e) == _lib.LF_ETIMEOUT
    assert cut < 0.5 * whole, (cut, whole)  # the traversal was cut short, not waited for
    # a generous timeout lets the same render complete, bitwise as without one
    a = _outputs(tracer.render(**args, **cfg))
    tracer.sync(timeout_ms=60000.0)
    b = _outputs(tracer.render(**args, **cfg))
    tracer.sync()
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_watchdog_arguments_and_an_idle_stream(tracer):
    """A negative timeout is an argument error (nothing waits, nothing is
    cut short); an idle stream passes the watchdog at once, also with the
    abort word raised (it is cleared, as lf_sync clears it)."""
    import paper_2608_29269_amd as lf
    from paper_2608_29269_amd import _lib
    with pytest.raises(lf.LFError) as e:
        tracer.sync(timeout_ms=-1.0)
    assert _status(e) == _lib.LF_EINVAL
    tracer.sync(timeout_ms=0.0)
    tracer.abort()
    tracer.sync(timeout_ms=1000.0)
    wl = scenegen.make_workload(1, scale=0.25, resolution=16)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    a = _outputs(tracer.render(**args, cameras=st.cameras, k=16, spp=1, seed=2, flags=1))
    tracer.sync(timeout_ms=60000.0)
    b = _outputs(tracer.render(**args, cameras=st.cameras, k=16, spp=1, seed=2, flags=1))
    tracer.sync()
    for k in a:
        assert np.array_equal(a[k], b[k]), k
