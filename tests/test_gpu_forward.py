"""GPU parity of the forward path (raygen, traversal, k-closest hit lists,
compositing, one-bounce shading) against the FP64 oracle, element by element,
through the C ABI.  Requires an MI355X."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.gpu_common import ambiguous, dev, rel_close, run_oracle, state_args, upload_scene

pytestmark = pytest.mark.gpu

RTOL = 1e-4  # radiance/depth/normal/alpha, relative with floor 1e-3 * mean|ref|


@pytest.fixture(scope="module")
def tracer():
    import paper_2608_29269_amd as lf
    return lf.Tracer()


def _compare(out, ref, amb, check_sec=False, spp=1, min_ok=0.99):
    T = out["radiance"].device
    g = {k: v.cpu().numpy() for k, v in out.items()}
    ok = ~amb
    assert ok.mean() >= min_ok, f"ambiguous fraction {amb.mean():.4f}"
    np.testing.assert_array_equal(g["hit_idx"][ok], ref["hit_idx"][ok])
    if check_sec:
        np.testing.assert_array_equal(g["sec_hit_idx"][ok], ref["sec_hit_idx"][ok])
    for key in ("radiance", "depth", "normal", "alpha"):
        e = rel_close(g[key][ok], ref[key][ok], RTOL)
        assert e < RTOL, (key, e)


def test_raygen_is_bitwise_identical(tracer):
    rng = np.random.default_rng(0)
    for w, h, fov in ((64, 64, 60.0), (37, 23, 50.0), (800, 800, 60.0), (1024, 1024, 60.0), (5, 300, 110.0)):
        cam = scenegen.sphere_camera(rng, w, h, fov_y_deg=fov)
        o, d = tracer.raygen(cam)
        ro, rd, _ = oracle.raygen(cam)
        assert np.array_equal(o.cpu().numpy().view(np.uint32), ro.view(np.uint32))
        assert np.array_equal(d.cpu().numpy().view(np.uint32), rd.view(np.uint32)), (w, h)


def test_c1_primary_only_full(tracer):
    wl = scenegen.make_workload(1)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cam = st.cameras[0]
    out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=wl.k, spp=wl.spp, seed=wl.seed,
                        flags=1, hit_idx=True)
    o, d, ids = oracle.raygen(cam)
    ref = run_oracle(wl.scene, st, o, d, ids, wl.k, wl.spp, wl.seed, 1)
    amb = ambiguous(ref["margins"], include_secondary=False)
    assert amb.sum() == 0
    _compare(out, ref, amb)


@pytest.mark.parametrize("k", [1, 5, 16, 40, 64])
def test_k_buckets_and_explicit_rays(tracer, k):
    wl = scenegen.make_workload(1)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    o, d, ids = oracle.raygen(st.cameras[0], np.arange(0, 4096, 3))  # 1366 rays: ragged last block
    out = tracer.render(**state_args(tracer, wl.scene, st), rays=(dev(o), dev(d)), k=k, spp=2, seed=3,
                        flags=1, hit_idx=True)
    ref = run_oracle(wl.scene, st, o, d, np.arange(len(o)), k, 2, 3, 1)
    _compare(out, ref, ambiguous(ref["margins"], False))


@pytest.fixture(scope="module")
def c2_small():
    return scenegen.make_workload(2, scale=0.1, resolution=96)  # 20k surfels, 96x96


def test_bvh_traversal_equals_brute_force(tracer, c2_small):
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    a = tracer.render(**state_args(tracer, wl.scene, st), cameras=st.cameras, k=32, spp=2, seed=9, hit_idx=True,
                      sec_hit_idx=True)
    b = tracer.render(**state_args(tracer, wl.scene, st), cameras=st.cameras, k=32, spp=2, seed=9, hit_idx=True,
                      sec_hit_idx=True, flags=16)
    for key in a:
        assert np.array_equal(a[key].cpu().numpy(), b[key].cpu().numpy()), key


@pytest.mark.parametrize("scene,w,h", [("c2_small", 512, 512), ("instanced", 512, 512), ("c2_small", 601, 433)])
def test_wave_packet_and_per_lane_traversals_agree(tracer, c2_small, scene, w, h):
    """Large camera launches are traced as wave packets (one node sequence
    per 8x8 pixels), explicit rays one per lane.  At 512x512 the camera's own
    rays passed as explicit rays (the same ids) give bitwise the same primary
    and secondary hit lists and outputs, on a surface scene and on an
    instanced one with moved objects, and at 601x433, whose last tile column
    and row are partial (packets with idle lanes); the per-ray node counts
    differ, so the two traversals really ran.  The replayed backward (order-fixed sums)
    gives bitwise the same gradients too: its primary replay runs each
    traversal from the forward's k-th distances."""
    import paper_2608_29269_amd as lf
    wl = c2_small if scene == "c2_small" else scenegen.make_workload(4, scale=0.02, resolution=48)
    st = wl.states[0] if scene == "c2_small" else wl.states[2]
    upload_scene(tracer, wl.scene)
    cam = scenegen.sphere_camera(np.random.default_rng(12), w, h)
    args = state_args(tracer, wl.scene, st)
    tracer.trace_counters()
    a = tracer.render(**args, cameras=[cam], k=32, spp=2, seed=4, hit_idx=True, sec_hit_idx=True,
                      flags=lf.FLAG_COUNT)
    ca = tracer.trace_counters()
    o, d = tracer.raygen(cam)
    b = tracer.render(**args, rays=(o, d), k=32, spp=2, seed=4, hit_idx=True, sec_hit_idx=True,
                      flags=lf.FLAG_COUNT)
    cb = tracer.trace_counters()
    for key in a:
        assert np.array_equal(a[key].cpu().numpy(), b[key].cpu().numpy()), key
    assert (a["hit_idx"].cpu().numpy() >= 0).any()
    assert ca["primary"]["rays"] == cb["primary"]["rays"] and ca["primary"]["nodes"] != cb["primary"]["nodes"], (ca, cb)
    up = dev(np.random.default_rng(3).standard_normal((o.shape[0], 3)).astype(np.float32))
    det = int(lf.FLAG_DETERMINISTIC)
    tracer.render(**args, cameras=[cam], k=32, spp=2, seed=4)
    ga = tracer.render_backward(**args, cameras=[cam], k=32, spp=2, seed=4, flags=det, d_radiance=up)
    ga = {key: v.cpu().numpy() for key, v in ga.items()}
    tracer.render(**args, rays=(o, d), k=32, spp=2, seed=4)
    gb = tracer.render_backward(**args, rays=(o, d), k=32, spp=2, seed=4, flags=det, d_radiance=up)
    for key, v in gb.items():
        assert np.array_equal(ga[key], v.cpu().numpy()), key


def test_c2_one_bounce_parity(tracer, c2_small):
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cam = st.cameras[0]
    spp = 2
    out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=32, spp=spp, seed=wl.seed,
                        hit_idx=True, sec_hit_idx=True)
    pix = np.arange(0, cam.w * cam.h, 4)
    o, d, ids = oracle.raygen(cam, pix)
    ref = run_oracle(wl.scene, st, o, d, ids, 32, spp, wl.seed, 0)
    amb = ambiguous(ref["margins"])
    sub = {k: v[pix] for k, v in out.items()}
    _compare(sub, ref, amb, check_sec=True, spp=spp)
    assert (ref["sec_alpha"] > 0).mean() > 0.05  # secondaries really hit geometry


@pytest.mark.parametrize("k", [12, 48, 64])
def test_one_bounce_parity_at_other_k(tracer, c2_small, k):
    """One-bounce forward at k in the 16- and 64-entry k-buffer
    instantiations (the secondary traversal and compositing kernels are
    compiled per bucket): primary and per-slot secondary hit lists and the
    outputs equal the oracle's."""
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cam = st.cameras[0]
    out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=k, spp=2, seed=wl.seed + k,
                        hit_idx=True, sec_hit_idx=True)
    pix = np.arange(k % 5, cam.w * cam.h, 5)
    o, d, ids = oracle.raygen(cam, pix)
    ref = run_oracle(wl.scene, st, o, d, ids, k, 2, wl.seed + k, 0)
    _compare({key: v[pix] for key, v in out.items()}, ref, ambiguous(ref["margins"]), check_sec=True, spp=2)
    assert (ref["sec_alpha"] > 0).mean() > 0.05


def test_traversal_stack_reaches_its_deepest_entries(tracer, c2_small):
    """The traversal stack keeps one LDS entry per level above the current
    node; on a 20k-surfel surface scene the primary and secondary traversals
    of a parity-checked render fill it to within one entry of the deepest
    level the hierarchy has, so every stack slot in use is compared."""
    import paper_2608_29269_amd as lf
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    info = tracer.info()
    cam = st.cameras[0]
    tracer.trace_counters()
    out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=32, spp=2, seed=8,
                        hit_idx=True, sec_hit_idx=True, flags=lf._lib.FLAG_COUNT)
    cnt = tracer.trace_counters()
    print(info, cnt, flush=True)
    for side in ("primary", "secondary"):
        assert cnt[side]["stack_pushes"] > 0
        assert info["wide_levels"] - 2 <= cnt[side]["stack_deepest"] <= info["wide_levels"] - 1, (side, cnt, info)
    pix = np.arange(1, cam.w * cam.h, 4)
    o, d, ids = oracle.raygen(cam, pix)
    ref = run_oracle(wl.scene, st, o, d, ids, 32, 2, 8, 0)
    _compare({key: v[pix] for key, v in out.items()}, ref, ambiguous(ref["margins"]), check_sec=True, spp=2)


@pytest.mark.parametrize("n", [1, 7, 63, 65, 129, 1001])
def test_persistent_pool_small_and_ragged_counts(tracer, c2_small, n):
    """Ray counts below, at and just above the eight item ranges and a wave
    of the persistent traversal: hit lists equal the oracle's."""
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cam = st.cameras[0]
    pix = np.sort(np.random.default_rng(n).choice(cam.w * cam.h, n, replace=False))
    o, d, _ = oracle.raygen(cam, pix)
    out = tracer.render(**state_args(tracer, wl.scene, st), rays=(dev(o), dev(d)), k=32, spp=2, seed=4,
                        hit_idx=True, sec_hit_idx=True)
    ref = run_oracle(wl.scene, st, o, d, np.arange(n), 32, 2, 4, 0)
    _compare(out, ref, ambiguous(ref["margins"]), check_sec=True, spp=2, min_ok=0.99 if n > 100 else 0.0)


@pytest.mark.parametrize("n", [40000, 140000])
def test_persistent_pool_wave_shares(tracer, c2_small, n):
    """Ray counts at which each wave of the resident grid takes a share of
    about 20 items, and above one item per lane of the whole grid (lanes
    refill from the pool): sampled hit lists equal the oracle's."""
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cam = scenegen.sphere_camera(np.random.default_rng(n), 512, 512)
    pix = np.sort(np.random.default_rng(n + 1).choice(cam.w * cam.h, n, replace=False))
    o, d, _ = oracle.raygen(cam, pix)
    out = tracer.render(**state_args(tracer, wl.scene, st), rays=(dev(o), dev(d)), k=32, spp=2, seed=4,
                        hit_idx=True, sec_hit_idx=True)
    sub = np.sort(np.random.default_rng(n + 2).choice(n, 2000, replace=False))
    ref = run_oracle(wl.scene, st, o[sub], d[sub], sub, 32, 2, 4, 0)
    got = {k: v.cpu()[sub] for k, v in out.items()}
    _compare(got, ref, ambiguous(ref["margins"]), check_sec=True, spp=2)
    assert (ref["alpha"] > 0).mean() > 0.2  # the sample really sees the scene


def test_odd_camera_partial_tiles(tracer, c2_small):
    """A 37x23 camera (partial 16x8 tiles on both edges) traced through the
    tile-ordered pool equals the oracle on every pixel."""
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    cam = scenegen.sphere_camera(np.random.default_rng(5), 37, 23, fov_y_deg=55.0)
    out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=32, spp=2, seed=6, hit_idx=True,
                        sec_hit_idx=True)
    o, d, ids = oracle.raygen(cam)
    ref = run_oracle(wl.scene, st, o, d, ids, 32, 2, 6, 0)
    _compare(out, ref, ambiguous(ref["margins"]), check_sec=True, spp=2)


def test_instanced_multi_state_parity(tracer):
    wl = scenegen.make_workload(4, scale=0.02, resolution=64)  # 10k background + 8 x 400
    upload_scene(tracer, wl.scene)
    for si, st in enumerate(wl.states[:2]):
        cam = st.cameras[0]
        out = tracer.render(**state_args(tracer, wl.scene, st), cameras=[cam], k=32, spp=4, seed=wl.seed + si,
                            hit_idx=True, sec_hit_idx=True)
        pix = np.arange(0, cam.w * cam.h, 3)
        o, d, ids = oracle.raygen(cam, pix)
        ref = run_oracle(wl.scene, st, o, d, ids, 32, 4, wl.seed + si, 0)
        sub = {k: v[pix] for k, v in out.items()}
        _compare(sub, ref, ambiguous(ref["margins"]), check_sec=True, spp=4)


def test_forward_is_deterministic(tracer, c2_small):
    """Two renders with the same arguments give bitwise the same outputs and
    hit lists.  A forward never starts its rays from the k-th distances of an
    earlier call (only the replay of a backward directly after its forward
    does), neither after a forward nor after a backward."""
    import paper_2608_29269_amd as lf
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    cfg = dict(cameras=st.cameras, k=32, spp=4, seed=1, hit_idx=True, sec_hit_idx=True)
    a = tracer.render(**args, **cfg)
    tracer.trace_counters()
    b = tracer.render(**args, **cfg, flags=lf.FLAG_COUNT)
    cnt = tracer.trace_counters()
    assert cnt["primary"]["hinted"] == 0 and cnt["secondary"]["hinted"] == 0, cnt
    for key in a:
        assert np.array_equal(a[key].cpu().numpy(), b[key].cpu().numpy()), key
    n = st.cameras[0].w * st.cameras[0].h * len(st.cameras)
    tracer.render_backward(**{k: v for k, v in cfg.items() if k not in ("hit_idx", "sec_hit_idx")}, **args,
                           d_radiance=dev(np.ones((n, 3), np.float32)))
    tracer.trace_counters()
    c = tracer.render(**args, **cfg, flags=lf.FLAG_COUNT)
    cnt = tracer.trace_counters()
    assert cnt["primary"]["hinted"] == 0 and cnt["secondary"]["hinted"] == 0, cnt
    for key in a:
        assert np.array_equal(a[key].cpu().numpy(), c[key].cpu().numpy()), key


def test_flags_furnace_on_gpu(tracer):
    # floor + roof, white Lambert, constant env: every sample returns a_bar * L_in (zero variance)
    from tests.helpers import make_scene
    sc = make_scene([[0, 0, 0], [0, 0, 0.5]], scale=[[10, 10]] * 2, opacity=[1, 1], albedo=[[1, 1, 1]] * 2,
                    metallic=[0, 0])
    upload_scene(tracer, sc)
    n = 300
    o = np.tile([[0.0, 0.0, 0.25]], (n, 1)).astype(np.float32)
    d = np.tile([[0.0, 0.0, -1.0]], (n, 1)).astype(np.float32)
    env = scenegen.constant_env(1.0, 8, 16)
    out = tracer.render(env=dev(env), rays=(dev(o), dev(d)), k=8, spp=2, seed=4, flags=4 | 8)
    L = out["radiance"].cpu().numpy()
    assert np.all(np.abs(L - 1.0) < 1e-5)
    st = scenegen.State(R=np.zeros((0, 3, 3), np.float32), t=np.zeros((0, 3), np.float32), env=env, cameras=[])
    ref = run_oracle(sc, st, o, d, np.arange(n), 8, 2, 4, 4 | 8)
    assert rel_close(L, ref["radiance"], 1e-6) < 1e-6


def test_edge_cases(tracer):
    from tests.helpers import make_scene
    import paper_2608_29269_amd as lf
    sc = make_scene([[0, 0, 0]], scale=[[0.3, 0.2]], opacity=[0.8])
    upload_scene(tracer, sc)
    env = dev(scenegen.lognormal_env(np.random.default_rng(1), 16, 32))
    # empty ray batch
    z = dev(np.zeros((0, 3), np.float32))
    out = tracer.render(env=env, rays=(z, z), k=4, spp=1)
    assert out["radiance"].shape[0] == 0
    # all rays miss: radiance = E(d), alpha = depth = 0, normal = 0
    o = np.tile([[5.0, 5.0, 5.0]], (10, 1)).astype(np.float32)
    d = np.tile([[0.0, 1.0, 0.0]], (10, 1)).astype(np.float32)
    out = tracer.render(env=env, rays=(dev(o), dev(d)), k=4, spp=3, seed=2)
    assert np.all(out["alpha"].cpu().numpy() == 0) and np.all(out["normal"].cpu().numpy() == 0)
    Ed = oracle.env_lookup(env.cpu().numpy(), [0, 1.0, 0])
    np.testing.assert_allclose(out["radiance"].cpu().numpy(), np.tile(Ed, (10, 1)), rtol=1e-6)
    # invalid arguments are rejected synchronously
    with pytest.raises(lf.LFError):
        tracer.render(env=env, rays=(dev(o), dev(d)), k=0, spp=1)
    with pytest.raises(lf.LFError):
        tracer.render(env=env, rays=(dev(o), dev(d)), k=4, spp=0)
    with pytest.raises(lf.LFError):
        tracer.render(env=env, rays=(dev(o), dev(d)), k=65, spp=1)
    tracer.sync()


def _check_wide(tracer, inst, leaf):
    """Every decoded slot box of a node reachable from the root contains the
    exact box of its subtree, and every leaf with a non-empty box is reached
    exactly once."""
    wb, wc = tracer.copy_wide(inst)
    none = np.iinfo(np.int32).min
    nonempty = np.all(leaf[:, :3] <= leaf[:, 3:], axis=1)
    seen = np.zeros(len(leaf), int)
    order, stack = [], [0]
    while stack:  # pre-order over the reachable nodes
        x = stack.pop()
        order.append(x)
        stack.extend(int(c) for c in wc[x] if c >= 0)
    assert len(set(order)) == len(order), "a node reached twice"
    for x in order:  # internal children occupy a node's first slots
        kinds = [0 if c >= 0 else 1 for c in wc[x] if c != none]
        assert kinds == sorted(kinds), (x, wc[x])
    exact = {}
    for x in reversed(order):  # children before parents
        lo = np.full(3, np.inf, np.float32)
        hi = np.full(3, -np.inf, np.float32)
        for i, c in enumerate(wc[x]):
            if c == none:
                continue
            if c < 0:
                seen[~c] += 1
            b = leaf[~c] if c < 0 else exact[int(c)]
            assert np.all(wb[x, i, :3] <= b[:3]) and np.all(wb[x, i, 3:] >= b[3:]), (x, i)
            lo, hi = np.minimum(lo, b[:3]), np.maximum(hi, b[3:])
        exact[x] = np.concatenate([lo, hi])
    assert np.all(seen[nonempty] == 1) and np.all(seen[~nonempty] == 0)


def test_bvh_structure_and_refit(tracer, c2_small):
    wl = c2_small
    ts = upload_scene(tracer, wl.scene)
    info = tracer.info()
    # the traversal stack holds one entry per level above the current node
    assert info["wide_levels"] - 1 <= info["stack_size"]
    assert 1 <= info["wide_levels"] <= info["max_depth"]

    def check():
        boxes, ch, perm, leaf = tracer.copy_bvh(0)
        n = wl.scene.n
        assert sorted(perm.tolist()) == list(range(n))
        # re-union from the leaves equals the stored child boxes exactly
        def union(c):
            if c < 0:
                return leaf[~c]
            b = boxes[c]
            return np.concatenate([np.minimum(b[0, :3], b[1, :3]), np.maximum(b[0, 3:], b[1, 3:])])
        seen = np.zeros(n, int)
        stack = [0]
        while stack:
            i = stack.pop()
            for s in range(2):
                c = ch[i, s]
                if c < 0:
                    seen[~c] += 1
                    assert np.array_equal(boxes[i, s], leaf[~c])
                else:
                    assert np.array_equal(boxes[i, s], union(c))
                    stack.append(c)
        assert np.all(seen == 1)
        _check_wide(tracer, 0, leaf)
    check()
    # in-place update + refit keeps the hierarchy valid and matches the oracle
    rng = np.random.default_rng(3)
    ts["mu"] += 0.01 * dev(rng.standard_normal((wl.scene.n, 3)).astype(np.float32))
    tracer.refit()
    check()
    moved = wl.scene.copy()
    moved.mu = ts["mu"].cpu().numpy()
    st = wl.states[0]
    cam = st.cameras[0]
    out = tracer.render(**state_args(tracer, moved, st), cameras=[cam], k=32, spp=1, seed=5, hit_idx=True,
                        flags=1)
    pix = np.arange(0, cam.w * cam.h, 5)
    o, d, ids = oracle.raygen(cam, pix)
    ref = run_oracle(moved, st, o, d, ids, 32, 1, 5, 1)
    _compare({k: v[pix] for k, v in out.items()}, ref, ambiguous(ref["margins"], False))


def test_secondary_regrouping_is_transparent(tracer, c2_small):
    """Tracing the secondary queue in regrouped order gives bitwise the same
    outputs as tracing it in queue order."""
    import paper_2608_29269_amd as lf
    wl = c2_small
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    a = tracer.render(**state_args(tracer, wl.scene, st), cameras=st.cameras, k=32, spp=4, seed=2,
                      sec_hit_idx=True)
    b = tracer.render(**state_args(tracer, wl.scene, st), cameras=st.cameras, k=32, spp=4, seed=2,
                      sec_hit_idx=True, flags=lf._lib.FLAG_UNSORTED)
    for key in a:
        assert np.array_equal(a[key].cpu().numpy(), b[key].cpu().numpy()), key


def test_key_collisions_are_resolved_exactly(tracer):
    """Exact duplicates (equal t: the lower index first) and near duplicates one
    binary32 step apart along z (equal binary32 keys, different double t) are
    placed by exact keys; every hit list equals the oracle's."""
    import paper_2608_29269_amd as lf
    from tests.helpers import make_scene
    rng = np.random.default_rng(7)
    n = 2000
    mu = np.column_stack([rng.uniform(-1, 1, n), rng.uniform(-1, 1, n), rng.uniform(-0.5, 0.5, n)])
    mu = mu.astype(np.float32).astype(np.float64)
    tilt = rng.normal(0, 0.1, (n, 2))
    q = np.column_stack([np.ones(n), tilt, np.zeros(n)])
    scale = np.exp(rng.uniform(np.log(0.1), np.log(0.3), (n, 2)))
    opac = np.full(n, 0.3)
    dup = rng.choice(n, 400, replace=False)
    near = rng.choice(n, 400, replace=False)
    mu_near = mu[near].copy()
    mu_near[:, 2] = np.nextafter(mu_near[:, 2].astype(np.float32), np.float32(np.inf)).astype(np.float64)
    sc = make_scene(np.vstack([mu, mu[dup], mu_near]), q=np.vstack([q, q[dup], q[near]]),
                    scale=np.vstack([scale, scale[dup], scale[near]]),
                    opacity=np.concatenate([opac, opac[dup], opac[near]]),
                    albedo=rng.uniform(0, 1, (n + 800, 3)), roughness=rng.uniform(0, 1, n + 800),
                    metallic=rng.uniform(0, 1, n + 800))
    upload_scene(tracer, sc)
    m = 3000
    o = np.column_stack([rng.uniform(-0.9, 0.9, m), rng.uniform(-0.9, 0.9, m), np.full(m, 3.0)]).astype(np.float32)
    dirs = np.column_stack([rng.normal(0, 0.05, m), rng.normal(0, 0.05, m), -np.ones(m)])
    d = (dirs / np.linalg.norm(dirs, axis=1, keepdims=True)).astype(np.float32)
    env = scenegen.constant_env(1.0, 8, 16)
    tracer.trace_counters()
    out = tracer.render(env=dev(env), rays=(dev(o), dev(d)), k=16, spp=1, seed=1, flags=lf._lib.FLAG_COUNT | 1,
                        hit_idx=True)
    cnt = tracer.trace_counters()
    st = scenegen.State(R=np.zeros((0, 3, 3), np.float32), t=np.zeros((0, 3), np.float32), env=env, cameras=[])
    ref = run_oracle(sc, st, o, d, np.arange(m), 16, 1, 1, 1)
    assert cnt["primary"]["ties"] > 20, cnt
    np.testing.assert_array_equal(out["hit_idx"].cpu().numpy(), ref["hit_idx"])
    for key in ("depth", "normal", "alpha"):
        assert rel_close(out[key].cpu().numpy(), ref[key], RTOL) < RTOL, key


def test_prefilter_keeps_hits_at_the_support_edge_and_t_min(tracer):
    """Rays aimed just inside a surfel's support edge (local radius
    (1 - delta) rho_max, delta from 1e-6 to 1e-3) at steep to grazing angles,
    over scales from 1e-3 to 10 and distances up to 300 scales, plus rays
    whose hit lies just beyond t_min: the binary32 pre-filter must pass every
    such hit, so the hit lists equal the oracle's.  A pre-filter whose error
    bound were too small would drop some of these surfels."""
    from tests.helpers import make_scene
    rng = np.random.default_rng(21)
    n = 800
    mu = rng.uniform(-20, 20, (n, 3))
    q = scenegen.uniform_quaternions(rng, n)
    scale = np.exp(rng.uniform(np.log(1e-3), np.log(10.0), (n, 2)))
    opac = rng.uniform(0.05, 1.0, n)
    sc = make_scene(mu, q=q, scale=scale, opacity=opac)
    mu32, q32, s32 = sc.mu.astype(np.float64), sc.q.astype(np.float64), sc.scale.astype(np.float64)
    a32 = sc.opacity.astype(np.float64)
    o = np.zeros((n, 3))
    d = np.zeros((n, 3))
    for i in range(n):
        tu, tv, nrm = oracle.quat_to_frame(q32[i])
        rho_max = np.sqrt(min(9.0, 2.0 * np.log(255.0 * a32[i])))
        rho = (1.0 - 10.0 ** rng.uniform(-6, -3)) * rho_max
        ph = rng.uniform(0, 2 * np.pi)
        x = mu32[i] + rho * (np.cos(ph) * s32[i, 0] * tu + np.sin(ph) * s32[i, 1] * tv)
        while True:  # |cos| between 0.02 (grazing) and 1
            w = rng.normal(size=3)
            w /= np.linalg.norm(w)
            if abs(w @ nrm) >= 0.02:
                break
        if i % 8 == 0:
            dist = 1e-4 * (1.0 + 10.0 ** rng.uniform(-3, -1))  # just beyond t_min
        else:
            dist = s32[i].min() * 10.0 ** rng.uniform(-1, 2.5)
        o[i], d[i] = x - dist * w, w
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    upload_scene(tracer, sc)
    env = scenegen.constant_env(1.0, 8, 16)
    out = tracer.render(env=dev(env), rays=(dev(o32), dev(d32)), k=16, spp=1, seed=1, flags=1, hit_idx=True)
    st = scenegen.State(R=np.zeros((0, 3, 3), np.float32), t=np.zeros((0, 3), np.float32), env=env, cameras=[])
    ref = run_oracle(sc, st, o32, d32, np.arange(n), 16, 1, 1, 1)
    amb = ambiguous(ref["margins"], include_secondary=False)
    own = (ref["hit_idx"] == np.arange(n)[:, None]).any(1)
    assert own.mean() > 0.8, own.mean()  # the aimed-at surfel really is hit
    assert amb.mean() < 0.05
    np.testing.assert_array_equal(out["hit_idx"].cpu().numpy()[~amb], ref["hit_idx"][~amb])


def test_degenerate_surfels_match_the_oracle(tracer):
    """One-bounce parity (primary and secondary hit lists, outputs) on a
    scene with degenerate surfels, and what the method fixes for them: a
    surfel below alpha_min, the needle and the edge-on surfel are never hit,
    a ray starting on a surfel's plane does not hit it (t = 0 < t_min), and
    two identical surfels sit next to each other in every list, the lower
    index first."""
    from tests.helpers import degenerate_scene, degenerate_rays
    sc = degenerate_scene()
    o, d = degenerate_rays()
    env = scenegen.lognormal_env(np.random.default_rng(7), 16, 32)
    upload_scene(tracer, sc)
    out = tracer.render(env=dev(env), rays=(dev(o), dev(d)), k=16, spp=2, seed=3, hit_idx=True, sec_hit_idx=True)
    st = scenegen.State(R=np.zeros((0, 3, 3), np.float32), t=np.zeros((0, 3), np.float32), env=env, cameras=[])
    ref = run_oracle(sc, st, o, d, np.arange(len(o)), 16, 2, 3, 0)
    amb = ambiguous(ref["margins"])
    _compare(out, ref, amb, check_sec=True, spp=2)
    h = out["hit_idx"].cpu().numpy()
    for i in (0, 2, 3):
        assert not (h == i).any(), i
    assert (h[:576] == 1).any(1).all() and (h[:576] == 4).any(1).all()
    assert not (h[576:] == 4).any()
    both = (h == 7).any(1) & (h == 8).any(1)
    assert both.all()
    assert np.array_equal(np.argmax(h == 8, axis=1), np.argmax(h == 7, axis=1) + 1)
    assert (ref["sec_alpha"] > 0).mean() > 0.2


def test_size_limits_are_reported_before_any_work(tracer):
    """Ray ids are 32-bit: a call with rays x secondary slots at or past
    2^31 - 1 is refused with LF_EUNSUPPORTED by the host checks, before any
    buffer is sized or kernel launched (so the cameras below cost nothing),
    and the context serves the next call as before."""
    import paper_2608_29269_amd as lf
    from paper_2608_29269_amd import _lib
    wl = scenegen.make_workload(1, scale=0.25, resolution=16)
    st = wl.states[0]
    upload_scene(tracer, wl.scene)
    args = state_args(tracer, wl.scene, st)
    ref = tracer.render(**args, cameras=st.cameras, k=16, spp=1, seed=2, flags=1)
    ref = {key: v.cpu().numpy() for key, v in ref.items()}
    big = scenegen.look_at_camera(np.array([0.0, 0.0, 3.0]), 46341, 46341)  # 2^31 + 4,280 pixels
    half = scenegen.look_at_camera(np.array([0.0, 0.0, 3.0]), 32768, 32768)  # 2^30 pixels, x 2 slots
    for cam, spp, flags in ((big, 1, 1), (half, 2, 0), (half, 1, int(lf.FLAG_NEE))):
        dummy = dev(np.zeros((1, 3), np.float32))
        out = dict(radiance=dummy, depth=dummy, normal=dummy, alpha=dummy)  # never written: the call is refused
        with pytest.raises(lf.LFError) as e:
            tracer.render(**args, cameras=[cam], k=16, spp=spp, seed=2, flags=flags, out=out)
        assert e.value.status == _lib.LF_EUNSUPPORTED, (cam.w, spp, flags)
        with pytest.raises(lf.LFError) as e:
            tracer.render_backward(**args, cameras=[cam], k=16, spp=spp, seed=2, flags=flags,
                                   d_radiance=None)
        assert e.value.status == _lib.LF_EUNSUPPORTED
    again = tracer.render(**args, cameras=st.cameras, k=16, spp=1, seed=2, flags=1)
    tracer.sync()
    for key in ref:
        assert np.array_equal(again[key].cpu().numpy(), ref[key]), key
