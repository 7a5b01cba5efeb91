"""Pins of the oracle's Owen-scrambled Sobol sampler (Sec. 3.3 PRB paragraph:
Sobol samples replayed from the recorded seed): the first points of the low
dimensions worked out by hand from the construction, the net properties of
the raw sequence, the prefix property of the nested scramble, stratification
of every ray's scrambled samples, and the estimator: unbiased against
quadrature, with a lower variance than the hash sampler.  CPU only."""
import numpy as np
import pytest

import oracle
import scenegen
from tests.helpers import make_scene, no_transforms

P = oracle.Params
DIMS = 11


def test_first_points_of_the_low_dimensions():
    # dimension 0: van der Corput (bit reversal of the index)
    assert [oracle.sobol(i, 0) / 2**32 for i in range(8)] == [0, .5, .25, .75, .125, .625, .375, .875]
    # dimension 1, polynomial x + 1 (m_1 = 1): m_k = 2 m_(k-1) ^ m_(k-1) gives m = 1, 3, 5, 15, i.e.
    # V = .5, .75, .625, .9375; point i XORs V_k over the set bits k of i
    assert [oracle.sobol(i, 1) / 2**32 for i in range(8)] == [0, .5, .75, .25, .625, .125, .375, .875]
    # dimension 2, polynomial x^2 + x + 1 (m_1, m_2 = 1, 3): m_3 = 2 m_2 ^ 4 m_1 ^ m_1 = 3, V_3 = .375
    assert [oracle.sobol(i, 2) / 2**32 for i in range(8)] == [0, .5, .75, .25, .375, .875, .625, .125]


@pytest.mark.parametrize("d", range(DIMS))
def test_every_dimension_is_a_0m1_net(d):
    x = np.array([oracle.sobol(i, d) for i in range(1 << 12)], dtype=np.uint64)
    for m in range(1, 13):
        for start in (0, 1 << m) if m < 12 else (0,):  # the first block and the next aligned one
            blk = x[start:start + (1 << m)] if start + (1 << m) <= x.size else None
            if blk is None:
                continue
            cells = np.sort(blk >> np.uint64(32 - m))
            assert np.array_equal(cells, np.arange(1 << m)), (d, m, start)


def test_dimensions_0_and_1_form_0m2_nets():
    n = 1 << 10
    x = np.array([[oracle.sobol(i, 0), oracle.sobol(i, 1)] for i in range(n)], dtype=np.uint64)
    for m in range(1, 11):
        pts = x[: 1 << m]
        for a in range(m + 1):
            cx = pts[:, 0] >> np.uint64(32 - a) if a else np.zeros(len(pts), np.uint64)
            cy = pts[:, 1] >> np.uint64(32 - (m - a)) if m - a else np.zeros(len(pts), np.uint64)
            cells = cx * np.uint64(1 << (m - a)) + cy
            assert np.array_equal(np.sort(cells), np.arange(1 << m)), (m, a)


def _gf2_mulmod(a, b, poly, deg):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> deg & 1:
            a ^= poly
    return r


def test_polynomials_are_distinct_and_primitive():
    """Sobol's construction needs primitive polynomials over GF(2): x has
    order 2^s - 1 modulo each; the direction numbers m_k are odd and
    below 2^k."""
    seen = set()
    for d in range(1, DIMS):
        s, a = oracle.sobol_poly(d)
        poly = (1 << s) | (a << 1) | 1
        assert poly not in seen
        seen.add(poly)
        order, x = 1, 2 % poly if s > 1 else 1
        while x != 1:
            x = _gf2_mulmod(x, 2, poly, s)
            order += 1
        assert order == (1 << s) - 1 or s == 1, (d, s, a, order)
        for k in range(1, 16):
            v = oracle.sobol(1 << (k - 1), d)  # point 2^(k-1) is V_k
            mk = v >> (32 - k)
            assert mk & 1 and mk < (1 << k) and v == mk << (32 - k), (d, k)


def _t_value(d1, d2, m):
    x = np.array([[oracle.sobol(i, d1), oracle.sobol(i, d2)] for i in range(1 << m)], dtype=np.uint64)
    for t in range(m + 1):
        k = m - t
        good = True
        for a in range(k + 1):
            cx = x[:, 0] >> np.uint64(32 - a) if a else np.zeros(len(x), np.uint64)
            cy = x[:, 1] >> np.uint64(32 - (k - a)) if k - a else np.zeros(len(x), np.uint64)
            cnt = np.bincount((cx * np.uint64(1 << (k - a)) + cy).astype(np.int64), minlength=1 << k)
            if not np.all(cnt == (1 << t)):
                good = False
                break
        if good:
            return t
    return m


def test_two_dimensional_projections_are_good_nets():
    """Every pair of the 11 dimensions is a (t,m,2)-net with t <= 4 for
    m = 6, 8 (the quality the chosen direction numbers are made for); the
    first pair has t = 0."""
    for m in (6, 8):
        for d1 in range(DIMS):
            for d2 in range(d1 + 1, DIMS):
                assert _t_value(d1, d2, m) <= 4, (d1, d2, m)
    assert _t_value(0, 1, 8) == 0


def test_owen_scramble_is_nested():
    """Values sharing their top j bits keep sharing them after the scramble
    (a nested permutation of the elementary intervals), and the scramble is
    one-to-one on every aligned block."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        seed = int(rng.integers(0, 2**32))
        j = int(rng.integers(1, 31))
        top = int(rng.integers(0, 2**32)) >> (32 - j) << (32 - j)
        a = top | int(rng.integers(0, 1 << (32 - j)))
        b = top | int(rng.integers(0, 1 << (32 - j)))
        sa, sb = oracle.owen_scramble(a, seed), oracle.owen_scramble(b, seed)
        assert sa >> (32 - j) == sb >> (32 - j)
    seed = 0x9E3779B9
    vals = {oracle.owen_scramble(v << 20, seed) >> 20 for v in range(1 << 12)}
    assert len(vals) == 1 << 12


@pytest.mark.parametrize("m", [2, 4, 6])
def test_scrambled_samples_of_a_ray_are_stratified(m):
    """The 2^m samples of one ray (spp = 2^m) take one cell of every 1/2^m
    stratum in each dimension and form a (0,m,2)-net in dimensions 0 and 1:
    the index scramble maps them onto an aligned block of the sequence."""
    for seed, ray in ((1, 0), (1005, 123456), (7, 2**40 + 3)):
        u = np.array([[oracle.sobol_uniform(seed, ray, s, d) for d in range(DIMS)] for s in range(1 << m)])
        for d in range(DIMS):
            assert np.array_equal(np.sort(np.floor(u[:, d] * (1 << m)).astype(int)), np.arange(1 << m)), (d,)
        for a in range(m + 1):
            cells = np.floor(u[:, 0] * (1 << a)).astype(int) * (1 << (m - a)) + np.floor(u[:, 1] * (1 << (m - a)))
            assert np.array_equal(np.sort(cells.astype(int)), np.arange(1 << m))
    u0 = [oracle.sobol_uniform(1, 0, s, 3) for s in range(8)]
    u1 = [oracle.sobol_uniform(1, 1, s, 3) for s in range(8)]
    assert u0 != u1  # every ray its own scramble
    assert all(v * 2**24 == int(v * 2**24) for v in u0)  # 24-bit uniforms


def test_sobol_estimator_is_unbiased_with_lower_variance():
    """Lambert plane under a smooth environment, 16 samples per estimate:
    both samplers agree with quadrature of int f cos E dw; the scrambled
    Sobol estimates scatter less than the hash sampler's."""
    env = scenegen.lognormal_env(np.random.default_rng(9), 8, 16, lobe_gain=5.0, lobe_width=0.6)
    a = np.array([0.8, 0.5, 0.3])
    sc = make_scene([[0, 0, 0]], scale=[[10, 10]], opacity=[1.0], albedo=[a], metallic=[0.0], roughness=[0.5])
    d = np.array([0.2, -0.1, -1.0])
    d /= np.linalg.norm(d)
    R, t = no_transforms(sc)
    sa = oracle.SceneArrays(sc, R, t, env)
    n = 3000
    oo, dd = np.tile(-3 * d, (n, 1)), np.tile(d, (n, 1))
    res = {}
    for name, fl in (("hash", 0), ("sobol", oracle.SOBOL)):
        p = P(k=8, spp=16, seed=5, flags=fl | oracle.NO_SECONDARY | oracle.DIFFUSE_ONLY)
        res[name] = oracle.render(sa, oo, dd, np.arange(n), p, lists=False)["radiance"]
    H, W = env.shape[:2]
    sub = 12
    acc = np.zeros(3)
    a32 = a.astype(np.float32).astype(np.float64)
    for i in range(H * sub):
        th = (i + 0.5) * np.pi / (H * sub)
        for j in range(W * sub):
            ph = (j + 0.5) * 2 * np.pi / (W * sub)
            w = np.array([np.sin(th) * np.cos(ph), np.cos(th), np.sin(th) * np.sin(ph)])
            if w[2] > 0:
                acc += a32 / np.pi * w[2] * oracle.env_lookup(env, w) * np.sin(th)
    acc *= (np.pi / (H * sub)) * (2 * np.pi / (W * sub))
    want = 0.99 * acc + 0.01 * oracle.env_lookup(env, d)
    for name, L in res.items():
        se = L.std(0) / np.sqrt(n)
        assert np.all(np.abs(L.mean(0) - want) < 4 * se + 2e-3 * np.abs(want)), (name, L.mean(0), want)
    assert np.all(res["sobol"].std(0) < 0.7 * res["hash"].std(0)), (res["sobol"].std(0), res["hash"].std(0))


def test_replay_of_the_sobol_sampler_is_exact():
    wl = scenegen.make_workload(2, scale=0.02, resolution=16)
    st = wl.states[0]
    o, d, ids = oracle.raygen(st.cameras[0])
    sa = oracle.SceneArrays(wl.scene, st.R, st.t, st.env)
    p = P(k=wl.k, spp=4, seed=3, flags=oracle.SOBOL | oracle.NEE)
    a = oracle.render(sa, o, d, ids, p)
    b = oracle.render(sa, o, d, ids, p)
    assert np.array_equal(a["radiance"], b["radiance"]) and np.array_equal(a["sec_hit_idx"], b["sec_hit_idx"])
    c = oracle.render(sa, o, d, ids, P(k=wl.k, spp=4, seed=3, flags=oracle.NEE))
    assert not np.array_equal(a["sec_hit_idx"], c["sec_hit_idx"])  # the sampler is in effect
