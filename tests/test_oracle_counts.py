"""Pins of the oracle's per-ray work counts and decision margins.

The counts (supports crossed before the k-th hit, composited hits, secondary
rays, environment lookups) are what the benchmark turns into algorithmic
bytes; the margins (distance of every discrete decision to its switching
point) decide which rays count as legitimately ambiguous in the parity tests
(several correct results: both sides decide in double precision from the
same binary32 inputs, so only rays whose decisions sit within rounding noise
of a switching point may differ).  Both are checked here on constructed
scenes whose values follow from the geometry alone:

  * counts: a stack of parallel surfels along the ray (Sec. 3.2, depth sort
    and k-truncation; a crossing below the opacity threshold is touched but
    not composited), and a floor under two roof layers whose every secondary
    ray (Sec. 3.3, one secondary interaction) meets both layers, with the
    environment lit only inside a polar cap so that each environment sample's
    hemisphere test is known in advance;
  * margins: each one is driven to its switching point and the decision is
    shown to flip there (t order, support/threshold, t_min, environment CDF
    edge, lobe choice), or equals a closed form of the published sampler
    (cosine of a Malley direction).

CPU only; tests/test_oracle_mutants.py shows that plausible slips in the
oracle's bookkeeping fail these pins."""
import functools

import numpy as np
import pytest

import oracle
import scenegen
from tests.helpers import axis_angle_quat, make_scene, no_transforms, rays_single

NS, DIFF, BSDF, NOBG, NEE = (oracle.NO_SECONDARY, oracle.DIFFUSE_ONLY, oracle.BSDF_ONLY, oracle.NO_BACKGROUND,
                             oracle.NEE)
C = dict(touch=oracle.C_TOUCH_PRI, comp=oracle.C_COMP_PRI, sec=oracle.C_SEC_RAYS, touch2=oracle.C_TOUCH_SEC,
         comp2=oracle.C_COMP_SEC, env=oracle.C_ENV)


def run(scene, o, d, ids, env=None, overrides=None, **kw):
    R, t = no_transforms(scene)
    if env is None:
        env = scenegen.constant_env(1.0, 8, 16)
    sa = oracle.SceneArrays(scene, R, t, env, overrides=overrides)
    p = oracle.Params(**{**dict(k=16, spp=1, seed=7, flags=NS), **kw})
    return oracle.render(sa, o, d, ids, p)


def counts(out, r=0):
    return {k: out["counts"][r, v] for k, v in C.items()}


# --- counts on a stack of parallel surfels -------------------------------------------------
# The ray runs from (0, 0, 5) down the z axis, so a surfel centred at height z
# is met at t = 5 - z.  Eight valid surfels at t = 1.0, 1.1, ..., 1.7 (on the
# axis: rho = 0); two faint ones (opacity 0.05: rho^2_max = 2 ln 12.75 = 5.09)
# crossed at rho = 2.5, inside the 3-sigma support but below the opacity
# threshold, at t = 1.25 and t = 1.75; one crossed at rho = 3.5, outside the
# support, at t = 1.05; and one behind the origin.
def stack_scene():
    t_valid = 1.0 + 0.1 * np.arange(8)
    s = 0.2
    mu = [[0, 0, 5 - t] for t in t_valid]
    mu += [[2.5 * s, 0, 5 - 1.25], [2.5 * s, 0, 5 - 1.75], [3.5 * s, 0, 5 - 1.05], [0, 0, 5.5]]
    op = [0.3] * 8 + [0.05, 0.05, 0.3, 0.3]
    return make_scene(mu, scale=np.full((12, 2), s), opacity=op)


@pytest.mark.parametrize("k,touch,comp", [
    (5, 6, 5),    # t_(k) = 1.4: five valid hits plus the faint crossing at 1.25
    (8, 9, 8),    # t_(k) = 1.7 is the last valid hit: the faint crossing at 1.75 lies beyond it
    (16, 10, 8),  # fewer valid hits than k: t_(k) is infinite and both faint crossings count
])
def test_counts_parallel_stack(k, touch, comp):
    sc = stack_scene()
    rays = rays_single([0, 0, 5], [0, 0, -1])
    c = counts(run(sc, *rays, k=k, spp=3, flags=NS | DIFF | BSDF))
    # with no secondary ray, each of the three cosine samples (all above the
    # surface) reads E(w) once, after the background lookup E(d)
    assert c == dict(touch=touch, comp=comp, sec=0, touch2=0, comp2=0, env=1 + 3)
    c = counts(run(sc, *rays, k=k, spp=3, flags=NS | DIFF | BSDF | NOBG))
    assert c["env"] == 3 and c["touch"] == touch


def test_counts_of_a_miss():
    sc = stack_scene()
    c = counts(run(sc, *rays_single([5, 5, 5], [0, 0, -1]), spp=4, flags=NS | DIFF | BSDF))
    assert c == dict(touch=0, comp=0, sec=0, touch2=0, comp2=0, env=1)  # only the background


# --- counts with secondary rays: a floor under two roof layers --------------------------
# Floor at y = 0 facing +Y, roofs at y = 1 and y = 1.5 so wide (scale 1e4) that
# every upward secondary ray crosses both near their centres.  The
# environment is lit only in its top row (polar angle below 45 degrees), so
# environment samples point up: at the floor they are live, at a roof (whose
# normal turns down to face the upward ray) they fall below the hemisphere.
# Cosine samples are live everywhere.  The camera looks straight down from
# between floor and roofs, so the roofs lie behind it.
def floor_roof():
    qy = axis_angle_quat([1, 0, 0], -np.pi / 2)  # e_z -> +Y
    sc = make_scene([[0, 0, 0], [0, 1.0, 0], [0, 1.5, 0]], q=[qy] * 3,
                    scale=[[10, 10], [1e4, 1e4], [1e4, 1e4]], opacity=[0.999, 0.5, 0.5])
    env = np.zeros((4, 8, 3))
    env[0] = 1.0
    return sc, env, rays_single([0.1, 0.5, 0.2], [0, -1, 0])


@pytest.mark.parametrize("flags,sec,env", [
    (DIFF, 1, 2),               # one ray per sample; E(w), then the roof's BSDF sample (its env sample is dead)
    (DIFF | NEE, 2, 3),         # next-event + continuation rays, both traced; only continuations sample at the roof
    (DIFF | NEE | BSDF, 1, 2),  # no environment sampling: the next-event slot is dead
    (DIFF | NS, 0, 1),          # nothing traced: E(w) per sample only
])
@pytest.mark.parametrize("bg", [0, NOBG])
def test_counts_floor_and_roof(flags, sec, env, bg):
    sc, E, rays = floor_roof()
    S = 3
    c = counts(run(sc, *rays, env=E, k=8, spp=S, flags=flags | bg))
    want = dict(touch=1, comp=1, sec=sec * S, touch2=2 * sec * S, comp2=2 * sec * S,
                env=(0 if bg else 1) + env * S)
    assert c == want
    # at k = 1 each secondary ray keeps only the nearer roof, which is then
    # its k-th hit: the farther roof is crossed beyond t_(k) and not touched
    c1 = counts(run(sc, *rays, env=E, k=1, spp=S, flags=flags | bg))
    assert (c1["touch2"], c1["comp2"]) == (sec * S, sec * S)


# --- margins at their switching points ------------------------------------------------------
@pytest.mark.parametrize("k,gap", [(1, 0.25), (2, 0.125), (3, 0.0625)])
def test_margin_t_gap_over_the_first_k_plus_one(k, gap):
    # hits at t = 1, 1.25, 1.375, 1.4375 (binary32-exact heights): the margin is
    # the smallest gap among the first k+1 hits, since the (k+1)-th could swap
    # with the k-th
    ts = [1.0, 1.25, 1.375, 1.4375]
    sc = make_scene([[0, 0, 5 - t] for t in ts], scale=np.full((4, 2), 1.0), opacity=[0.3] * 4)
    out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]), k=k)
    assert out["margins"][0, oracle.M_TGAP_PRI] == gap


def test_margin_t_gap_ignores_exact_ties():
    # an exact duplicate is ordered by index, not by t: its zero gap is no margin
    sc = make_scene([[0, 0, 4], [0, 0, 4], [0, 0, 3.5]], scale=np.full((3, 2), 1.0), opacity=[0.3] * 3)
    out = run(sc, *rays_single([0, 0, 5], [0, 0, -1]), k=2)
    assert out["margins"][0, oracle.M_TGAP_PRI] == 0.5


def _bisect(valid, lo, hi, it=200):
    """Switching point of a monotone decision valid(lo) = True, valid(hi) = False."""
    for _ in range(it):
        mid = 0.5 * (lo + hi)
        if mid in (lo, hi):
            break
        lo, hi = (mid, hi) if valid(mid) else (lo, mid)
    return lo, hi


@pytest.mark.parametrize("alpha", [0.1, 1.0])  # threshold below 3 sigma / the 3-sigma support itself
def test_margin_support_threshold_at_its_switching_point(alpha):
    # a surfel at the origin facing +z, scale 0.25 (rho = x / 0.25 on the x
    # axis); rays straight down at offset x.  The margin must equal the
    # distance of rho^2 to the value at which the validity decision switches.
    s = 0.25
    sc = make_scene([[0, 0, 0]], scale=[[s, s]], opacity=[alpha])

    def out(x):
        return run(sc, *rays_single([x, 0, 3], [0, 0, -1]))

    lo, hi = _bisect(lambda x: out(x)["hit_idx"][0, 0] == 0, 0.0, 4 * s)
    rho2_star = (0.5 * (lo + hi) / s) ** 2
    for x in (lo - 1e-7, lo - 1e-4, hi + 1e-7, hi + 1e-4):
        m = out(x)["margins"][0, oracle.M_RHO_PRI]
        assert m == pytest.approx(abs((x / s) ** 2 - rho2_star), abs=1e-12)
    assert out(lo - 1e-7)["hit_idx"][0, 0] == 0 and out(hi + 1e-7)["hit_idx"][0, 0] == -1


def test_margin_t_min():
    # a surfel met at t = t_min + eta: the margin is |eta| and the hit switches sign with eta
    sc = make_scene([[0, 0, 0]], scale=[[1.0, 1.0]], opacity=[0.5])
    t_min = oracle.Params().t_min
    for eta in (3e-9, -3e-9, 2e-6):
        out = run(sc, *rays_single([0, 0, t_min + eta], [0, 0, -1]))
        assert out["margins"][0, oracle.M_TMIN] == pytest.approx(abs(eta), abs=1e-18)
        assert (out["hit_idx"][0, 0] == 0) == (eta > 0)


def _find_ray(seed, want, n=4000):
    for i in range(n):
        if want(i):
            return i
    raise AssertionError("no suitable ray id")


def test_margin_environment_cdf_edge():
    # a 4x8 map lit in its two upper rows only, each row grey and uniform: the
    # marginal CDF's first inner edge lies at a s0 / (a s0 + b s1), with
    # s_r = sin(theta) at the row centres.  Place it eta above (below) the row
    # uniform of an environment-sampled ray: the margin is |eta| and the
    # sample falls in row 0 (row 1).  The direction is continuous across the
    # edge but the texel pdf is not (a != b), so the frozen weight and hence
    # the radiance jump there.
    seed = 11

    def ok(i):
        ub = oracle.uniform(seed, i, 0, 3) * 8
        return (oracle.uniform(seed, i, 0, 0) < 0.5 and 0.45 < oracle.uniform(seed, i, 0, 2) < 0.8
                and abs(ub - np.round(ub)) > 1e-2)

    rid = _find_ray(seed, ok)
    ua = oracle.uniform(seed, rid, 0, 2)
    s0, s1 = np.sin(np.pi / 8), np.sin(3 * np.pi / 8)
    qy = axis_angle_quat([1, 0, 0], -np.pi / 2)
    sc = make_scene([[0, 0, 0]], q=[qy], scale=[[10, 10]], opacity=[0.9])
    o, d, _ = rays_single([0, 1, 0], [0, -1, 0])
    L = {}
    for eta in (2e-9, -2e-9):
        e = ua + eta
        env = np.zeros((4, 8, 3))
        env[0], env[1] = e * s1 / (s0 * (1.0 - e)), 1.0
        out = run(sc, o, d, np.array([rid]), env=env, seed=seed, flags=NS | DIFF | NOBG)
        assert out["margins"][0, oracle.M_ENV] == pytest.approx(abs(eta), abs=1e-15)
        L[eta > 0] = out["radiance"][0, 0]
    assert abs(L[True] - L[False]) > 1e-2 * abs(L[True])


@pytest.mark.parametrize("eta", [1e-9, -1e-9])
def test_margin_lobe_choice(eta):
    # grey albedo a, metallic 0: q_spec = 0.04 / (0.04 + a).  Choose a so that
    # q_spec = u1 + eta for the lobe uniform u1: the margin is |eta| and the
    # lobe (GGX below q_spec, cosine above) flips with the sign of eta
    seed = 5
    rid = _find_ray(seed, lambda i: 0.2 < oracle.uniform(seed, i, 0, 1) < 0.8)
    u1 = oracle.uniform(seed, rid, 0, 1)

    sc = make_scene([[0, 0, 0]], scale=[[1, 1]], opacity=[0.9], roughness=[0.3])
    o, d, _ = rays_single([0.1, 0, 2], [0, 0, -1])
    env = scenegen.lognormal_env(np.random.default_rng(1), 8, 16)  # E(w) tells the two directions apart

    def render(q, A=None):
        # the lobe is chosen from the composited albedo a A / (A + eps)
        a = 0.04 * (1.0 - q) / q * (1.0 if A is None else (A + 1e-6) / A)
        ov = dict(albedo=np.full((1, 3), a), metallic=np.zeros(1))
        return run(sc, o, d, np.array([rid]), env=env, overrides=ov, seed=seed, flags=NS | BSDF)

    A = render(0.5)["alpha"][0]
    render = functools.partial(render, A=A)

    out = render(u1 + eta)
    assert out["margins"][0, oracle.M_LOBE] == pytest.approx(abs(eta), abs=1e-15)
    other = render(u1 - eta)
    assert abs(out["radiance"][0, 0] - other["radiance"][0, 0]) > 1e-2 * out["radiance"][0, 0]


def test_margin_cosine_of_malley_directions():
    # cosine sampling about the composited normal: n.w = sqrt(1 - u2) for the
    # direction uniform u2 (dimension 2), whatever the normal's orientation
    seed, S = 3, 4
    q = axis_angle_quat([1, 0, 0], 0.4)
    sc = make_scene([[0, 0, 0]], q=[q], scale=[[1, 1]], opacity=[0.9])
    for rid in (0, 17, 123):
        o, d, _ = rays_single([0.05, -0.02, 2], [0, 0, -1])
        out = run(sc, o, d, np.array([rid]), seed=seed, spp=S, flags=NS | DIFF | BSDF)
        want = min(np.sqrt(1.0 - oracle.uniform(seed, rid, s, 2)) for s in range(S))
        assert out["margins"][0, oracle.M_COS] == pytest.approx(want, abs=1e-12)


# the pins run again against deliberately broken builds of the oracle
PINS = [
    (test_counts_parallel_stack, [(5, 6, 5), (8, 9, 8), (16, 10, 8)]),
    (test_counts_of_a_miss, [()]),
    (test_counts_floor_and_roof, [(DIFF, 1, 2, 0), (DIFF | NEE, 2, 3, 0), (DIFF | NEE | BSDF, 1, 2, 0),
                                  (DIFF | NS, 0, 1, 0), (DIFF, 1, 2, NOBG)]),
    (test_margin_t_gap_over_the_first_k_plus_one, [(1, 0.25), (2, 0.125), (3, 0.0625)]),
    (test_margin_t_gap_ignores_exact_ties, [()]),
    (test_margin_support_threshold_at_its_switching_point, [(0.1,), (1.0,)]),
    (test_margin_t_min, [()]),
    (test_margin_environment_cdf_edge, [()]),
    (test_margin_lobe_choice, [(1e-9,), (-1e-9,)]),
    (test_margin_cosine_of_malley_directions, [()]),
]
