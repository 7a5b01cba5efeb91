"""Small scene builders shared by the tests (inputs only; no method arithmetic)."""
import numpy as np

import scenegen


def make_scene(mu, q=None, scale=None, opacity=None, albedo=None, roughness=None, metallic=None,
               object_offset=None):
    mu = np.asarray(mu, dtype=np.float64).reshape(-1, 3)
    n = mu.shape[0]
    if q is None:
        q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    if scale is None:
        scale = np.full((n, 2), 0.1)
    if opacity is None:
        opacity = np.full(n, 0.5)
    if albedo is None:
        albedo = np.full((n, 3), 0.5)
    if roughness is None:
        roughness = np.full(n, 0.5)
    if metallic is None:
        metallic = np.zeros(n)
    if object_offset is None:
        object_offset = [0, n]
    f = np.float32
    return scenegen.Scene(mu=mu.astype(f), q=np.asarray(q, dtype=np.float64).reshape(n, 4).astype(f),
                          scale=np.asarray(scale, dtype=np.float64).reshape(n, 2).astype(f),
                          opacity=np.asarray(opacity, dtype=np.float64).reshape(n).astype(f),
                          albedo=np.asarray(albedo, dtype=np.float64).reshape(n, 3).astype(f),
                          roughness=np.asarray(roughness, dtype=np.float64).reshape(n).astype(f),
                          metallic=np.asarray(metallic, dtype=np.float64).reshape(n).astype(f),
                          object_offset=np.asarray(object_offset, dtype=np.int64))


def axis_angle_quat(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    return np.concatenate([[np.cos(angle / 2)], np.sin(angle / 2) * axis])


def no_transforms(scene):
    M = scene.n_objects
    return np.tile(np.eye(3, dtype=np.float32), (M, 1, 1)), np.zeros((M, 3), dtype=np.float32)


def rays_single(o, d):
    o = np.asarray(o, dtype=np.float64).reshape(-1, 3)
    d = np.asarray(d, dtype=np.float64).reshape(-1, 3)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    return o, d, np.arange(o.shape[0], dtype=np.int64)


def degenerate_scene():
    """A stack of surfels along +z with degenerate members, above 200 random
    ones: opacity below alpha_min (no support), an unnormalised quaternion
    (5 x a unit one), a needle (one scale 1e-6), a surfel edge-on to the rays,
    one whose plane holds some rays' origins (z = 0.8), a huge one (scales
    50), one at opacity 1 (capped at alpha_cap), and two identical surfels."""
    rng = np.random.default_rng(5)
    c, s = np.cos(0.3), np.sin(0.3)
    r4 = np.cos(np.pi / 4)
    mu = [[0, 0, 0.0], [0, 0, 0.2], [0, 0, 0.4], [0, 0, 0.6], [0, 0, 0.8], [0, 0, 1.0], [0, 0, 1.2],
          [0.01, 0, 1.4], [0.01, 0, 1.4]]
    q = [[1, 0, 0, 0], [5 * c, 5 * s, 0, 0], [1, 0, 0, 0], [r4, r4, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0],
         [1, 0, 0, 0], [1, 0, 0, 0], [1, 0, 0, 0]]
    scale = [[0.3, 0.3], [0.3, 0.2], [1e-6, 0.2], [0.3, 0.3], [0.3, 0.3], [50.0, 50.0], [0.3, 0.3],
             [0.25, 0.25], [0.25, 0.25]]
    opac = [0.002, 0.6, 0.9, 0.8, 0.5, 0.3, 1.0, 0.4, 0.4]
    m = 200
    mu = np.concatenate([np.array(mu), np.c_[rng.uniform(-1, 1, (m, 2)), rng.uniform(1.8, 3.0, m)]])
    q = np.concatenate([np.array(q, float), scenegen.uniform_quaternions(rng, m)])
    scale = np.concatenate([np.array(scale), np.exp(rng.uniform(np.log(0.05), np.log(0.4), (m, 2)))])
    opac = np.concatenate([opac, rng.uniform(0.05, 1.0, m)])
    n = len(mu)
    return make_scene(mu, q=q, scale=scale, opacity=opac, albedo=rng.uniform(0, 1, (n, 3)),
                      roughness=rng.uniform(0.05, 1, n), metallic=rng.uniform(0, 1, n))



def degenerate_rays():
    """576 rays from z = -2 up through the stack of degenerate_scene(), and 64
    rays along +z that start on the plane of its surfel 4 (binary32)."""
    g = np.linspace(-0.3, 0.3, 24)
    X, Y = np.meshgrid(g, g)
    d = np.c_[0.05 * X.ravel(), 0.05 * Y.ravel(), np.ones(X.size)]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o = np.c_[X.ravel(), Y.ravel(), np.full(X.size, -2.0)]
    o2 = np.c_[np.random.default_rng(6).uniform(-0.2, 0.2, (64, 2)), np.full(64, 0.8)]
    o = np.concatenate([o, o2]).astype(np.float32)
    d = np.concatenate([d, np.tile([0.0, 0.0, 1.0], (64, 1))]).astype(np.float32)
    return o, d
