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
