"""Seeded synthetic inputs for the surfel ray tracer and for its FP64 oracle.

This module is the only code shared by the GPU path's tests/benchmarks and the
oracle: it draws surfel scenes, rigid transforms, environment maps and cameras
from fixed seeds.  It contains none of the method's arithmetic (no
intersection, compositing, shading or sampling); it only produces the inputs
the method consumes.

Surfel tuple (Sec. 3.1, Eq. gaussian-primitive): centre mu, unit quaternion q
(stored w, x, y, z), in-plane scale s (2), opacity alpha, base colour a (3),
roughness r and metallic m.  The splatting feature f is not part of the traced
scene.  Scenes are a background plus M objects (Eq. state-assembly); object
surfels live in object space and each state supplies one rigid transform per
object.

The paper's datasets (four Blender rooms and real captures, Sec. 4.1) are not
available; these generators stand in for them with the recipe below.

Common surfel draw: opacity sigmoid(N(0,1)); scales log-uniform in
[0.01, 0.1] per axis; albedo, roughness, metallic U[0,1]; orientation uniform
on S^3 (Shoemake 1992) unless the surface-like recipe sets it.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

F32 = np.float32


@dataclasses.dataclass
class Camera:
    """Pinhole camera: pose is the 3x4 camera-to-world matrix, row-major, whose
    columns are (right, up, back, centre); the camera looks along -back."""
    pose: np.ndarray  # [12] float32
    fov_y_deg: float
    w: int
    h: int

    @property
    def n_rays(self) -> int:
        return self.w * self.h


@dataclasses.dataclass
class Scene:
    mu: np.ndarray        # [N,3] f32 (object space for object surfels)
    q: np.ndarray         # [N,4] f32, (w,x,y,z), not necessarily unit
    scale: np.ndarray     # [N,2] f32 > 0
    opacity: np.ndarray   # [N]   f32 in (0,1]
    albedo: np.ndarray    # [N,3] f32 in [0,1]
    roughness: np.ndarray  # [N]  f32 in [0,1]
    metallic: np.ndarray  # [N]   f32 in [0,1]
    object_offset: np.ndarray  # [M+2] int64: [0,off1) background, [off_o, off_o+1) object o

    @property
    def n(self) -> int:
        return int(self.mu.shape[0])

    @property
    def n_objects(self) -> int:
        return int(self.object_offset.shape[0]) - 2

    def copy(self) -> "Scene":
        return Scene(**{f.name: np.array(getattr(self, f.name), copy=True)
                        for f in dataclasses.fields(self)})


@dataclasses.dataclass
class State:
    """One observed state k: per-object rigid transforms, env map, cameras."""
    R: np.ndarray        # [M,3,3] f32 row-major rotations
    t: np.ndarray        # [M,3]   f32
    env: np.ndarray      # [H,W,3] f32, scene-linear, row 0 at +Y
    cameras: List[Camera]


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    states: List[State]
    k: int
    spp: int
    seed: int                 # tracer seed
    no_secondary: bool = False
    target_scene: Optional[Scene] = None   # C3: perturbed-parameter target
    target_envs: Optional[List[np.ndarray]] = None


# ----------------------------------------------------------------------------
# primitive draws
# ----------------------------------------------------------------------------

def uniform_quaternions(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random unit quaternions (Shoemake 1992), returned as (w,x,y,z)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1.0 - u1)
    b = np.sqrt(u1)
    x = a * np.sin(2 * np.pi * u2)
    y = a * np.cos(2 * np.pi * u2)
    z = b * np.sin(2 * np.pi * u3)
    w = b * np.cos(2 * np.pi * u3)
    return np.stack([w, x, y, z], axis=1)


def quat_to_matrix_np(q: np.ndarray) -> np.ndarray:
    """Rotation matrices of unit quaternions (w,x,y,z); used here only to draw
    rigid object transforms."""
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def matrix_to_quaternion_np(R: np.ndarray) -> np.ndarray:
    """Unit quaternion (w,x,y,z) of rotation matrices [...,3,3] (Shepperd's
    branch on the largest diagonal term); used to encode drawn surfel frames."""
    R = np.asarray(R, dtype=np.float64)
    m00, m11, m22 = R[..., 0, 0], R[..., 1, 1], R[..., 2, 2]
    tr = m00 + m11 + m22
    out = np.empty(R.shape[:-2] + (4,))
    c0 = tr > 0
    c1 = (~c0) & (m00 >= m11) & (m00 >= m22)
    c2 = (~c0) & (~c1) & (m11 >= m22)
    c3 = (~c0) & (~c1) & (~c2)
    s = np.sqrt(np.maximum(tr[c0] + 1.0, 1e-300)) * 2
    out[c0, 0] = 0.25 * s
    out[c0, 1] = (R[c0, 2, 1] - R[c0, 1, 2]) / s
    out[c0, 2] = (R[c0, 0, 2] - R[c0, 2, 0]) / s
    out[c0, 3] = (R[c0, 1, 0] - R[c0, 0, 1]) / s
    s = np.sqrt(np.maximum(1.0 + m00[c1] - m11[c1] - m22[c1], 1e-300)) * 2
    out[c1, 0] = (R[c1, 2, 1] - R[c1, 1, 2]) / s
    out[c1, 1] = 0.25 * s
    out[c1, 2] = (R[c1, 0, 1] + R[c1, 1, 0]) / s
    out[c1, 3] = (R[c1, 0, 2] + R[c1, 2, 0]) / s
    s = np.sqrt(np.maximum(1.0 + m11[c2] - m00[c2] - m22[c2], 1e-300)) * 2
    out[c2, 0] = (R[c2, 0, 2] - R[c2, 2, 0]) / s
    out[c2, 1] = (R[c2, 0, 1] + R[c2, 1, 0]) / s
    out[c2, 2] = 0.25 * s
    out[c2, 3] = (R[c2, 1, 2] + R[c2, 2, 1]) / s
    s = np.sqrt(np.maximum(1.0 + m22[c3] - m00[c3] - m11[c3], 1e-300)) * 2
    out[c3, 0] = (R[c3, 1, 0] - R[c3, 0, 1]) / s
    out[c3, 1] = (R[c3, 0, 2] + R[c3, 2, 0]) / s
    out[c3, 2] = (R[c3, 1, 2] + R[c3, 2, 1]) / s
    out[c3, 3] = 0.25 * s
    return out / np.linalg.norm(out, axis=-1, keepdims=True)


def unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def common_attributes(rng: np.random.Generator, n: int) -> dict:
    opacity = 1.0 / (1.0 + np.exp(-rng.standard_normal(n)))
    scale = np.exp(rng.uniform(np.log(0.01), np.log(0.1), size=(n, 2)))
    albedo = rng.random((n, 3))
    roughness = rng.random(n)
    metallic = rng.random(n)
    return dict(opacity=opacity, scale=scale, albedo=albedo,
                roughness=roughness, metallic=metallic)


def _pack(mu, q, attrs, object_offset) -> Scene:
    return Scene(mu=np.ascontiguousarray(mu, dtype=F32),
                 q=np.ascontiguousarray(q, dtype=F32),
                 scale=np.ascontiguousarray(attrs["scale"], dtype=F32),
                 opacity=np.ascontiguousarray(attrs["opacity"], dtype=F32),
                 albedo=np.ascontiguousarray(attrs["albedo"], dtype=F32),
                 roughness=np.ascontiguousarray(attrs["roughness"], dtype=F32),
                 metallic=np.ascontiguousarray(attrs["metallic"], dtype=F32),
                 object_offset=np.asarray(object_offset, dtype=np.int64))


def _tangent_basis(n: np.ndarray):
    """Any orthonormal tangent pair for unit normals n [N,3]."""
    helper = np.where(np.abs(n[:, :1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    t1 = np.cross(helper, n)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(n, t1)
    return t1, t2


def surface_samples(rng: np.random.Generator, n: int, n_shapes: int,
                    centre_lo: float, centre_hi: float,
                    sphere_radius=(0.15, 0.5), plane_side=(0.5, 1.5),
                    tilt_deg: float = 10.0, offset_sigma: float = 0.005):
    """Surface-like surfel centres and orientations on random spheres and
    square plane patches; surfels are allocated to shapes by area, centres are
    uniform on the surface plus a normal offset N(0, offset_sigma^2), and each
    surfel normal is the surface normal tilted by N(0, tilt^2) per tangent axis
    with a uniform in-plane rotation."""
    kinds = rng.random(n_shapes) < 0.5  # True = sphere
    centres = rng.uniform(centre_lo, centre_hi, size=(n_shapes, 3))
    radii = rng.uniform(*sphere_radius, size=n_shapes)
    pnormals = unit_vectors(rng, n_shapes)
    sides = rng.uniform(*plane_side, size=n_shapes)
    area = np.where(kinds, 4 * np.pi * radii ** 2, sides ** 2)
    counts = np.floor(area / area.sum() * n).astype(np.int64)
    rem = n - counts.sum()
    if rem > 0:
        extra = rng.choice(n_shapes, size=rem, p=area / area.sum())
        np.add.at(counts, extra, 1)
    shape_of = np.repeat(np.arange(n_shapes), counts)
    rng.shuffle(shape_of)
    pos = np.empty((n, 3))
    nrm = np.empty((n, 3))
    sph = kinds[shape_of]
    ns = int(sph.sum())
    if ns:
        dirs = unit_vectors(rng, ns)
        pos[sph] = centres[shape_of[sph]] + radii[shape_of[sph], None] * dirs
        nrm[sph] = dirs
    npl = n - ns
    if npl:
        idx = shape_of[~sph]
        pn = pnormals[idx]
        t1, t2 = _tangent_basis(pn)
        uv = rng.uniform(-0.5, 0.5, size=(npl, 2)) * sides[idx, None]
        pos[~sph] = centres[idx] + uv[:, :1] * t1 + uv[:, 1:] * t2
        nrm[~sph] = pn
    pos += nrm * rng.normal(0.0, offset_sigma, size=(n, 1))
    t1, t2 = _tangent_basis(nrm)
    tilt = np.deg2rad(tilt_deg)
    e = rng.normal(0.0, tilt, size=(n, 2))
    n2 = nrm + e[:, :1] * t1 + e[:, 1:] * t2
    n2 /= np.linalg.norm(n2, axis=1, keepdims=True)
    b1, b2 = _tangent_basis(n2)
    psi = rng.uniform(0, 2 * np.pi, size=(n, 1))
    tu = np.cos(psi) * b1 + np.sin(psi) * b2
    tv = np.cross(n2, tu)
    R = np.stack([tu, tv, n2], axis=2)  # columns t_u, t_v, n
    q = matrix_to_quaternion_np(R)
    return pos, q


def lognormal_env(rng: np.random.Generator, h: int = 256, w: int = 512,
                  lobe_gain: float = 1000.0, lobe_width: float = 0.05) -> np.ndarray:
    """Lat-long RGB env: texels i.i.d. lognormal(0,1) plus one bright lobe
    gain*exp((cos(gamma)-1)/width^2) about a uniform direction.  Row r spans
    polar angle [r, r+1)*pi/h from +Y; column c spans azimuth [c, c+1)*2pi/w
    measured from +X towards +Z."""
    env = np.exp(rng.standard_normal((h, w, 3)))
    lobe = unit_vectors(rng, 1)[0]
    th = (np.arange(h) + 0.5) * np.pi / h
    ph = (np.arange(w) + 0.5) * 2 * np.pi / w
    st, ct = np.sin(th)[:, None], np.cos(th)[:, None]
    dx, dy, dz = st * np.cos(ph)[None, :], ct * np.ones((1, w)), st * np.sin(ph)[None, :]
    cosg = dx * lobe[0] + dy * lobe[1] + dz * lobe[2]
    env += (lobe_gain * np.exp((cosg - 1.0) / lobe_width ** 2))[..., None]
    return np.ascontiguousarray(env, dtype=F32)


def constant_env(value: float = 1.0, h: int = 16, w: int = 32) -> np.ndarray:
    return np.full((h, w, 3), value, dtype=F32)


def look_at_camera(eye: np.ndarray, w: int, h: int, fov_y_deg: float = 60.0,
                   target=(0.0, 0.0, 0.0)) -> Camera:
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up_w = np.array([0.0, 1.0, 0.0]) if abs(fwd[1]) < 0.999 else np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up_w)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    back = -fwd
    pose = np.zeros((3, 4))
    pose[:, 0], pose[:, 1], pose[:, 2], pose[:, 3] = right, up, back, eye
    return Camera(pose=np.ascontiguousarray(pose.reshape(-1), dtype=F32),
                  fov_y_deg=float(fov_y_deg), w=int(w), h=int(h))


def sphere_camera(rng: np.random.Generator, w: int, h: int, radius: float = 3.0,
                  fov_y_deg: float = 60.0) -> Camera:
    return look_at_camera(radius * unit_vectors(rng, 1)[0], w, h, fov_y_deg)


def random_rigid(rng: np.random.Generator, m: int, t_lo=-1.0, t_hi=1.0):
    R = quat_to_matrix_np(uniform_quaternions(rng, m))
    t = rng.uniform(t_lo, t_hi, size=(m, 3))
    return R.astype(F32), t.astype(F32)


def identity_transforms(m: int):
    return np.tile(np.eye(3, dtype=F32), (m, 1, 1)), np.zeros((m, 3), dtype=F32)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------

def volume_scene(rng: np.random.Generator, n: int) -> Scene:
    mu = rng.uniform(-1.0, 1.0, size=(n, 3))
    q = uniform_quaternions(rng, n)
    return _pack(mu, q, common_attributes(rng, n), [0, n])


def surface_scene(rng: np.random.Generator, n: int, n_shapes: int = 20,
                  lo: float = -1.0, hi: float = 1.0) -> Scene:
    mu, q = surface_samples(rng, n, n_shapes, lo, hi)
    return _pack(mu, q, common_attributes(rng, n), [0, n])


def instanced_scene(rng: np.random.Generator, n_background: int, n_objects: int,
                    n_per_object: int, bg_lo=-1.5, bg_hi=1.5) -> Scene:
    """Background on 20 shapes plus objects made of 1-3 small shapes each,
    generated in object space around the object origin."""
    mus, qs = [], []
    mu, q = surface_samples(rng, n_background, 20, bg_lo, bg_hi)
    mus.append(mu)
    qs.append(q)
    for _ in range(n_objects):
        ns = int(rng.integers(1, 4))
        mu, q = surface_samples(rng, n_per_object, ns, -0.2, 0.2,
                                sphere_radius=(0.1, 0.25), plane_side=(0.2, 0.5))
        mus.append(mu)
        qs.append(q)
    n = n_background + n_objects * n_per_object
    offsets = [0, n_background] + [n_background + (o + 1) * n_per_object for o in range(n_objects)]
    return _pack(np.concatenate(mus), np.concatenate(qs), common_attributes(rng, n), offsets)


def perturb_scene(rng: np.random.Generator, scene: Scene) -> Scene:
    """Target parameters for the training step: mu += N(0,0.005^2);
    q += N(0,0.02^2) then renormalised; log s += N(0,0.05^2);
    logit alpha += N(0,0.2^2); a, r, m += N(0,0.05^2) clamped to [0,1]."""
    n = scene.n
    out = scene.copy()
    out.mu = (scene.mu + rng.normal(0, 0.005, (n, 3))).astype(F32)
    q = scene.q.astype(np.float64) + rng.normal(0, 0.02, (n, 4))
    out.q = (q / np.linalg.norm(q, axis=1, keepdims=True)).astype(F32)
    out.scale = np.exp(np.log(scene.scale.astype(np.float64)) + rng.normal(0, 0.05, (n, 2))).astype(F32)
    a = np.clip(scene.opacity.astype(np.float64), 1e-6, 1 - 1e-6)
    logit = np.log(a / (1 - a)) + rng.normal(0, 0.2, n)
    out.opacity = (1 / (1 + np.exp(-logit))).astype(F32)
    out.albedo = np.clip(scene.albedo + rng.normal(0, 0.05, (n, 3)), 0, 1).astype(F32)
    out.roughness = np.clip(scene.roughness + rng.normal(0, 0.05, n), 0, 1).astype(F32)
    out.metallic = np.clip(scene.metallic + rng.normal(0, 0.05, n), 0, 1).astype(F32)
    return out


def make_workload(i: int, scale: float = 1.0, resolution: Optional[int] = None) -> Workload:
    """Workload i in 1..5 (seed i, tracer seed 1000+i).  `scale` shrinks the
    surfel count (parity tests at reduced size keep the same recipe);
    `resolution` overrides the image side."""
    rng = np.random.default_rng(i)

    def ns(n):
        return max(1, int(round(n * scale)))

    if i == 1:
        scene = volume_scene(rng, ns(4096))
        res = resolution or 64
        cam = sphere_camera(rng, res, res)
        M = scene.n_objects
        R, t = identity_transforms(M)
        st = State(R=R, t=t, env=constant_env(1.0), cameras=[cam])
        return Workload("C1 primary-only 4k surfels 64x64", scene, [st], k=16, spp=1,
                        seed=1001, no_secondary=True)
    if i == 2:
        scene = surface_scene(rng, ns(200_000))
        res = resolution or 800
        env = lognormal_env(rng)
        cam = sphere_camera(rng, res, res)
        R, t = identity_transforms(0)
        return Workload("C2 one-bounce 200k surfels 800x800", scene,
                        [State(R=R, t=t, env=env, cameras=[cam])], k=32, spp=1, seed=1002)
    if i == 3:
        scene = surface_scene(rng, ns(300_000))
        res = resolution or 800
        env = lognormal_env(rng)
        cams = [sphere_camera(rng, res, res) for _ in range(4)]
        R, t = identity_transforms(0)
        prng = np.random.default_rng(2000)
        target = perturb_scene(prng, scene)
        tenv = (env * np.exp(prng.normal(0, 0.1, env.shape))).astype(F32)
        return Workload("C3 training step 300k surfels 4x800x800", scene,
                        [State(R=R, t=t, env=env, cameras=cams)], k=32, spp=1, seed=1003,
                        target_scene=target, target_envs=[tenv])
    if i == 4:
        scene = instanced_scene(rng, ns(500_000), 8, ns(20_000))
        res = resolution or 1024
        states = []
        for _k in range(4):
            R, t = random_rigid(rng, 8)
            env = lognormal_env(rng)
            states.append(State(R=R, t=t, env=env, cameras=[sphere_camera(rng, res, res)]))
        return Workload("C4 multi-state 660k surfels 4x1024x1024 S=4", scene, states,
                        k=32, spp=4, seed=1004)
    if i == 5:
        scene = instanced_scene(rng, ns(760_000), 8, ns(30_000))
        res = resolution or 1024
        R, t = random_rigid(rng, 8)
        env = lognormal_env(rng)
        st = State(R=R, t=t, env=env, cameras=[sphere_camera(rng, res, res)])
        return Workload("C5 resident 1M surfels 1024x1024", scene, [st], k=32, spp=4, seed=1005)
    raise ValueError(f"workload {i} not in 1..5")


@dataclasses.dataclass
class Request:
    arrival_s: float
    R: np.ndarray
    t: np.ndarray
    env: np.ndarray
    camera: Camera
    spp: int
    seed: int


def request_stream(n_objects: int, n_requests: int, rate_per_s: float, seed: int = 5,
                   resolutions=(256, 512, 1024), spps=(1, 4), env_hw=(256, 512)) -> List[Request]:
    """Poisson arrivals at `rate_per_s`; each request draws a new rigid transform
    per object, a new lognormal env, a resolution and a secondary count."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        R, tr = random_rigid(rng, n_objects)
        env = lognormal_env(rng, env_hw[0], env_hw[1])
        res = int(rng.choice(resolutions))
        spp = int(rng.choice(spps))
        cam = sphere_camera(rng, res, res)
        out.append(Request(arrival_s=t, R=R, t=tr, env=env, camera=cam, spp=spp,
                           seed=10_000 + j))
    return out
