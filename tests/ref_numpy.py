"""A second, tiny, independent re-implementation of the tracing steps (world
transform, plane intersection, support and opacity culling, (t, index) sort,
k truncation and front-to-back compositing; Sec. 3.1-3.2,
Eq. state-assembly, Eq. gaussian-response, Eq. surface-record) in NumPy.

It is deliberately written along a different route from the C oracle: surfel
frames come from the quaternion sandwich product q v q* (Hamilton product)
instead of the rotation-matrix formula, object transforms are applied as
quaternion compositions, and everything is vectorised over surfels.  It is
used only to cross-check the oracle on small inputs.
"""
import numpy as np


def hamilton(a, b):
    aw, ax, ay, az = np.moveaxis(a, -1, 0)
    bw, bx, by, bz = np.moveaxis(b, -1, 0)
    return np.stack([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def rotate(q, v):
    """Rotate vectors v [...,3] by unit quaternions q [...,4] via q v q*."""
    vq = np.concatenate([np.zeros(v.shape[:-1] + (1,)), v], axis=-1)
    qc = q * np.array([1.0, -1.0, -1.0, -1.0])
    return hamilton(hamilton(q, vq), qc)[..., 1:]


def matrix_to_quat(R):
    """Quaternion of a proper rotation (Shepperd), used for object transforms."""
    R = np.asarray(R, dtype=np.float64)
    tr = np.trace(R)
    cands = [tr, R[0, 0], R[1, 1], R[2, 2]]
    k = int(np.argmax(cands))
    if k == 0:
        s = np.sqrt(tr + 1.0) * 2
        q = [0.25 * s, (R[2, 1] - R[1, 2]) / s, (R[0, 2] - R[2, 0]) / s, (R[1, 0] - R[0, 1]) / s]
    elif k == 1:
        s = np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2]) * 2
        q = [(R[2, 1] - R[1, 2]) / s, 0.25 * s, (R[0, 1] + R[1, 0]) / s, (R[0, 2] + R[2, 0]) / s]
    elif k == 2:
        s = np.sqrt(1.0 + R[1, 1] - R[0, 0] - R[2, 2]) * 2
        q = [(R[0, 2] - R[2, 0]) / s, (R[0, 1] + R[1, 0]) / s, 0.25 * s, (R[1, 2] + R[2, 1]) / s]
    else:
        s = np.sqrt(1.0 + R[2, 2] - R[0, 0] - R[1, 1]) * 2
        q = [(R[1, 0] - R[0, 1]) / s, (R[0, 2] + R[2, 0]) / s, (R[1, 2] + R[2, 1]) / s, 0.25 * s]
    q = np.array(q)
    return q / np.linalg.norm(q)


def world_surfels(scene, R, t):
    q = scene.q.astype(np.float64)
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    mu = scene.mu.astype(np.float64).copy()
    off = scene.object_offset
    for o in range(len(off) - 2):
        a, b = off[o + 1], off[o + 2]
        Ro = np.asarray(R[o], dtype=np.float64)
        # same orthonormalisation of the FP32 rotation as the method's reading
        c0 = Ro[:, 0] / np.linalg.norm(Ro[:, 0])
        c1 = Ro[:, 1] - np.dot(c0, Ro[:, 1]) * c0
        c1 /= np.linalg.norm(c1)
        Rn = np.stack([c0, c1, np.cross(c0, c1)], axis=1)
        qo = matrix_to_quat(Rn)
        q[a:b] = hamilton(np.broadcast_to(qo, (b - a, 4)), q[a:b])
        mu[a:b] = mu[a:b] @ Rn.T + np.asarray(t[o], dtype=np.float64)
    ex = np.broadcast_to(np.array([1.0, 0, 0]), mu.shape)
    ey = np.broadcast_to(np.array([0, 1.0, 0]), mu.shape)
    ez = np.broadcast_to(np.array([0, 0, 1.0]), mu.shape)
    return mu, rotate(q, ex), rotate(q, ey), rotate(q, ez)


def trace(scene, R, t, o, d, k, alpha_min=1 / 255, alpha_cap=0.99, sigma=3.0, eps=1e-6, t_min=1e-4):
    """Returns hit lists [n,k] (-1 padded), A, T, depth, normal for rays (o, d)."""
    mu, tu, tv, nn = world_surfels(scene, R, t)
    su = scene.scale[:, 0].astype(np.float64)
    sv = scene.scale[:, 1].astype(np.float64)
    al = scene.opacity.astype(np.float64)
    r2max = np.minimum(sigma * sigma, 2.0 * np.log(al / alpha_min))
    nr = o.shape[0]
    hits = -np.ones((nr, k), dtype=np.int64)
    A = np.zeros(nr)
    T = np.ones(nr)
    depth = np.zeros(nr)
    normal = np.zeros((nr, 3))
    for r in range(nr):
        orr = o[r].astype(np.float64)
        dr = d[r].astype(np.float64)
        den = nn @ dr
        ok = np.abs(den) >= 1e-12
        with np.errstate(divide="ignore", invalid="ignore"):
            tt = np.einsum("ij,ij->i", nn, mu - orr) / den
        x = orr + tt[:, None] * dr
        rel = x - mu
        xi_u = np.einsum("ij,ij->i", rel, tu) / su
        xi_v = np.einsum("ij,ij->i", rel, tv) / sv
        rho2 = xi_u ** 2 + xi_v ** 2
        valid = ok & (tt > t_min) & (rho2 <= r2max)
        idx = np.nonzero(valid)[0]
        order = idx[np.lexsort((idx, tt[idx]))][:k]
        hits[r, :len(order)] = order
        at = np.minimum(alpha_cap, al[order] * np.exp(-0.5 * rho2[order]))
        trans = np.concatenate([[1.0], np.cumprod(1.0 - at)])
        w = trans[:-1] * at
        A[r] = w.sum()
        T[r] = trans[-1]
        face = np.where((den[order] > 0)[:, None], -nn[order], nn[order])
        depth[r] = (w * tt[order]).sum() / (A[r] + eps)
        nbar = (w[:, None] * face).sum(0) / (A[r] + eps)
        ln = np.linalg.norm(nbar)
        normal[r] = nbar / ln if (len(order) and ln > 0) else 0.0
    return hits, A, T, depth, normal
