"""FP64 reference of the training objectives (geometry refinement, environment TV) and their gradients.

TEST INFRASTRUCTURE ONLY: imported by tests and by the benchmark's CPU leg,
never by the GPU library or its binding.  Every function is the plain
definition of one objective written out in NumPy float64, with the gradient
by the chain rule; nothing is blocked, fused or reordered.

  l1_loss            Sec. 3.4, Eq. training-objectives (scene-linear HDR data term)
  coverage_loss      Sec. 3.1, Eq. alpha-coverage
  scale_loss         Sec. 3.1, Eq. scale-regularization
  depth_loss         Sec. 3.2, Eq. reconstruction-depth
  normal_loss        Sec. 3.2, Eq. reconstruction-normal (rendered normal)
  depth_normals      the depth-derived normal map of Eq. reconstruction-normal
  depth_normal_loss  Sec. 3.2, Eq. reconstruction-normal (depth-derived normal)
  tv_loss            Sec. 3.4, Eq. training-objectives (L_TV of the environment map)

Readings of points the paper leaves open:
  * sign(0) = 0 in every L1 gradient;
  * the data term is the mean over every pixel and colour channel of the
    absolute difference of the linear (not tonemapped) radiances;
  * the infinity norm of the scale pair is max(|s_u|, |s_v|); its gradient
    goes to the first component attaining the maximum;
  * the confidence enters the depth objective as |C| (the L1 norm of C*x);
  * the depth-derived normal at pixel (x, y) is the unit vector along
    (P(x+1,y) - P(x-1,y)) x (P(x,y-1) - P(x,y+1)), P = o + D d the point at
    the rendered depth along the pixel's ray (y = 0 is the top row), which
    faces the camera on a smooth surface; it is zero on the image border,
    where a neighbour has depth <= 0 (no surface), or where the cross
    product vanishes.  Both normal objectives average over all H*W pixels;
  * L_TV (not defined in the paper) is the anisotropic first-order total
    variation of the lat-long map: |E(y,x+1) - E(y,x)| with x wrapping
    around in azimuth, plus |E(y+1,x) - E(y,x)| for y < H-1 (no wrap over the
    poles), summed over channels and divided by 3 H W.
"""
from __future__ import annotations

import numpy as np


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def l1_loss(pred, target):
    """L1^HDR = (1/n) * sum |L - L*| over all n = pixels x channels values of
    the scene-linear radiance (Sec. 3.4, Eq. training-objectives, data term);
    returns (loss, dL/dpred) with the gradient sign(L - L*)/n."""
    p, t = _f64(pred).reshape(-1), _f64(target).reshape(-1)
    if p.shape != t.shape:
        raise ValueError("pred and target sizes differ")
    n = p.size
    if n == 0:
        return 0.0, np.zeros(0)
    r = p - t
    return float(np.abs(r).sum() / n), np.sign(r) / n


def coverage_loss(alpha):
    """L_alpha = (1/HW) * sum |A - 1| (Eq. alpha-coverage) over the accumulated
    opacity map alpha [H*W]; returns (loss, dL/dalpha)."""
    a = _f64(alpha).reshape(-1)
    n = a.size
    if n == 0:
        return 0.0, np.zeros(0)
    r = a - 1.0
    return float(np.abs(r).sum() / n), np.sign(r) / n


def scale_loss(scale, s_max):
    """L_s = (1/N) * sum_i max(0, ||s_i||_inf / s_max - 1)^2
    (Eq. scale-regularization) over in-plane scales [N,2]; returns
    (loss, dL/dscale [N,2])."""
    s = _f64(scale).reshape(-1, 2)
    n = s.shape[0]
    g = np.zeros_like(s)
    if n == 0:
        return 0.0, g
    mag = np.abs(s)
    j = np.argmax(mag, axis=1)  # first maximal component
    m = mag[np.arange(n), j]
    h = np.maximum(0.0, m / s_max - 1.0)
    g[np.arange(n), j] = 2.0 * h * np.sign(s[np.arange(n), j]) / (n * s_max)
    return float((h * h).sum() / n), g


def depth_loss(depth, ref, conf, eps):
    """L_D = ||C .* (D - D*)||_1 / (||C .* D*||_1 + eps)
    (Eq. reconstruction-depth); returns (loss, dL/ddepth)."""
    d, r, c = _f64(depth).reshape(-1), _f64(ref).reshape(-1), _f64(conf).reshape(-1)
    num = np.abs(c * (d - r)).sum()
    den = np.abs(c * r).sum() + eps
    return float(num / den), np.abs(c) * np.sign(d - r) / den


def normal_loss(normal, ref):
    """L_N = 1 - (1/HW) <N, N*>_F (Eq. reconstruction-normal) over normal
    maps [H*W,3]; returns (loss, dL/dnormal)."""
    nrm, r = _f64(normal).reshape(-1, 3), _f64(ref).reshape(-1, 3)
    n = nrm.shape[0]
    if n == 0:
        return 0.0, np.zeros((0, 3))
    return float(1.0 - (nrm * r).sum() / n), -r / n


def _points(o, d, depth, h, w):
    return (_f64(o).reshape(h, w, 3) + _f64(depth).reshape(h, w, 1) * _f64(d).reshape(h, w, 3))


def depth_normals(o, d, depth, h, w):
    """Depth-derived normal map [H*W,3] of the rendered depth (ray parameter
    along the unit rays o, d of an h x w image, row-major)."""
    P = _points(o, d, depth, h, w)
    D = _f64(depth).reshape(h, w)
    N = np.zeros((h, w, 3))
    for y in range(1, h - 1):
        for x in range(1, w - 1):
            if min(D[y, x - 1], D[y, x + 1], D[y - 1, x], D[y + 1, x]) <= 0.0:
                continue
            a = P[y, x + 1] - P[y, x - 1]
            b = P[y - 1, x] - P[y + 1, x]
            c = np.cross(a, b)
            ln = np.linalg.norm(c)
            if ln > 0.0:
                N[y, x] = c / ln
    return N.reshape(-1, 3)


def depth_normal_loss(o, d, depth, ref, h, w):
    """L_DN = 1 - (1/HW) <N^D, N*>_F (Eq. reconstruction-normal) with N^D the
    depth-derived normal map; returns (loss, dL/ddepth [H*W]).

    The gradient follows the chain normalisation -> cross product -> central
    differences -> points P = o + D d, whose derivative in D is d."""
    P = _points(o, d, depth, h, w)
    D = _f64(depth).reshape(h, w)
    R = _f64(ref).reshape(h, w, 3)
    dd = _f64(d).reshape(h, w, 3)
    n = h * w
    if n == 0:
        return 0.0, np.zeros(0)
    dot = 0.0
    gP = np.zeros((h, w, 3))
    for y in range(1, h - 1):
        for x in range(1, w - 1):
            if min(D[y, x - 1], D[y, x + 1], D[y - 1, x], D[y + 1, x]) <= 0.0:
                continue
            a = P[y, x + 1] - P[y, x - 1]
            b = P[y - 1, x] - P[y + 1, x]
            c = np.cross(a, b)
            ln = np.linalg.norm(c)
            if not ln > 0.0:
                continue
            u = c / ln
            dot += float(u @ R[y, x])
            # d/dc of -(1/n) <c/|c|, r> = -(1/n) (r - u (u.r)) / |c|
            gc = -(R[y, x] - u * (u @ R[y, x])) / (ln * n)
            ga = np.cross(b, gc)  # (da x b).gc = da.(b x gc)
            gb = np.cross(gc, a)  # (a x db).gc = db.(gc x a)
            gP[y, x + 1] += ga
            gP[y, x - 1] -= ga
            gP[y - 1, x] += gb
            gP[y + 1, x] -= gb
    return 1.0 - dot / n, (gP * dd).sum(axis=2).reshape(-1)


def tv_loss(env):
    """L_TV of a lat-long environment map [H,W,3] (Eq. training-objectives):
    returns (loss, dL/denv [H,W,3])."""
    E = _f64(env)
    H, W = E.shape[:2]
    n = 3 * H * W
    if n == 0:
        return 0.0, np.zeros_like(E)
    g = np.zeros_like(E)
    total = 0.0
    for y in range(H):
        for x in range(W):
            for c in range(3):
                dh = E[y, (x + 1) % W, c] - E[y, x, c]
                total += abs(dh)
                g[y, (x + 1) % W, c] += np.sign(dh)
                g[y, x, c] -= np.sign(dh)
                if y + 1 < H:
                    dv = E[y + 1, x, c] - E[y, x, c]
                    total += abs(dv)
                    g[y + 1, x, c] += np.sign(dv)
                    g[y, x, c] -= np.sign(dv)
    return total / n, g / n
