"""Closed-form geometry used by the oracle's pins (binary64, independent of
both the oracle and the HIP path)."""
import math

import numpy as np


def camera_rays_f64(sc):
    """Pixel-centre camera rays in binary64 from the scene's binary32 camera vectors."""
    W, H = sc.width, sc.height
    x, y = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    sx = 2.0 * x / W - 1.0
    sy = 1.0 - 2.0 * y / H
    f, r, u = (np.asarray(v, np.float64) for v in (sc.fwd, sc.right, sc.up))
    d = f[None, None, :] + sx[..., None] * r[None, None, :] + sy[..., None] * u[None, None, :]
    d /= np.linalg.norm(d, axis=-1, keepdims=True)
    return np.asarray(sc.eye, np.float64), d


def plane_hits(sc, z=0.0):
    """Points where the pixel-centre rays meet the plane of height z, [H][W][3]."""
    o, d = camera_rays_f64(sc)
    t = (z - o[2]) / d[..., 2]
    return o[None, None, :] + t[..., None] * d


def polygon_form_factor(p, n, verts):
    """Point-to-polygon form factor (Lambert's formula): the fraction of the
    cosine-weighted hemisphere of the unit normal n at p that the planar
    polygon `verts` ([m][3], in order around its boundary, wholly above the
    tangent plane of p) covers,
        F = (1 / 2 pi) |sum_i gamma_i  n . unit(a_i x a_{i+1})|
    with a_i the unit vector from p to vertex i and gamma_i the angle between
    consecutive ones."""
    p = np.asarray(p, np.float64)
    n = np.asarray(n, np.float64)
    a = np.asarray(verts, np.float64) - p
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    total = 0.0
    m = a.shape[0]
    for i in range(m):
        u, v = a[i], a[(i + 1) % m]
        c = np.cross(u, v)
        gamma = math.acos(max(-1.0, min(1.0, float(u @ v))))
        total += gamma * float(n @ (c / np.linalg.norm(c)))
    return abs(total) / (2.0 * math.pi)


def parallelogram(o, e1, e2):
    """The four corners of the parallelogram o + [0,1] e1 + [0,1] e2, in order."""
    o, e1, e2 = (np.asarray(v, np.float64) for v in (o, e1, e2))
    return np.stack([o, o + e1, o + e1 + e2, o + e2])
