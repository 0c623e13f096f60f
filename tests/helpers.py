"""Independent test-side constructions (numpy / scipy only).

Nothing here calls the oracle or the device library: these are the second
routes that the oracle's pins compare against.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import ndimage


def kmat(K):
    fx, fy, cx, cy = K
    return np.array([[fx, 0.0, cx], [0.0, fy, cy], [0.0, 0.0, 1.0]])


def plane_homography(K, R, t, n, d):
    """Plane-induced homography for the plane {X : n.X = d} (keyframe
    coordinates) and the pose X' = R X + t:  x' ~ K (R + t n^T / d) K^-1 x."""
    Km = kmat(K)
    return Km @ (np.asarray(R) + np.outer(t, n) / d) @ np.linalg.inv(Km)


def apply_h(Hm, x, y):
    v = Hm @ np.array([x, y, 1.0])
    return v[0] / v[2], v[1] / v[2]


def bilinear_scipy(img, x, y):
    """Bilinear interpolation through scipy's order-1 spline."""
    return float(ndimage.map_coordinates(np.asarray(img, np.float64), [[y], [x]], order=1,
                                         mode="nearest", prefilter=False)[0])


def bilinear_scipy_many(img, xs, ys):
    return ndimage.map_coordinates(np.asarray(img, np.float64), [np.asarray(ys), np.asarray(xs)],
                                   order=1, mode="nearest", prefilter=False)


def smooth_texture(W, H, seed, periods=(12.0, 40.0), count=6, x0=0.0, y0=0.0):
    """Sum of random sinusoids in pixel coordinates, evaluated on an integer
    grid offset by (x0, y0)."""
    rng = np.random.default_rng(seed)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.float64)
    xs = xs + x0
    ys = ys + y0
    out = np.full((H, W), 0.5)
    for _ in range(count):
        ang = rng.uniform(0, 2 * math.pi)
        per = math.exp(rng.uniform(math.log(periods[0]), math.log(periods[1])))
        ph = rng.uniform(0, 2 * math.pi)
        out += (0.4 / count) * np.sin(2 * math.pi * (math.cos(ang) * xs + math.sin(ang) * ys) / per + ph)
    return out


def huber(r, k):
    a = abs(r)
    return 0.5 * r * r if a <= k else k * a - 0.5 * k * k


def ray(K, x, y):
    fx, fy, cx, cy = K
    return np.array([(x - cx) / fx, (y - cy) / fy, 1.0])


def angle_deg(n1, n2):
    n1 = np.asarray(n1, np.float64).reshape(-1, 3)
    n2 = np.asarray(n2, np.float64).reshape(-1, 3)
    c = np.linalg.norm(np.cross(n1, n2), axis=1)
    d = np.abs((n1 * n2).sum(1))
    return np.degrees(np.arctan2(c, d))


def random_unit_cap(rng, deg=40.0):
    cth = rng.uniform(math.cos(math.radians(deg)), 1.0)
    sth = math.sqrt(1 - cth * cth)
    phi = rng.uniform(0, 2 * math.pi)
    return np.array([sth * math.cos(phi), sth * math.sin(phi), -cth])


def rot(axis, ang):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(ang) * k + (1 - math.cos(ang)) * (k @ k)
