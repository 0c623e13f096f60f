"""Disc surfels (Eq. 4) for a synthetic keyframe: centres on a square
lattice, ground truth from the scene's planes, perturbed starting states, and
holes in the lattice that leave empty areas for the placement of new
surfels.

The paper's evaluation uses 640x480 images with surfels of radius 10 px
(System evaluation section); the lattice step defaults to floor(r sqrt 2), the
largest integer step at which discs of radius r centred on the lattice cover
the image.  Like the rest of this package it draws numbers and reads the
scene; it holds none of the method's arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Tuple

import numpy as np

from .scene import Keyframe, _perturb


@dataclass
class DiscSet:
    radius: float
    spacing: int
    ux: np.ndarray               # (m,) float32 centres (pixels)
    uy: np.ndarray
    gt_id: np.ndarray            # (m,) float64 inverse depth of the true plane at the centre ray
    gt_n: np.ndarray             # (m, 3) float64
    init_id: np.ndarray          # (m,) float32
    init_n: np.ndarray           # (m, 3) float32
    pure: np.ndarray             # (m,) bool: every pixel of the disc sees the centre's plane
    holes: Tuple[Tuple[int, int, int, int], ...]   # removed lattice rectangles x0, y0, x1, y1


def lattice(width: int, height: int, spacing: int):
    """Pixels (spacing/2 + i spacing, spacing/2 + j spacing) inside the image,
    row by row."""
    xs = np.arange(spacing // 2, width, spacing)
    ys = np.arange(spacing // 2, height, spacing)
    yy, xx = np.meshgrid(ys, xs, indexing="ij")
    return xx.reshape(-1), yy.reshape(-1)


def make_disc_surfels(kf: Keyframe, radius: float = 10.0, spacing: int = 0, n_holes: int = 3,
                      hole_frac: Tuple[float, float] = (0.08, 0.18), seed: int = 0,
                      depth_noise: float = None, normal_deg: float = None) -> DiscSet:
    """Disc surfels of keyframe `kf` on the lattice of step `spacing`
    (default floor(r sqrt 2)), minus `n_holes` random rectangles whose sides
    are hole_frac of the image's; starting states perturbed like the tile
    workloads (the keyframe spec's noise unless given)."""
    spacing = int(spacing) if spacing else int(math.floor(radius * math.sqrt(2.0)))
    rng = np.random.default_rng(int(kf.spec.seed) * 1009 + 7 + int(seed))
    W, H = kf.width, kf.height
    xs, ys = lattice(W, H, spacing)
    holes = []
    keep = np.ones(xs.size, bool)
    for _ in range(n_holes):
        hw = int(rng.uniform(*hole_frac) * W)
        hh = int(rng.uniform(*hole_frac) * H)
        x0 = int(rng.integers(0, max(1, W - hw)))
        y0 = int(rng.integers(0, max(1, H - hh)))
        holes.append((x0, y0, x0 + hw, y0 + hh))
        keep &= ~((xs >= x0) & (xs < x0 + hw) & (ys >= y0) & (ys < y0 + hh))
    xs, ys = xs[keep], ys[keep]
    fx, fy, cx, cy = kf.K
    pid = kf.kf_plane_id[ys, xs].astype(np.int64)
    Nn = np.stack([p.n for p in kf.planes])[pid]
    P0 = np.stack([p.p0 for p in kf.planes])[pid]
    r = np.stack([(xs - cx) / fx, (ys - cy) / fy, np.ones(xs.size)], 1)
    gt_id = (Nn * r).sum(1) / (Nn * P0).sum(1)
    # purity: all pixels within r of the centre hit the centre's plane
    R = int(math.ceil(radius))
    off = np.array([(dx, dy) for dy in range(-R, R + 1) for dx in range(-R, R + 1)
                    if dx * dx + dy * dy < radius * radius])
    px = np.clip(xs[:, None] + off[None, :, 0], 0, W - 1)
    py = np.clip(ys[:, None] + off[None, :, 1], 0, H - 1)
    pure = (kf.kf_plane_id[py, px] == pid[:, None]).all(1)
    dn = kf.spec.init_depth_noise if depth_noise is None else depth_noise
    ndeg = kf.spec.init_normal_deg if normal_deg is None else normal_deg
    init_id, init_n = _perturb(rng, gt_id[None, :], Nn[None, :, :], dn, ndeg)
    return DiscSet(radius=float(radius), spacing=spacing, ux=xs.astype(np.float32),
                   uy=ys.astype(np.float32), gt_id=gt_id, gt_n=Nn.copy(),
                   init_id=init_id.reshape(-1), init_n=init_n.reshape(-1, 3), pure=pure,
                   holes=tuple(holes))
