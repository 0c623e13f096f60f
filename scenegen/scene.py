"""Synthetic piecewise-planar scenes of the paper's workload shape.

The paper evaluates on 640x480 grayscale sequences with surfels of about ten
pixels (System evaluation section).  Those sequences are not available, so
seeded scenes stand in for them:

* the keyframe is split (kd-split, boundaries on multiples of 8 px) into
  rectangles, each carrying one textured plane; configurations with a ground
  plane add it in the bottom quarter of the rows;
* plane depth at the rectangle's centre ray ~ U[1, 4] m, normal uniform on the
  40 degree cap around -z (towards the camera);
* texture = 0.5 + 1/16 * sum of 8 sinusoids in in-plane metric coordinates,
  periods log-uniform in [8, 64] px at the plane's depth;
* neighbour poses (keyframe -> neighbour, X_n = R X_kf + t): |t| = 0.05 m in a
  uniform direction, R a rotation of U[0, 2] degrees about a uniform axis;
* every image gets N(0, (2/255)^2) noise and is clamped to [0, 1];
* initial surfels: ground-truth inverse depth / U[0.9, 1.1] and the
  ground-truth normal rotated by U[0, 10] degrees about a uniform tangent axis;
  where requested the checkerboard-odd half of the grid is marked "new".

Only scene parameters are drawn with numpy; the rendering itself (ray/plane
intersection and texture evaluation) runs in torch float64 on the requested
device so that large batches can be produced quickly on a GPU.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

RESOLUTIONS_BATCH = ((320, 240), (640, 480), (1280, 720))
RESOLUTIONS_STREAM = ((320, 240), (640, 480), (1280, 720), (1920, 1080))


@dataclass
class SceneSpec:
    width: int
    height: int
    n_nbr: int
    patch: int                  # surfel tile edge S (pixels)
    iters: int
    n_rects: int                # textured planes in the kd-split region
    ground: bool                # bottom-quarter ground plane
    seed: int
    half_new: bool              # checkerboard-odd tiles are "new"
    K: Optional[Tuple[float, float, float, float]] = None  # fx, fy, cx, cy
    noise_sigma: float = 2.0 / 255.0
    init_depth_noise: float = 0.10
    init_normal_deg: float = 10.0
    trans: float = 0.05
    rot_deg: float = 2.0

    def intrinsics(self) -> Tuple[float, float, float, float]:
        if self.K is not None:
            return tuple(float(v) for v in self.K)
        f = 0.9375 * self.width
        return (f, f, self.width / 2.0, self.height / 2.0)


@dataclass
class Plane:
    n: np.ndarray               # unit normal (keyframe coordinates)
    p0: np.ndarray              # a point of the plane (texture origin)
    rect: Optional[Tuple[int, int, int, int]]  # keyframe pixel rect x0,y0,x1,y1 (None: unbounded)
    omega: np.ndarray           # (8, 2) spatial frequencies, cycles per metre
    phase: np.ndarray           # (8,)
    e1: np.ndarray = field(default=None)
    e2: np.ndarray = field(default=None)


@dataclass
class Keyframe:
    spec: SceneSpec
    K: Tuple[float, float, float, float]
    width: int
    height: int
    patch: int
    iters: int
    kf_image: torch.Tensor       # (H, W) float32
    nbr_images: torch.Tensor     # (N, H, W) float32
    R: np.ndarray                # (N, 3, 3) float64, keyframe -> neighbour
    t: np.ndarray                # (N, 3) float64
    gt_id: np.ndarray            # (gh, gw) float64
    gt_n: np.ndarray             # (gh, gw, 3) float64
    init_id: np.ndarray          # (gh, gw) float32
    init_n: np.ndarray           # (gh, gw, 3) float32
    is_new: np.ndarray           # (gh, gw) uint8
    kf_plane_id: np.ndarray      # (H, W) int16, plane index hit by each keyframe pixel
    nbr_plane_id: Optional[torch.Tensor] = None  # (N, H, W) int16
    planes: List[Plane] = field(default_factory=list)

    @property
    def grid(self) -> Tuple[int, int]:
        return (self.width // self.patch, self.height // self.patch)

    @property
    def n_nbr(self) -> int:
        return int(self.R.shape[0])

    @property
    def n_surfels(self) -> int:
        gw, gh = self.grid
        return gw * gh


def rotation_about(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rodrigues rotation matrix for a unit axis and an angle in radians."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    k = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * k + (1 - math.cos(angle)) * (k @ k)


def _unit(rng: np.random.Generator) -> np.ndarray:
    v = rng.normal(size=3)
    return v / np.linalg.norm(v)


def _tangent_basis(n: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    e = np.array([1.0, 0.0, 0.0]) if abs(n[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    b1 = e - np.dot(e, n) * n
    b1 /= np.linalg.norm(b1)
    return b1, np.cross(n, b1)


def _kd_split(rng, x0, y0, x1, y1, count, snap=8, min_side=16):
    rects = [(x0, y0, x1, y1)]
    guard = 0
    while len(rects) < count and guard < 10000:
        guard += 1
        rects.sort(key=lambda r: (r[2] - r[0]) * (r[3] - r[1]), reverse=True)
        rx0, ry0, rx1, ry1 = rects[0]
        w, h = rx1 - rx0, ry1 - ry0
        along_x = w >= h
        lo, hi = (rx0, rx1) if along_x else (ry0, ry1)
        cand = [v for v in range(lo + min_side, hi - min_side + 1, snap) if v % snap == 0]
        if not cand:
            break
        # keep the cut away from the extremes for a balanced split
        mid = len(cand)
        c = cand[int(rng.integers(max(0, mid // 4), max(1, mid - mid // 4)))]
        rects.pop(0)
        if along_x:
            rects += [(rx0, ry0, c, ry1), (c, ry0, rx1, ry1)]
        else:
            rects += [(rx0, ry0, rx1, c), (rx0, c, rx1, ry1)]
    rects.sort(key=lambda r: (r[1], r[0]))
    return rects


def _texture(rng, depth, f) -> Tuple[np.ndarray, np.ndarray]:
    ang = rng.uniform(0.0, 2.0 * math.pi, size=8)
    period_px = np.exp(rng.uniform(math.log(8.0), math.log(64.0), size=8))
    period_m = period_px * depth / f
    mag = 1.0 / period_m
    omega = np.stack([mag * np.cos(ang), mag * np.sin(ang)], axis=1)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=8)
    return omega, phase


def _make_planes(spec: SceneSpec, rng: np.random.Generator) -> List[Plane]:
    fx, fy, cx, cy = spec.intrinsics()
    W, H = spec.width, spec.height
    planes: List[Plane] = []
    top_h = H
    if spec.ground:
        top_h = int(round(0.75 * H / 8.0)) * 8
    rects = _kd_split(rng, 0, 0, W, top_h, spec.n_rects)
    cos_max = math.cos(math.radians(40.0))
    for (x0, y0, x1, y1) in rects:
        uc = 0.5 * (x0 + x1 - 1)
        vc = 0.5 * (y0 + y1 - 1)
        ray = np.array([(uc - cx) / fx, (vc - cy) / fy, 1.0])
        depth = rng.uniform(1.0, 4.0)
        cth = rng.uniform(cos_max, 1.0)
        sth = math.sqrt(max(0.0, 1.0 - cth * cth))
        phi = rng.uniform(0.0, 2.0 * math.pi)
        n = np.array([sth * math.cos(phi), sth * math.sin(phi), -cth])
        p0 = ray * depth
        omega, phase = _texture(rng, depth, fx)
        planes.append(Plane(n=n, p0=p0, rect=(x0, y0, x1, y1), omega=omega, phase=phase))
    if spec.ground:
        ytop = float(top_h)
        h = 4.0 * (ytop - cy) / fy
        n = np.array([0.0, -1.0, 0.0])
        p0 = np.array([0.0, h, 4.0])
        omega, phase = _texture(rng, 6.0, fx)
        planes.append(Plane(n=n, p0=p0, rect=(0, top_h, W, H), omega=omega, phase=phase))
    # unbounded fronto-parallel background, used only where no quad is hit
    omega, phase = _texture(rng, 6.0, fx)
    planes.append(Plane(n=np.array([0.0, 0.0, -1.0]), p0=np.array([0.0, 0.0, 6.0]),
                        rect=None, omega=omega, phase=phase))
    for p in planes:
        p.e1, p.e2 = _tangent_basis(p.n)
    return planes


def _render(planes: Sequence[Plane], K, W, H, R, t, device, noise_sigma, gen):
    """Ray-cast one view (pose X_cam = R X_kf + t) of the bounded planes,
    all planes at once."""
    fx, fy, cx, cy = K
    dt = torch.float64
    dev = torch.device(device)
    ys = torch.arange(H, device=dev, dtype=dt).view(H, 1).expand(H, W)
    xs = torch.arange(W, device=dev, dtype=dt).view(1, W).expand(H, W)
    dcam = torch.stack([(xs - cx) / fx, (ys - cy) / fy, torch.ones_like(xs)], dim=-1)
    Rt = torch.as_tensor(np.asarray(R).T.copy(), device=dev, dtype=dt)
    C = -(torch.as_tensor(np.asarray(R).T @ np.asarray(t), device=dev, dtype=dt))
    d = (dcam @ Rt.T).reshape(-1, 3)                 # ray directions, keyframe coordinates
    quads = [i for i, p in enumerate(planes) if p.rect is not None]
    bg_index = len(planes) - 1
    N = torch.as_tensor(np.stack([planes[i].n for i in quads]), device=dev, dtype=dt)      # (P,3)
    P0 = torch.as_tensor(np.stack([planes[i].p0 for i in quads]), device=dev, dtype=dt)    # (P,3)
    rects = torch.as_tensor(np.array([planes[i].rect for i in quads], dtype=np.float64), device=dev, dtype=dt)
    den = d @ N.T                                     # (M,P)
    num = ((P0 - C) * N).sum(1)                       # (P,)
    lam = num / den
    X = C.view(1, 1, 3) + lam.unsqueeze(-1) * d.unsqueeze(1)   # (M,P,3)
    Z = X[..., 2]
    ok = (lam > 0) & (Z > 1e-9) & torch.isfinite(lam)
    u = fx * X[..., 0] / Z + cx
    v = fy * X[..., 1] / Z + cy
    ok &= (u >= rects[:, 0] - 0.5) & (u < rects[:, 2] - 0.5) & (v >= rects[:, 1] - 0.5) & (v < rects[:, 3] - 0.5)
    lam_ok = torch.where(ok, lam, torch.full_like(lam, float("inf")))
    best, arg = lam_ok.min(dim=1)
    hit = torch.isfinite(best)
    qidx = torch.as_tensor(quads, device=dev, dtype=torch.int64)
    pid = torch.where(hit, qidx[arg], torch.full_like(arg, bg_index))
    # texture of the winning plane at its hit point
    allN = torch.as_tensor(np.stack([p.n for p in planes]), device=dev, dtype=dt)
    allP0 = torch.as_tensor(np.stack([p.p0 for p in planes]), device=dev, dtype=dt)
    E1 = torch.as_tensor(np.stack([p.e1 for p in planes]), device=dev, dtype=dt)
    E2 = torch.as_tensor(np.stack([p.e2 for p in planes]), device=dev, dtype=dt)
    OM = torch.as_tensor(np.stack([p.omega for p in planes]), device=dev, dtype=dt)      # (Q,8,2)
    PH = torch.as_tensor(np.stack([p.phase for p in planes]), device=dev, dtype=dt)      # (Q,8)
    n_w, p0_w = allN[pid], allP0[pid]
    lam_w = ((p0_w - C) * n_w).sum(1) / (d * n_w).sum(1)
    Xw = C + lam_w.unsqueeze(-1) * d - p0_w
    a = (Xw * E1[pid]).sum(1)
    b = (Xw * E2[pid]).sum(1)
    om = OM[pid]
    arg_ = 2.0 * math.pi * (a.unsqueeze(-1) * om[..., 0] + b.unsqueeze(-1) * om[..., 1]) + PH[pid]
    img = (0.5 + torch.sin(arg_).sum(-1) / 16.0).view(H, W)
    if noise_sigma > 0:
        img = img + noise_sigma * torch.randn((H, W), device=dev, dtype=dt, generator=gen)
    img = img.clamp(0.0, 1.0)
    return img.to(torch.float32), pid.view(H, W).to(torch.int16)


def _gt_surfels(planes, K, W, H, S, kf_pid: np.ndarray):
    """Ground-truth plane of every tile: tiles are pure (rectangle edges lie
    on multiples of 8 px), so the plane hit by the tile's first pixel owns it;
    its inverse depth along the tile's centre ray is the ray/plane
    intersection."""
    fx, fy, cx, cy = K
    gw, gh = W // S, H // S
    pid = kf_pid[0:gh * S:S, 0:gw * S:S].astype(np.int64)             # (gh, gw)
    Nn = np.stack([p.n for p in planes])[pid]                          # (gh, gw, 3)
    P0 = np.stack([p.p0 for p in planes])[pid]
    tx = np.arange(gw)[None, :]
    ty = np.arange(gh)[:, None]
    us = S * tx + 0.5 * (S - 1)
    vs = S * ty + 0.5 * (S - 1)
    r = np.stack(np.broadcast_arrays((us - cx) / fx, (vs - cy) / fy, np.ones((gh, gw))), -1)
    gt_id = (Nn * r).sum(-1) / (Nn * P0).sum(-1)
    return gt_id, Nn.copy()


def _perturb(rng, gt_id, gt_n, depth_noise, normal_deg):
    gh, gw = gt_id.shape
    scale = rng.uniform(1.0 - depth_noise, 1.0 + depth_noise, size=(gh, gw))
    init_id = gt_id / scale
    ang = np.radians(rng.uniform(0.0, normal_deg, size=(gh, gw)))
    psi = rng.uniform(0.0, 2.0 * math.pi, size=(gh, gw))
    n = gt_n
    e = np.where((np.abs(n[..., 0]) < 0.9)[..., None], np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0]))
    b1 = e - (e * n).sum(-1, keepdims=True) * n
    b1 /= np.linalg.norm(b1, axis=-1, keepdims=True)
    b2 = np.cross(n, b1)
    axis = np.cos(psi)[..., None] * b1 + np.sin(psi)[..., None] * b2      # unit, orthogonal to n
    # Rodrigues for an axis orthogonal to n: n cos + (axis x n) sin
    init_n = n * np.cos(ang)[..., None] + np.cross(axis, n) * np.sin(ang)[..., None]
    return init_id.astype(np.float32), init_n.astype(np.float32)


def make_keyframe(spec: SceneSpec, device="cpu", keep_nbr_plane_id=False) -> Keyframe:
    rng = np.random.default_rng(spec.seed)
    K = spec.intrinsics()
    W, H, S = spec.width, spec.height, spec.patch
    planes = _make_planes(spec, rng)
    R = np.zeros((spec.n_nbr, 3, 3))
    t = np.zeros((spec.n_nbr, 3))
    for j in range(spec.n_nbr):
        R[j] = rotation_about(_unit(rng), math.radians(rng.uniform(0.0, spec.rot_deg)))
        t[j] = spec.trans * _unit(rng)
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(spec.seed) * 7919 + 17)
    kf_img, kf_pid = _render(planes, K, W, H, np.eye(3), np.zeros(3), dev, spec.noise_sigma, gen)
    nbrs, nbr_pids = [], []
    for j in range(spec.n_nbr):
        im, pid = _render(planes, K, W, H, R[j], t[j], dev, spec.noise_sigma, gen)
        nbrs.append(im)
        if keep_nbr_plane_id:
            nbr_pids.append(pid)
    nbr_images = torch.stack(nbrs) if nbrs else torch.zeros((0, H, W), device=dev)
    kf_pid_np = kf_pid.cpu().numpy()
    gt_id, gt_n = _gt_surfels(planes, K, W, H, S, kf_pid_np)
    init_id, init_n = _perturb(rng, gt_id, gt_n, spec.init_depth_noise, spec.init_normal_deg)
    gh, gw = gt_id.shape
    if spec.half_new:
        yy, xx = np.mgrid[0:gh, 0:gw]
        is_new = ((xx + yy) % 2 == 1).astype(np.uint8)
    else:
        is_new = np.zeros((gh, gw), dtype=np.uint8)
    return Keyframe(spec=spec, K=K, width=W, height=H, patch=S, iters=spec.iters,
                    kf_image=kf_img, nbr_images=nbr_images, R=R, t=t,
                    gt_id=gt_id, gt_n=gt_n, init_id=init_id, init_n=init_n,
                    is_new=is_new, kf_plane_id=kf_pid_np,
                    nbr_plane_id=torch.stack(nbr_pids) if keep_nbr_plane_id else None,
                    planes=planes)


def spec_for_config(index: int, sub: int = 0) -> SceneSpec:
    """Scene specs of the five workloads (0-based index).

    0: 160x120, 3 planes, 2 neighbours, 8x8 surfels, 10 iterations, seed 1.
    1: 640x480, 20 planes + ground, 8 neighbours, 4x4 surfels, 15 iterations,
       half the surfels new, seed 2.
    2/3: keyframe `sub` (0..63) of the 64-keyframe batch, seed 300+sub.
    4: stream `sub` (0..31) of the serving workload, seed 500+sub.
    """
    if index == 0:
        return SceneSpec(160, 120, 2, 8, 10, 3, False, 1, False, K=(150.0, 150.0, 80.0, 60.0))
    if index == 1:
        return SceneSpec(640, 480, 8, 4, 15, 20, True, 2, True)
    if index in (2, 3):
        seed = 300 + sub
        rng = np.random.default_rng(seed + 100000)
        W, H = RESOLUTIONS_BATCH[int(rng.integers(0, 3))]
        n = int(rng.integers(4, 13))
        return SceneSpec(W, H, n, 4, 15, 20, True, seed, True)
    if index == 4:
        seed = 500 + sub
        rng = np.random.default_rng(seed + 100000)
        W, H = RESOLUTIONS_STREAM[int(rng.integers(0, 4))]
        n = int(rng.integers(4, 11))
        return SceneSpec(W, H, n, 4, 15, 20, True, seed, True)
    raise ValueError(f"no workload {index}")


def batch_specs(count: int = 64) -> List[SceneSpec]:
    return [spec_for_config(2, i) for i in range(count)]


def stream_specs(count: int = 32) -> List[SceneSpec]:
    return [spec_for_config(4, i) for i in range(count)]


def make_config(index: int, device="cpu", sub: int = 0) -> Keyframe:
    return make_keyframe(spec_for_config(index, sub), device=device)
