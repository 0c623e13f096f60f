"""Plain FP64 CPU oracle of the per-surfel Gauss-Newton update (ctypes binding).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark use it; the product library never imports it.  The
arithmetic lives in ``sgo.c`` (plain C, IEEE double); this module only
marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgo.so")

DEGENERATE = 1 << 0
FEW_SAMPLES = 1 << 1
SOLVE_FAIL = 1 << 2
REJECTED = 1 << 3
FP64_SOLVE = 1 << 4
UNINIT = 1 << 5


def build(force: bool = True) -> str:
    """Compile sgo.c with gcc (no fast-math, no FMA contraction)."""
    src = os.path.join(_HERE, "sgo.c")
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(src):
        return LIB_PATH
    tmp = f"{LIB_PATH}.tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Intrinsics(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class Pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class Image(C.Structure):
    _fields_ = [("pix", C.POINTER(C.c_double)), ("width", C.c_int32), ("height", C.c_int32)]


class KeyframeC(C.Structure):
    _fields_ = [("kf", Image), ("nbr", C.POINTER(Image)), ("pose", C.POINTER(Pose)),
                ("n_nbr", C.c_int32), ("K", Intrinsics), ("patch", C.c_int32)]


class SurfelsC(C.Structure):
    _fields_ = [("inv_depth", C.POINTER(C.c_double)), ("nx", C.POINTER(C.c_double)),
                ("ny", C.POINTER(C.c_double)), ("nz", C.POINTER(C.c_double)),
                ("flags", C.POINTER(C.c_uint32)), ("cost", C.POINTER(C.c_double)),
                ("nvalid", C.POINTER(C.c_int32)), ("last_update", C.POINTER(C.c_uint32)),
                ("kappa", C.POINTER(C.c_double)), ("margin", C.POINTER(C.c_double))]


class GridC(C.Structure):
    _fields_ = [("K", Intrinsics), ("width", C.c_int32), ("height", C.c_int32), ("patch", C.c_int32)]


class ParamsC(C.Structure):
    _fields_ = [("iters", C.c_int32), ("huber_k", C.c_double), ("depth_only", C.c_int32),
                ("beta_r", C.c_double), ("stamp", C.c_uint32), ("lm_lambda", C.c_double),
                ("perturb", C.c_double), ("perturb_seed", C.c_uint32), ("perturb_parts", C.c_int32),
                ("tie_window", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.sgo_pixel_inverse_depth.restype = C.c_double
        L.sgo_pixel_inverse_depth.argtypes = [C.POINTER(Intrinsics), C.c_double, C.c_double,
                                              C.c_double, dp, C.c_double, C.c_double]
        L.sgo_warp.restype = C.c_int
        L.sgo_warp.argtypes = [C.POINTER(Intrinsics), C.POINTER(Pose), C.c_double, C.c_double,
                               C.c_double, dp]
        L.sgo_bilinear.restype = C.c_int
        L.sgo_bilinear.argtypes = [C.POINTER(Image), C.c_double, C.c_double, dp]
        L.sgo_tangent_basis.restype = None
        L.sgo_tangent_basis.argtypes = [dp, dp, dp]
        L.sgo_eval_sample.restype = C.c_int
        L.sgo_eval_sample.argtypes = [C.POINTER(Intrinsics), C.POINTER(Pose), C.POINTER(Image),
                                      C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_double, dp, C.c_int, dp, dp]
        L.sgo_linearize.restype = C.c_int32
        L.sgo_linearize.argtypes = [C.POINTER(KeyframeC), C.c_int32, C.c_int32, C.c_double, dp,
                                    C.c_double, C.c_int, dp, dp, dp]
        L.sgo_solve3.restype = C.c_uint32
        L.sgo_solve3.argtypes = [dp, dp, dp]
        L.sgo_kappa_eq.restype = C.c_double
        L.sgo_kappa_eq.argtypes = [dp]
        ip = C.POINTER(C.c_int32)
        L.sgo_optimize_keyframe.restype = C.c_int
        L.sgo_optimize_keyframe.argtypes = [C.POINTER(KeyframeC), C.POINTER(SurfelsC),
                                            C.POINTER(ParamsC), ip, C.c_int32]
        L.sgo_init_from_neighbours.restype = C.c_int
        L.sgo_init_from_neighbours.argtypes = [C.POINTER(KeyframeC), C.POINTER(SurfelsC),
                                               C.POINTER(C.c_uint8), C.POINTER(ParamsC), ip,
                                               C.c_int32]
        L.sgo_render_inverse_depth.restype = C.c_int
        L.sgo_render_inverse_depth.argtypes = [C.POINTER(KeyframeC), C.POINTER(SurfelsC), dp, ip]
        L.sgo_transfer_surfels.restype = C.c_int
        L.sgo_transfer_surfels.argtypes = [C.POINTER(Intrinsics), C.POINTER(Pose), C.c_int32,
                                           dp, dp, dp, dp, dp, dp, dp, dp]
        L.sgo_transfer_regrid.restype = C.c_int
        L.sgo_transfer_regrid.argtypes = [C.POINTER(GridC), C.POINTER(SurfelsC), C.POINTER(Pose),
                                          C.POINTER(GridC), C.POINTER(SurfelsC),
                                          C.POINTER(C.c_uint8), ip]
        L.sgo_disc_support.restype = C.c_int32
        L.sgo_disc_support.argtypes = [C.c_int32, C.c_int32, C.c_double, C.c_double, C.c_double,
                                       ip, ip, C.c_int32]
        L.sgo_disc_linearize.restype = C.c_int32
        L.sgo_disc_linearize.argtypes = [C.POINTER(KeyframeC), C.c_double, C.c_double, C.c_double,
                                         C.c_double, dp, C.c_double, C.c_int, dp, dp, dp]
        L.sgo_disc_optimize.restype = C.c_int
        L.sgo_disc_optimize.argtypes = [C.POINTER(KeyframeC), C.POINTER(SurfelsC), dp, dp,
                                        C.c_int32, C.c_double, C.POINTER(ParamsC), ip, C.c_int32]
        L.sgo_disc_render.restype = C.c_int
        L.sgo_disc_render.argtypes = [C.POINTER(KeyframeC), C.POINTER(SurfelsC), dp, dp,
                                      C.c_int32, C.c_double, dp, ip]
        L.sgo_disc_search.restype = C.c_int32
        L.sgo_disc_search.argtypes = [C.c_int32, C.c_int32, ip, C.c_double, C.c_double,
                                      C.c_int32, ip, ip, C.c_int32]
        L.sgo_disc_init.restype = C.c_int
        L.sgo_disc_init.argtypes = [C.POINTER(KeyframeC), C.POINTER(SurfelsC), dp, dp, ip,
                                    C.c_int32, C.c_int32, C.c_double, C.c_double]
        L.sgo_disc_transfer.restype = C.c_int32
        L.sgo_disc_transfer.argtypes = [C.POINTER(Intrinsics), C.POINTER(Intrinsics), C.c_int32,
                                        C.c_int32, C.POINTER(Pose), C.POINTER(SurfelsC), dp, dp,
                                        C.c_int32, C.POINTER(SurfelsC), dp, dp, C.c_int32, ip, ip]
        L.sgo_costs_at.restype = C.c_int
        L.sgo_costs_at.argtypes = [C.POINTER(KeyframeC), dp, dp, dp, dp, ip, C.c_int32, C.c_double,
                                   dp, dp, C.c_double, dp, ip]
        L.sgo_set_threads.restype = None
        L.sgo_set_threads.argtypes = [C.c_int32]
        L.sgo_max_threads.restype = C.c_int32
        L.sgo_max_threads.argtypes = []
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def intrinsics(K: Sequence[float]) -> Intrinsics:
    return Intrinsics(*[float(v) for v in K])


def pose(R, t) -> Pose:
    p = Pose()
    R = np.asarray(R, dtype=np.float64).reshape(9)
    t = np.asarray(t, dtype=np.float64).reshape(3)
    for i in range(9):
        p.R[i] = float(R[i])
    for i in range(3):
        p.t[i] = float(t[i])
    return p


def image(arr: np.ndarray):
    a = _f64(arr)
    im = Image(_dp(a), a.shape[1], a.shape[0])
    return im, a


@dataclass
class OracleParams:
    iters: int = 10
    huber_k: float = 9.0 / 255.0
    depth_only: bool = False
    beta_r: Optional[float] = None   # default: the tile edge S
    stamp: int = 1
    lm_lambda: float = 0.0
    perturb: float = 0.0        # conditioning probe (tests only), 0 = off
    perturb_seed: int = 0
    perturb_parts: int = 0      # bit set: 1 normal equations, 2 state, 4 LM acceptance; 0 = all
    tie_window: float = 0.0     # probe: relative noise of the LM acceptance threshold (0: perturb)

    def c(self, patch: int) -> ParamsC:
        br = float(self.beta_r) if self.beta_r is not None else float(patch)
        return ParamsC(int(self.iters), float(self.huber_k), int(bool(self.depth_only)), br,
                       int(self.stamp), float(self.lm_lambda), float(self.perturb),
                       int(self.perturb_seed), int(self.perturb_parts), float(self.tie_window))


class OracleKeyframe:
    """Keeps FP64 copies of one keyframe's images and poses alive for C calls.

    ``kf_image`` (H, W) and ``nbr_images`` (N, H, W) must already hold the
    exact values the device path sees (dequantised f16/u8 values included).
    """

    def __init__(self, K, kf_image, nbr_images, R, t, patch: int):
        self.K = intrinsics(K)
        self.patch = int(patch)
        self.kf_img, self._kf_arr = image(kf_image)
        nbr_images = np.asarray(nbr_images)
        self.n_nbr = int(nbr_images.shape[0])
        self._nbr_arrs = [_f64(nbr_images[i]) for i in range(self.n_nbr)]
        self._nbr = (Image * max(1, self.n_nbr))()
        for i, a in enumerate(self._nbr_arrs):
            self._nbr[i] = Image(_dp(a), a.shape[1], a.shape[0])
        self._poses = (Pose * max(1, self.n_nbr))()
        for i in range(self.n_nbr):
            self._poses[i] = pose(R[i], t[i])
        self.c = KeyframeC(self.kf_img, self._nbr, self._poses, self.n_nbr, self.K, self.patch)
        self.width = int(self._kf_arr.shape[1])
        self.height = int(self._kf_arr.shape[0])

    @property
    def grid(self):
        return (self.width // self.patch, self.height // self.patch)

    @property
    def n_surfels(self):
        gw, gh = self.grid
        return gw * gh


def new_state(inv_depth, normals, flags=None) -> Dict[str, np.ndarray]:
    inv_depth = _f64(inv_depth).reshape(-1).copy()
    normals = _f64(normals).reshape(-1, 3)
    n = inv_depth.shape[0]
    return {
        "inv_depth": inv_depth,
        "nx": normals[:, 0].copy(), "ny": normals[:, 1].copy(), "nz": normals[:, 2].copy(),
        "flags": (np.zeros(n, np.uint32) if flags is None
                  else np.ascontiguousarray(np.asarray(flags, np.uint32).reshape(-1)).copy()),
        "cost": np.zeros(n), "nvalid": np.zeros(n, np.int32),
        "last_update": np.zeros(n, np.uint32), "kappa": np.zeros(n),
        "margin": np.full(n, np.inf),
    }


def _surfels_c(st: Dict[str, np.ndarray]) -> SurfelsC:
    return SurfelsC(_dp(st["inv_depth"]), _dp(st["nx"]), _dp(st["ny"]), _dp(st["nz"]),
                    st["flags"].ctypes.data_as(C.POINTER(C.c_uint32)), _dp(st["cost"]),
                    st["nvalid"].ctypes.data_as(C.POINTER(C.c_int32)),
                    st["last_update"].ctypes.data_as(C.POINTER(C.c_uint32)), _dp(st["kappa"]),
                    _dp(st["margin"]))


def _subset(subset):
    if subset is None:
        return None, 0, None
    arr = np.ascontiguousarray(np.asarray(subset, dtype=np.int32))
    return arr.ctypes.data_as(C.POINTER(C.c_int32)), int(arr.shape[0]), arr


def optimize(kf: OracleKeyframe, st: Dict[str, np.ndarray], params: OracleParams,
             subset=None) -> Dict[str, np.ndarray]:
    """Gauss-Newton iterations, in place on ``st`` (returned for convenience)."""
    sc = _surfels_c(st)
    pc = params.c(kf.patch)
    ptr, n, keep = _subset(subset)
    rc = lib().sgo_optimize_keyframe(C.byref(kf.c), C.byref(sc), C.byref(pc), ptr, n)
    if rc != 0:
        raise RuntimeError("sgo_optimize_keyframe failed")
    return st


def init_from_neighbours(kf: OracleKeyframe, st, is_new, params: OracleParams, subset=None):
    sc = _surfels_c(st)
    pc = params.c(kf.patch)
    nw = np.ascontiguousarray(np.asarray(is_new, dtype=np.uint8).reshape(-1))
    ptr, n, keep = _subset(subset)
    rc = lib().sgo_init_from_neighbours(C.byref(kf.c), C.byref(sc),
                                        nw.ctypes.data_as(C.POINTER(C.c_uint8)), C.byref(pc),
                                        ptr, n)
    if rc != 0:
        raise RuntimeError("sgo_init_from_neighbours failed")
    return st


def render(kf: OracleKeyframe, st):
    sc = _surfels_c(st)
    idm = np.zeros((kf.height, kf.width))
    ind = np.zeros((kf.height, kf.width), np.int32)
    lib().sgo_render_inverse_depth(C.byref(kf.c), C.byref(sc), _dp(idm),
                                   ind.ctypes.data_as(C.POINTER(C.c_int32)))
    return idm, ind


def linearize(kf: OracleKeyframe, tx, ty, id_s, n, huber_k=9.0 / 255.0, depth_only=False):
    H = np.zeros(9)
    b = np.zeros(3)
    cost = C.c_double(0.0)
    nn = _f64(n)
    nv = lib().sgo_linearize(C.byref(kf.c), int(tx), int(ty), float(id_s), _dp(nn),
                             float(huber_k), int(bool(depth_only)), _dp(H), _dp(b), C.byref(cost))
    return H.reshape(3, 3), b, float(cost.value), int(nv)


def eval_sample(K, R, t, nbr_img, kf_value, us, u, id_s, n, depth_only=False):
    Kc = intrinsics(K)
    P = pose(R, t)
    im, keep = image(nbr_img)
    nn = _f64(n)
    r = C.c_double(0.0)
    J = np.zeros(3)
    ok = lib().sgo_eval_sample(C.byref(Kc), C.byref(P), C.byref(im), float(kf_value),
                               float(us[0]), float(us[1]), float(u[0]), float(u[1]),
                               float(id_s), _dp(nn), int(bool(depth_only)), C.byref(r), _dp(J))
    return bool(ok), float(r.value), J


def pixel_inverse_depth(K, us, id_s, n, u):
    Kc = intrinsics(K)
    nn = _f64(n)
    return float(lib().sgo_pixel_inverse_depth(C.byref(Kc), float(us[0]), float(us[1]),
                                               float(id_s), _dp(nn), float(u[0]), float(u[1])))


def warp(K, R, t, u, id_u):
    Kc = intrinsics(K)
    P = pose(R, t)
    uv = np.zeros(2)
    ok = lib().sgo_warp(C.byref(Kc), C.byref(P), float(u[0]), float(u[1]), float(id_u), _dp(uv))
    return bool(ok), uv


def bilinear(img, x, y):
    im, keep = image(img)
    out = np.zeros(3)
    ok = lib().sgo_bilinear(C.byref(im), float(x), float(y), _dp(out))
    return bool(ok), out


def tangent_basis(n):
    nn = _f64(n)
    b1 = np.zeros(3)
    b2 = np.zeros(3)
    lib().sgo_tangent_basis(_dp(nn), _dp(b1), _dp(b2))
    return b1, b2


def solve3(H, b):
    Hm = _f64(H).reshape(9).copy()
    bb = _f64(b).reshape(3).copy()
    d = np.zeros(3)
    st = lib().sgo_solve3(_dp(Hm), _dp(bb), _dp(d))
    return int(st), d


def kappa_eq(H):
    Hm = _f64(H).reshape(9).copy()
    return float(lib().sgo_kappa_eq(_dp(Hm)))


def transfer(K, R, t, us, id_s, n):
    """Eq. 10 for arrays of surfels: us (M, 2), id_s (M,), n (M, 3)."""
    Kc = intrinsics(K)
    P = pose(R, t)
    us = _f64(us).reshape(-1, 2)
    m = us.shape[0]
    usx = np.ascontiguousarray(us[:, 0])
    usy = np.ascontiguousarray(us[:, 1])
    ids = _f64(id_s).reshape(-1)
    nn = _f64(n).reshape(-1, 3)
    ux = np.zeros(m)
    uy = np.zeros(m)
    ido = np.zeros(m)
    no = np.zeros((m, 3))
    lib().sgo_transfer_surfels(C.byref(Kc), C.byref(P), m, _dp(usx), _dp(usy), _dp(ids),
                               _dp(nn), _dp(ux), _dp(uy), _dp(ido), _dp(no))
    return np.stack([ux, uy], 1), ido, no


def transfer_regrid(src_grid, st, R, t, dst_grid):
    """Eq. 10 and re-gridding (see ``sgo_transfer_regrid``).

    src_grid / dst_grid: (K, width, height, patch).  ``st`` is a state dict of
    the source grid (``new_state``).  Returns (dst state dict, is_new (gh, gw)
    uint8, winning source index (gh, gw) int32, number of filled tiles)."""
    def grid(g):
        K, W, H, S = g
        return GridC(intrinsics(K), int(W), int(H), int(S))
    sg, dg = grid(src_grid), grid(dst_grid)
    gw, gh = dst_grid[1] // dst_grid[3], dst_grid[2] // dst_grid[3]
    m = gw * gh
    out = new_state(np.zeros(m), np.zeros((m, 3)))
    is_new = np.zeros(m, np.uint8)
    win = np.zeros(m, np.int32)
    P = pose(R, t)
    sc, dc = _surfels_c(st), _surfels_c(out)
    filled = lib().sgo_transfer_regrid(C.byref(sg), C.byref(sc), C.byref(P), C.byref(dg),
                                       C.byref(dc), is_new.ctypes.data_as(C.POINTER(C.c_uint8)),
                                       win.ctypes.data_as(C.POINTER(C.c_int32)))
    return out, is_new.reshape(gh, gw), win.reshape(gh, gw), int(filled)


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def disc_support(width, height, us, radius):
    """Pixels (x, y) of the disc of radius r centred at us (Eq. 4), row by row."""
    cap = 4 * int(math.ceil(radius) + 1) ** 2 + 16
    xs = np.zeros(cap, np.int32)
    ys = np.zeros(cap, np.int32)
    n = lib().sgo_disc_support(int(width), int(height), float(us[0]), float(us[1]), float(radius),
                               _ip(xs), _ip(ys), cap)
    return xs[:n].copy(), ys[:n].copy()


def disc_linearize(kf: OracleKeyframe, us, radius, id_s, n, huber_k=9.0 / 255.0, depth_only=False):
    H = np.zeros(9)
    b = np.zeros(3)
    cost = C.c_double(0.0)
    nn = _f64(n)
    nv = lib().sgo_disc_linearize(C.byref(kf.c), float(us[0]), float(us[1]), float(radius),
                                  float(id_s), _dp(nn), float(huber_k), int(bool(depth_only)),
                                  _dp(H), _dp(b), C.byref(cost))
    return H.reshape(3, 3), b, float(cost.value), int(nv)


def disc_optimize(kf: OracleKeyframe, st, ux, uy, radius, params: OracleParams, subset=None):
    """Gauss-Newton over disc surfels, in place on ``st`` (centres ux, uy)."""
    sc = _surfels_c(st)
    pc = params.c(1)
    cx, cy = _f64(ux).reshape(-1), _f64(uy).reshape(-1)
    ptr, n, keep = _subset(subset)
    rc = lib().sgo_disc_optimize(C.byref(kf.c), C.byref(sc), _dp(cx), _dp(cy), int(cx.size),
                                 float(radius), C.byref(pc), ptr, n)
    if rc != 0:
        raise RuntimeError("sgo_disc_optimize failed")
    return st


def disc_render(kf: OracleKeyframe, st, ux, uy, radius):
    sc = _surfels_c(st)
    cx, cy = _f64(ux).reshape(-1), _f64(uy).reshape(-1)
    idm = np.zeros((kf.height, kf.width))
    ind = np.zeros((kf.height, kf.width), np.int32)
    lib().sgo_disc_render(C.byref(kf.c), C.byref(sc), _dp(cx), _dp(cy), int(cx.size), float(radius),
                          _dp(idm), _ip(ind))
    return idm, ind


def disc_search(index_map, radius, alpha, spacing, capacity=None):
    """Lattice candidates farther than alpha r from every non-empty pixel:
    (xs, ys) of the first ``capacity`` and the number that qualify."""
    im = np.ascontiguousarray(np.asarray(index_map, np.int32))
    H, W = im.shape
    cap = (W // max(1, spacing) + 1) * (H // max(1, spacing) + 1) if capacity is None else int(capacity)
    xs = np.zeros(max(1, cap), np.int32)
    ys = np.zeros(max(1, cap), np.int32)
    found = lib().sgo_disc_search(W, H, _ip(im), float(radius), float(alpha), int(spacing),
                                  _ip(xs), _ip(ys), cap)
    if found < 0:
        raise RuntimeError("sgo_disc_search failed")
    k = min(found, cap)
    return xs[:k].copy(), ys[:k].copy(), int(found)


def disc_init(kf: OracleKeyframe, st, ux, uy, index_map, first, radius, beta):
    """Neighbour initialisation of surfels first .. len(ux)-1, in place on ``st``."""
    sc = _surfels_c(st)
    cx, cy = _f64(ux).reshape(-1), _f64(uy).reshape(-1)
    im = np.ascontiguousarray(np.asarray(index_map, np.int32))
    rc = lib().sgo_disc_init(C.byref(kf.c), C.byref(sc), _dp(cx), _dp(cy), _ip(im), int(first),
                             int(cx.size) - int(first), float(radius), float(beta))
    if rc != 0:
        raise RuntimeError("sgo_disc_init failed")
    return st


def disc_transfer(src_K, dst_K, dst_size, R, t, st, ux, uy, capacity=None):
    """Eq. 10 for disc surfels (see ``sgo_disc_transfer``): returns (dst state
    dict, centres (ux, uy), source indices, number landed)."""
    m = int(np.asarray(ux).size)
    cap = m if capacity is None else int(capacity)
    out = new_state(np.zeros(max(cap, 1)), np.zeros((max(cap, 1), 3)))
    dux = np.zeros(max(cap, 1))
    duy = np.zeros(max(cap, 1))
    idx = np.zeros(max(cap, 1), np.int32)
    landed = C.c_int32(0)
    sc, dc = _surfels_c(st), _surfels_c(out)
    cx, cy = _f64(ux).reshape(-1), _f64(uy).reshape(-1)
    Ks, Kd = intrinsics(src_K), intrinsics(dst_K)
    P = pose(R, t)
    n = lib().sgo_disc_transfer(C.byref(Ks), C.byref(Kd), int(dst_size[0]), int(dst_size[1]), C.byref(P),
                                C.byref(sc), _dp(cx), _dp(cy), m, C.byref(dc), _dp(dux), _dp(duy), cap,
                                _ip(idx), C.byref(landed))
    out = {k: v[:n] for k, v in out.items()}
    return out, (dux[:n], duy[:n]), idx[:n], int(landed.value)


def costs_at(kf: OracleKeyframe, inv_depth, normals, idx, huber_k=9.0 / 255.0, disc=None):
    """Huber cost and valid count of surfels idx at the states (inv_depth[i],
    normals[i]) (arrays over all surfels; normals renormalised); disc =
    (ux, uy, radius) for disc surfels."""
    ids = _f64(inv_depth).reshape(-1)
    nn = _f64(normals).reshape(-1, 3)
    nn = nn / np.linalg.norm(nn, axis=1, keepdims=True)
    nx, ny, nz = (np.ascontiguousarray(nn[:, k]) for k in range(3))
    ix = np.ascontiguousarray(np.asarray(idx, np.int32).reshape(-1))
    cost = np.zeros(ix.size)
    nv = np.zeros(ix.size, np.int32)
    if disc is not None:
        ux, uy = _f64(disc[0]).reshape(-1), _f64(disc[1]).reshape(-1)
        rc = lib().sgo_costs_at(C.byref(kf.c), _dp(ids), _dp(nx), _dp(ny), _dp(nz), _ip(ix), int(ix.size),
                                float(huber_k), _dp(ux), _dp(uy), float(disc[2]), _dp(cost), _ip(nv))
    else:
        rc = lib().sgo_costs_at(C.byref(kf.c), _dp(ids), _dp(nx), _dp(ny), _dp(nz), _ip(ix), int(ix.size),
                                float(huber_k), None, None, 0.0, _dp(cost), _ip(nv))
    if rc != 0:
        raise RuntimeError("sgo_costs_at failed")
    return cost, nv


def set_threads(n: int):
    lib().sgo_set_threads(int(n))


def max_threads() -> int:
    return int(lib().sgo_max_threads())


def dequantize_u8(codes: np.ndarray, scale: float) -> np.ndarray:
    """Exact FP64 value of u8 codes with a (float) scale: code * scale."""
    return np.asarray(codes, dtype=np.float64) * float(scale)
