"""ctypes binding of libsurfgn.so (include/surfgn.h).

Argument marshalling only: every step of the surfel Gauss-Newton path runs in
the library's HIP kernels.  torch supplies device memory and the stream.
The binding refuses to run without the compiled library (no fallback).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SURFGN_LIB") or os.path.join(HERE, "libsurfgn.so")

SGN_OK = 0
SGN_E_INVALID = -1
SGN_E_NOMEM = -2
SGN_E_DEVICE = -3
SGN_E_UNSUPPORTED = -4
SGN_E_BUSY = -5

SGN_F32, SGN_F16, SGN_U8 = 0, 1, 2

FLAG_DEGENERATE = 1 << 0
FLAG_FEW_SAMPLES = 1 << 1
FLAG_SOLVE_FAIL = 1 << 2
FLAG_REJECTED = 1 << 3
FLAG_FP64_SOLVE = 1 << 4
FLAG_UNINIT = 1 << 5

MAX_NBR = 16

EXPORTED = [
    "sgn_create", "sgn_destroy", "sgn_set_stream", "sgn_init_from_neighbours",
    "sgn_optimize_keyframe", "sgn_render_inverse_depth", "sgn_optimize_batch", "sgn_autotune",
    "sgn_quantize", "sgn_last_kernel_ms", "sgn_device_info", "sgn_status_str", "sgn_last_error",
    "sgn_version", "sgn_transfer_surfels", "sgn_disc_optimize", "sgn_disc_render", "sgn_disc_place",
    "sgn_recent_kernel_ms", "sgn_disc_transfer", "sgn_disc_render_batch", "sgn_disc_place_batch",
    "sgn_transfer_surfels_batch", "sgn_disc_transfer_batch", "sgn_transfer_workspace_bytes",
    "sgn_disc_render_workspace_bytes", "sgn_disc_place_workspace_bytes", "sgn_autotune_workspace_bytes",
    "sgn_transfer_surfels_static",
]

STATIC_SCRATCH_BYTES = 4 << 20


class SurfgnError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class sgn_intrinsics(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class sgn_pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class sgn_image(C.Structure):
    _fields_ = [("data", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("pitch", C.c_int32), ("dtype", C.c_int32), ("scale", C.c_float)]


class sgn_keyframe(C.Structure):
    _fields_ = [("kf", sgn_image), ("nbr", C.POINTER(sgn_image)), ("pose", C.POINTER(sgn_pose)),
                ("n_nbr", C.c_int32), ("K", sgn_intrinsics), ("patch", C.c_int32)]


class sgn_grid(C.Structure):
    _fields_ = [("K", sgn_intrinsics), ("width", C.c_int32), ("height", C.c_int32),
                ("patch", C.c_int32)]


class sgn_surfels(C.Structure):
    _fields_ = [("inv_depth", C.c_void_p), ("nx", C.c_void_p), ("ny", C.c_void_p),
                ("nz", C.c_void_p), ("flags", C.c_void_p), ("cost", C.c_void_p),
                ("nvalid", C.c_void_p), ("last_update", C.c_void_p)]


class sgn_params(C.Structure):
    _fields_ = [("iters", C.c_int32), ("huber_k", C.c_float), ("kappa_fp64", C.c_float),
                ("depth_only", C.c_int32), ("beta_r", C.c_float), ("stamp", C.c_uint32),
                ("lm_lambda", C.c_float)]


class sgn_plan(C.Structure):
    _fields_ = [("tiles_x", C.c_int32), ("tiles_y", C.c_int32), ("persistent", C.c_int32),
                ("waves_per_cu", C.c_int32), ("lds_stage", C.c_int32), ("xcd_queues", C.c_int32),
                ("groups", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class sgn_batch_item(C.Structure):
    _fields_ = [("kf", sgn_keyframe), ("surfels", sgn_surfels), ("is_new", C.c_void_p),
                ("inv_depth_out", C.c_void_p), ("index_out", C.c_void_p)]


class sgn_disc_item(C.Structure):
    _fields_ = [("kf", sgn_keyframe), ("surfels", sgn_surfels), ("ux", C.c_void_p),
                ("uy", C.c_void_p), ("count", C.c_int32), ("radius", C.c_float)]


class sgn_disc_place_params(C.Structure):
    _fields_ = [("alpha", C.c_float), ("beta", C.c_float), ("spacing", C.c_int32)]


class sgn_device_props(C.Structure):
    _fields_ = [("device", C.c_int32), ("compute_units", C.c_int32), ("xcds", C.c_int32),
                ("clock_khz", C.c_int32), ("memory_clock_khz", C.c_int32),
                ("memory_bus_bits", C.c_int32), ("total_global_mem", C.c_int64),
                ("lds_per_cu", C.c_int32), ("name", C.c_char * 64), ("arch", C.c_char * 32)]


_lib = None


def lib():
    """Load libsurfgn.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python paper_1910_01997_amd/build.py")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        vp = C.c_void_p
        L.sgn_create.restype = st
        L.sgn_create.argtypes = [C.POINTER(vp), C.c_int32, vp]
        L.sgn_destroy.restype = st
        L.sgn_destroy.argtypes = [vp]
        L.sgn_set_stream.restype = st
        L.sgn_set_stream.argtypes = [vp, vp]
        L.sgn_init_from_neighbours.restype = st
        L.sgn_init_from_neighbours.argtypes = [vp, C.POINTER(sgn_keyframe), C.POINTER(sgn_surfels),
                                               vp, C.POINTER(sgn_params)]
        L.sgn_optimize_keyframe.restype = st
        L.sgn_optimize_keyframe.argtypes = [vp, C.POINTER(sgn_keyframe), C.POINTER(sgn_surfels),
                                            C.POINTER(sgn_params), C.POINTER(sgn_plan)]
        L.sgn_render_inverse_depth.restype = st
        L.sgn_render_inverse_depth.argtypes = [vp, C.POINTER(sgn_keyframe), C.POINTER(sgn_surfels),
                                               vp, vp]
        L.sgn_optimize_batch.restype = st
        L.sgn_optimize_batch.argtypes = [vp, C.POINTER(sgn_batch_item), C.c_int32,
                                         C.POINTER(sgn_params), C.POINTER(sgn_plan)]
        L.sgn_autotune.restype = st
        L.sgn_autotune.argtypes = [vp, C.POINTER(sgn_batch_item), C.c_int32, C.POINTER(sgn_params),
                                   C.POINTER(sgn_plan), vp, C.c_size_t]
        L.sgn_autotune_workspace_bytes.restype = C.c_size_t
        L.sgn_autotune_workspace_bytes.argtypes = [C.c_int32, C.POINTER(sgn_batch_item)]
        L.sgn_quantize.restype = st
        L.sgn_quantize.argtypes = [vp, vp, C.c_int32, C.POINTER(sgn_image)]
        L.sgn_transfer_surfels.restype = st
        L.sgn_transfer_surfels.argtypes = [vp, C.POINTER(sgn_grid), C.POINTER(sgn_surfels),
                                           C.POINTER(sgn_pose), C.POINTER(sgn_grid),
                                           C.POINTER(sgn_surfels), vp, vp, vp, C.c_size_t]
        L.sgn_transfer_surfels_static.restype = st
        L.sgn_transfer_surfels_static.argtypes = [vp, C.POINTER(sgn_grid), C.POINTER(sgn_surfels),
                                                  C.POINTER(sgn_pose), C.POINTER(sgn_grid),
                                                  C.POINTER(sgn_surfels), vp, vp]
        L.sgn_transfer_surfels_batch.restype = st
        L.sgn_transfer_surfels_batch.argtypes = [vp, C.c_int32, C.POINTER(sgn_grid), C.POINTER(sgn_surfels),
                                                 C.POINTER(sgn_pose), C.POINTER(sgn_grid),
                                                 C.POINTER(sgn_surfels), C.POINTER(C.c_void_p),
                                                 C.POINTER(C.c_void_p), vp, C.c_size_t]
        L.sgn_transfer_workspace_bytes.restype = C.c_size_t
        L.sgn_transfer_workspace_bytes.argtypes = [C.c_int32, C.POINTER(sgn_grid)]
        L.sgn_disc_optimize.restype = st
        L.sgn_disc_optimize.argtypes = [vp, C.POINTER(sgn_disc_item), C.c_int32, C.POINTER(sgn_params)]
        L.sgn_disc_render.restype = st
        L.sgn_disc_render.argtypes = [vp, C.POINTER(sgn_disc_item), vp, vp, vp, C.c_size_t]
        L.sgn_disc_place.restype = st
        L.sgn_disc_place.argtypes = [vp, C.POINTER(sgn_disc_item), vp, C.c_int32,
                                     C.POINTER(sgn_disc_place_params), vp, vp, C.c_size_t]
        L.sgn_disc_place_batch.restype = st
        L.sgn_disc_place_batch.argtypes = [vp, C.POINTER(sgn_disc_item), C.c_int32, C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_int32), C.POINTER(sgn_disc_place_params),
                                           C.POINTER(C.c_void_p), vp, C.c_size_t]
        L.sgn_disc_render_batch.restype = st
        L.sgn_disc_render_batch.argtypes = [vp, C.POINTER(sgn_disc_item), C.c_int32,
                                            C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), vp, C.c_size_t]
        L.sgn_disc_render_workspace_bytes.restype = C.c_size_t
        L.sgn_disc_render_workspace_bytes.argtypes = [C.c_int32, C.POINTER(sgn_disc_item)]
        L.sgn_disc_place_workspace_bytes.restype = C.c_size_t
        L.sgn_disc_place_workspace_bytes.argtypes = [C.c_int32, C.POINTER(sgn_disc_item), C.c_int32]
        L.sgn_disc_transfer.restype = st
        L.sgn_disc_transfer.argtypes = [vp, C.POINTER(sgn_disc_item), C.POINTER(sgn_pose),
                                        C.POINTER(sgn_disc_item), C.c_int32, vp, vp]
        L.sgn_disc_transfer_batch.restype = st
        L.sgn_disc_transfer_batch.argtypes = [vp, C.c_int32, C.POINTER(sgn_disc_item), C.POINTER(sgn_pose),
                                              C.POINTER(sgn_disc_item), C.POINTER(C.c_int32),
                                              C.POINTER(C.c_void_p), C.POINTER(C.c_void_p)]
        L.sgn_recent_kernel_ms.restype = st
        L.sgn_recent_kernel_ms.argtypes = [vp, C.c_int32, C.POINTER(C.c_float)]
        L.sgn_last_kernel_ms.restype = st
        L.sgn_last_kernel_ms.argtypes = [vp, C.POINTER(C.c_float)]
        L.sgn_device_info.restype = st
        L.sgn_device_info.argtypes = [C.c_int32, C.POINTER(sgn_device_props)]
        L.sgn_status_str.restype = C.c_char_p
        L.sgn_status_str.argtypes = [C.c_int]
        L.sgn_last_error.restype = C.c_char_p
        L.sgn_last_error.argtypes = []
        L.sgn_version.restype = C.c_char_p
        L.sgn_version.argtypes = []
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != SGN_OK:
        detail = lib().sgn_last_error().decode(errors="replace")
        raise SurfgnError(status, where, detail)


# --- the C entry points under their own names -------------------------------

def sgn_create(device: int = 0, stream_ptr: int = 0) -> int:
    h = C.c_void_p()
    check(lib().sgn_create(C.byref(h), int(device), C.c_void_p(stream_ptr or None)), "sgn_create")
    return h.value


def sgn_destroy(ctx: int):
    check(lib().sgn_destroy(C.c_void_p(ctx)), "sgn_destroy")


def sgn_set_stream(ctx: int, stream_ptr: int):
    check(lib().sgn_set_stream(C.c_void_p(ctx), C.c_void_p(stream_ptr or None)), "sgn_set_stream")


def sgn_init_from_neighbours(ctx, kf: sgn_keyframe, surfels: sgn_surfels, is_new_ptr: int,
                             params: sgn_params):
    check(lib().sgn_init_from_neighbours(C.c_void_p(ctx), C.byref(kf), C.byref(surfels),
                                         C.c_void_p(is_new_ptr), C.byref(params)),
          "sgn_init_from_neighbours")


def sgn_optimize_keyframe(ctx, kf: sgn_keyframe, surfels: sgn_surfels, params: sgn_params,
                          plan: Optional[sgn_plan] = None):
    check(lib().sgn_optimize_keyframe(C.c_void_p(ctx), C.byref(kf), C.byref(surfels),
                                      C.byref(params), C.byref(plan) if plan is not None else None),
          "sgn_optimize_keyframe")


def sgn_render_inverse_depth(ctx, kf: sgn_keyframe, surfels: sgn_surfels, inv_depth_ptr: int,
                             index_ptr: int = 0):
    check(lib().sgn_render_inverse_depth(C.c_void_p(ctx), C.byref(kf), C.byref(surfels),
                                         C.c_void_p(inv_depth_ptr), C.c_void_p(index_ptr or None)),
          "sgn_render_inverse_depth")


def sgn_optimize_batch(ctx, items, n: int, params: sgn_params, plan: Optional[sgn_plan] = None):
    check(lib().sgn_optimize_batch(C.c_void_p(ctx), items, int(n), C.byref(params),
                                   C.byref(plan) if plan is not None else None), "sgn_optimize_batch")


def sgn_autotune(ctx, items, n: int, params: sgn_params, ws) -> sgn_plan:
    """ws: (device pointer, bytes) of a workspace of at least
    sgn_autotune_workspace_bytes(n, items) bytes (Context.workspace)."""
    out = sgn_plan()
    check(lib().sgn_autotune(C.c_void_p(ctx), items, int(n), C.byref(params), C.byref(out),
                             C.c_void_p(ws[0]), C.c_size_t(ws[1])), "sgn_autotune")
    return out


def sgn_autotune_workspace_bytes(n: int, items) -> int:
    return int(lib().sgn_autotune_workspace_bytes(int(n), items))


def sgn_quantize(ctx, src_ptr: int, src_pitch: int, dst: sgn_image):
    check(lib().sgn_quantize(C.c_void_p(ctx), C.c_void_p(src_ptr), int(src_pitch), C.byref(dst)),
          "sgn_quantize")


def sgn_transfer_surfels(ctx, src_grid: sgn_grid, src: sgn_surfels, pose: sgn_pose,
                         dst_grid: sgn_grid, dst: sgn_surfels, dst_is_new_ptr: int,
                         dst_src_index_ptr: Optional[int], ws):
    """ws: (device pointer, bytes), at least sgn_transfer_workspace_bytes([dst_grid])."""
    check(lib().sgn_transfer_surfels(C.c_void_p(ctx), C.byref(src_grid), C.byref(src),
                                     C.byref(pose), C.byref(dst_grid), C.byref(dst),
                                     C.c_void_p(dst_is_new_ptr),
                                     C.c_void_p(dst_src_index_ptr) if dst_src_index_ptr else None,
                                     C.c_void_p(ws[0]), C.c_size_t(ws[1])),
          "sgn_transfer_surfels")


def sgn_transfer_surfels_static(ctx, src_grid: sgn_grid, src: sgn_surfels, pose: sgn_pose,
                                dst_grid: sgn_grid, dst: sgn_surfels, dst_is_new_ptr: int,
                                dst_src_index_ptr: Optional[int]):
    """sgn_transfer_surfels with the library's static scratch (no workspace)."""
    check(lib().sgn_transfer_surfels_static(C.c_void_p(ctx), C.byref(src_grid), C.byref(src),
                                            C.byref(pose), C.byref(dst_grid), C.byref(dst),
                                            C.c_void_p(dst_is_new_ptr),
                                            C.c_void_p(dst_src_index_ptr) if dst_src_index_ptr else None),
          "sgn_transfer_surfels_static")


def sgn_transfer_workspace_bytes(dst_grids: Sequence[sgn_grid]) -> int:
    n = len(dst_grids)
    return int(lib().sgn_transfer_workspace_bytes(n, (sgn_grid * n)(*dst_grids)))


def c_array(T, xs):
    """xs as a ctypes array of T: returned as it is when it already is one
    (so a caller that calls with the same arguments many times can build
    them once), else built from the sequence.  Integers of a c_void_p array
    may be None (a null pointer)."""
    if isinstance(xs, C.Array) and getattr(xs, "_type_", None) is T:
        return xs
    if T is C.c_void_p:
        xs = [int(p) if p else None for p in xs]
    elif T is C.c_int32:
        xs = [int(v) for v in xs]
    return (T * len(xs))(*xs)


def sgn_transfer_surfels_batch(ctx, src_grids: Sequence[sgn_grid], srcs: Sequence[sgn_surfels],
                               poses: Sequence[sgn_pose], dst_grids: Sequence[sgn_grid],
                               dsts: Sequence[sgn_surfels], dst_is_new_ptrs: Sequence[int],
                               dst_src_index_ptrs: Optional[Sequence[int]], ws):
    """ws: (device pointer, bytes), at least sgn_transfer_workspace_bytes(dst_grids).
    Each sequence may also be a ctypes array of its type (see c_array)."""
    n = len(srcs)
    args = [c_array(sgn_grid, src_grids), c_array(sgn_surfels, srcs), c_array(sgn_pose, poses),
            c_array(sgn_grid, dst_grids), c_array(sgn_surfels, dsts), c_array(C.c_void_p, dst_is_new_ptrs)]
    if any(len(x) != n for x in args):
        raise ValueError("sgn_transfer_surfels_batch: sequences of different lengths")
    idx = c_array(C.c_void_p, dst_src_index_ptrs) if dst_src_index_ptrs is not None else None
    if idx is not None and len(idx) != n:
        raise ValueError("sgn_transfer_surfels_batch: sequences of different lengths")
    check(lib().sgn_transfer_surfels_batch(C.c_void_p(ctx), n, *args, idx, C.c_void_p(ws[0]), C.c_size_t(ws[1])),
          "sgn_transfer_surfels_batch")


def sgn_disc_optimize(ctx, items, n: int, params: sgn_params):
    check(lib().sgn_disc_optimize(C.c_void_p(ctx), items, int(n), C.byref(params)), "sgn_disc_optimize")


def sgn_disc_render(ctx, item: sgn_disc_item, inv_depth_ptr: int, index_ptr: int, ws):
    """ws: (device pointer, bytes), at least sgn_disc_render_workspace_bytes(1, item)."""
    check(lib().sgn_disc_render(C.c_void_p(ctx), C.byref(item), C.c_void_p(inv_depth_ptr),
                                C.c_void_p(index_ptr or None), C.c_void_p(ws[0]), C.c_size_t(ws[1])),
          "sgn_disc_render")


def sgn_disc_render_workspace_bytes(n: int, items) -> int:
    if isinstance(items, sgn_disc_item):
        items = C.byref(items)
    return int(lib().sgn_disc_render_workspace_bytes(int(n), items))


def sgn_disc_place(ctx, item: sgn_disc_item, index_map_ptr: int, capacity: int,
                   params: sgn_disc_place_params, counts_ptr: int, ws):
    """ws: (device pointer, bytes), at least sgn_disc_place_workspace_bytes(1, item, spacing)."""
    check(lib().sgn_disc_place(C.c_void_p(ctx), C.byref(item), C.c_void_p(index_map_ptr),
                               int(capacity), C.byref(params), C.c_void_p(counts_ptr),
                               C.c_void_p(ws[0]), C.c_size_t(ws[1])),
          "sgn_disc_place")


def sgn_disc_place_workspace_bytes(n: int, items, spacing: int) -> int:
    if isinstance(items, sgn_disc_item):
        items = C.byref(items)
    return int(lib().sgn_disc_place_workspace_bytes(int(n), items, int(spacing)))


def sgn_disc_transfer(ctx, src: sgn_disc_item, pose: sgn_pose, dst: sgn_disc_item, capacity: int,
                      counts_ptr: int, src_index_ptr: int = 0):
    check(lib().sgn_disc_transfer(C.c_void_p(ctx), C.byref(src), C.byref(pose), C.byref(dst),
                                  int(capacity), C.c_void_p(counts_ptr), C.c_void_p(src_index_ptr or None)),
          "sgn_disc_transfer")


def sgn_disc_place_batch(ctx, items, n: int, index_map_ptrs: Sequence[int], capacities: Sequence[int],
                         params: sgn_disc_place_params, counts_ptrs: Sequence[int], ws):
    maps = (C.c_void_p * int(n))(*[int(p) if p else None for p in index_map_ptrs])
    caps = (C.c_int32 * int(n))(*[int(c) for c in capacities])
    cnts = (C.c_void_p * int(n))(*[int(p) if p else None for p in counts_ptrs])
    check(lib().sgn_disc_place_batch(C.c_void_p(ctx), items, int(n), maps, caps, C.byref(params), cnts,
                                     C.c_void_p(ws[0]), C.c_size_t(ws[1])),
          "sgn_disc_place_batch")


def sgn_disc_transfer_batch(ctx, srcs: Sequence[sgn_disc_item], poses: Sequence[sgn_pose],
                            dsts: Sequence[sgn_disc_item], capacities: Sequence[int],
                            counts_ptrs: Sequence[int], src_index_ptrs: Optional[Sequence[int]] = None):
    n = len(srcs)
    args = [c_array(sgn_disc_item, srcs), c_array(sgn_pose, poses), c_array(sgn_disc_item, dsts),
            c_array(C.c_int32, capacities), c_array(C.c_void_p, counts_ptrs)]
    idx = c_array(C.c_void_p, src_index_ptrs) if src_index_ptrs is not None else None
    if any(len(x) != n for x in args) or (idx is not None and len(idx) != n):
        raise ValueError("sgn_disc_transfer_batch: sequences of different lengths")
    check(lib().sgn_disc_transfer_batch(C.c_void_p(ctx), n, *args, idx), "sgn_disc_transfer_batch")


def sgn_disc_render_batch(ctx, items, n: int, inv_depth_ptrs: Sequence[int],
                          index_ptrs: Optional[Sequence[int]], ws):
    outs = (C.c_void_p * int(n))(*[int(p) for p in inv_depth_ptrs])
    idxs = (C.c_void_p * int(n))(*[int(p) if p else None for p in index_ptrs]) if index_ptrs else None
    check(lib().sgn_disc_render_batch(C.c_void_p(ctx), items, int(n), outs, idxs, C.c_void_p(ws[0]),
                                      C.c_size_t(ws[1])), "sgn_disc_render_batch")


def disc_array(items: List[sgn_disc_item]):
    arr = (sgn_disc_item * len(items))()
    for i, it in enumerate(items):
        arr[i] = it
    return arr


def grid_of(K, width: int, height: int, patch: int) -> sgn_grid:
    return sgn_grid(sgn_intrinsics(*[float(v) for v in K]), int(width), int(height), int(patch))


def sgn_last_kernel_ms(ctx) -> float:
    ms = C.c_float(0.0)
    check(lib().sgn_last_kernel_ms(C.c_void_p(ctx), C.byref(ms)), "sgn_last_kernel_ms")
    return float(ms.value)


def sgn_recent_kernel_ms(ctx, n: int) -> List[float]:
    out = (C.c_float * int(n))()
    check(lib().sgn_recent_kernel_ms(C.c_void_p(ctx), int(n), out), "sgn_recent_kernel_ms")
    return [float(v) for v in out]


def sgn_device_info(device: int = 0) -> dict:
    p = sgn_device_props()
    check(lib().sgn_device_info(int(device), C.byref(p)), "sgn_device_info")
    d = {k: getattr(p, k) for k, _ in p._fields_}
    d["name"] = p.name.decode(errors="replace")
    d["arch"] = p.arch.decode(errors="replace")
    return d


def sgn_status_str(status: int) -> str:
    return lib().sgn_status_str(int(status)).decode()


def sgn_last_error() -> str:
    return lib().sgn_last_error().decode(errors="replace")


def sgn_version() -> str:
    return lib().sgn_version().decode()


# --- marshalling helpers (structs from torch tensors) -----------------------

_TORCH_DTYPE_CODE = {"torch.float32": SGN_F32, "torch.float16": SGN_F16, "torch.uint8": SGN_U8}


def image_of(t, scale: float = 1.0) -> sgn_image:
    """sgn_image view of a 2-D CUDA tensor (row-major, any row stride)."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("image tensor must be 2-D with unit column stride")
    code = _TORCH_DTYPE_CODE.get(str(t.dtype))
    if code is None:
        raise ValueError(f"unsupported image dtype {t.dtype}")
    return sgn_image(t.data_ptr(), t.shape[1], t.shape[0], t.stride(0), code, float(scale))


def pose_of(R, t) -> sgn_pose:
    p = sgn_pose()
    Rf = [float(v) for v in list(R.reshape(-1))]
    tf = [float(v) for v in list(t.reshape(-1))]
    for i in range(9):
        p.R[i] = Rf[i]
    for i in range(3):
        p.t[i] = tf[i]
    return p


class KeyframeView:
    """Keeps the ctypes arrays of one sgn_keyframe alive."""

    def __init__(self, kf_image, nbr_images: Sequence, R, t, K, patch: int, scale: float = 1.0):
        self.kf_img = image_of(kf_image, scale)
        n = len(nbr_images)
        self.nbr = (sgn_image * max(1, n))(*[image_of(im, scale) for im in nbr_images])
        self.poses = (sgn_pose * max(1, n))(*[pose_of(R[i], t[i]) for i in range(n)])
        self.c = sgn_keyframe(self.kf_img, self.nbr, self.poses, n,
                              sgn_intrinsics(*[float(v) for v in K]), int(patch))
        self._keep = (kf_image, list(nbr_images))


class SurfelState:
    """Device SoA surfel state (torch tensors) and its sgn_surfels view."""

    def __init__(self, inv_depth, nx, ny, nz, flags, cost, nvalid, last_update):
        self.inv_depth, self.nx, self.ny, self.nz = inv_depth, nx, ny, nz
        self.flags, self.cost, self.nvalid, self.last_update = flags, cost, nvalid, last_update
        self.c = sgn_surfels(inv_depth.data_ptr(), nx.data_ptr(), ny.data_ptr(), nz.data_ptr(),
                             flags.data_ptr(), cost.data_ptr(), nvalid.data_ptr(),
                             last_update.data_ptr())

    @classmethod
    def from_arrays(cls, inv_depth, normals, flags=None, device="cuda"):
        import numpy as np
        import torch
        idt = torch.as_tensor(np.ascontiguousarray(np.asarray(inv_depth, np.float32).reshape(-1)),
                              device=device)
        n = np.asarray(normals, np.float32).reshape(-1, 3)
        m = idt.numel()
        fl = (torch.zeros(m, dtype=torch.int32, device=device) if flags is None else
              torch.as_tensor(np.asarray(flags, np.uint32).astype(np.int32).reshape(-1), device=device))
        mk = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=device)
        return cls(idt, mk(n[:, 0]), mk(n[:, 1]), mk(n[:, 2]), fl,
                   torch.zeros(m, dtype=torch.float32, device=device),
                   torch.zeros(m, dtype=torch.int32, device=device),
                   torch.zeros(m, dtype=torch.int32, device=device))

    def clone(self) -> "SurfelState":
        return SurfelState(*[t.clone() for t in (self.inv_depth, self.nx, self.ny, self.nz,
                                                 self.flags, self.cost, self.nvalid,
                                                 self.last_update)])

    def to_host(self) -> dict:
        import numpy as np
        return {
            "inv_depth": self.inv_depth.cpu().numpy(),
            "n": np.stack([self.nx.cpu().numpy(), self.ny.cpu().numpy(), self.nz.cpu().numpy()], 1),
            "flags": self.flags.cpu().numpy().astype(np.uint32),
            "cost": self.cost.cpu().numpy(),
            "nvalid": self.nvalid.cpu().numpy().astype(np.int64),
            "last_update": self.last_update.cpu().numpy().astype(np.uint32),
        }


def params(iters=15, huber_k=9.0 / 255.0, kappa_fp64=1e6, depth_only=False, beta_r=0.0,
           stamp=1, lm_lambda=0.0) -> sgn_params:
    return sgn_params(int(iters), float(huber_k), float(kappa_fp64), int(bool(depth_only)),
                      float(beta_r), int(stamp), float(lm_lambda))


def plan(tiles_x=0, tiles_y=0, persistent=1, waves_per_cu=0, lds_stage=0, xcd_queues=1,
         groups=0) -> sgn_plan:
    return sgn_plan(tiles_x, tiles_y, persistent, waves_per_cu, lds_stage, xcd_queues, groups)


class Context:
    """Owns one sgn_ctx bound to a torch stream (default: the current stream),
    and the caller-side workspace its calls use (a torch byte tensor on the
    context's device, grown on demand; the stream orders its reuse)."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.handle = sgn_create(device, self.stream.cuda_stream)
        self._ws = None

    def workspace(self, nbytes: int):
        """(device pointer, bytes) of a workspace of at least nbytes bytes."""
        import torch
        if nbytes <= 0:
            raise ValueError("invalid arguments: the library reports no workspace size")
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(int(nbytes), dtype=torch.uint8,
                                   device=torch.device("cuda", self.device))
        return self._ws.data_ptr(), self._ws.numel()

    def close(self):
        if self.handle:
            sgn_destroy(self.handle)
            self.handle = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_array(items: List[sgn_batch_item]):
    arr = (sgn_batch_item * len(items))(*items)
    return arr
