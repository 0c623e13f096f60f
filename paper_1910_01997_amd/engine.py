"""Keyframe-level helpers over the C ABI: device-resident keyframes and
surfel state as torch tensors, and the plain (one keyframe at a time) and
batched update calls.  Marshalling only; all arithmetic runs in the HIP
kernels of libsurfgn.so."""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import surfgn as sg

STORAGE = {"f32": sg.SGN_F32, "f16": sg.SGN_F16, "u8": sg.SGN_U8}
U8_SCALE = 1.0 / 255.0


class DeviceKeyframe:
    """One keyframe, its neighbour frames and its surfels, resident on the GPU.

    images: float32 tensors (any device) of the sampled values; they are
    uploaded and, for f16/u8 storage, quantised on the device by the
    library's quantize kernel.
    """

    def __init__(self, ctx: sg.Context, kf_image, nbr_images, R, t, K, patch: int,
                 init_id, init_n, is_new=None, storage: str = "f32", render: bool = True,
                 index_map: bool = False, flags=None, u8_scale: float = U8_SCALE):
        dev = torch.device("cuda", ctx.device)
        self.ctx = ctx
        self.storage = storage
        self.patch = int(patch)
        self.K = tuple(float(v) for v in K)
        self.R = np.asarray(R, np.float64)
        self.t = np.asarray(t, np.float64)
        kf32 = torch.as_tensor(kf_image, dtype=torch.float32).to(dev).contiguous()
        nb32 = torch.as_tensor(nbr_images, dtype=torch.float32).to(dev).contiguous()
        self.height, self.width = kf32.shape
        self.n_nbr = int(nb32.shape[0])
        self.scale = 1.0
        if storage == "f32":
            self.kf_img, self.nbr_imgs = kf32, nb32
        else:
            code = STORAGE[storage]
            tdt = torch.float16 if storage == "f16" else torch.uint8
            self.scale = 1.0 if storage == "f16" else float(u8_scale)
            self.kf_img = torch.empty((self.height, self.width), dtype=tdt, device=dev)
            self.nbr_imgs = torch.empty((self.n_nbr, self.height, self.width), dtype=tdt, device=dev)
            for src, dst in [(kf32, self.kf_img)] + [(nb32[i], self.nbr_imgs[i]) for i in range(self.n_nbr)]:
                sg.sgn_quantize(ctx.handle, src.data_ptr(), src.stride(0),
                                sg.sgn_image(dst.data_ptr(), self.width, self.height, dst.stride(0),
                                             code, float(self.scale)))
        self.view = sg.KeyframeView(self.kf_img, [self.nbr_imgs[i] for i in range(self.n_nbr)],
                                    self.R, self.t, self.K, self.patch, self.scale)
        self.state = sg.SurfelState.from_arrays(init_id, init_n, flags=flags, device=dev)
        self.is_new = None
        if is_new is not None:
            self.is_new = torch.as_tensor(np.asarray(is_new, np.uint8).reshape(-1), device=dev)
        self.inv_depth_out = (torch.zeros((self.height, self.width), dtype=torch.float32, device=dev)
                              if render else None)
        self.index_out = (torch.full((self.height, self.width), -1, dtype=torch.int32, device=dev)
                          if (render and index_map) else None)

    @classmethod
    def from_scene(cls, ctx, kf, storage="f32", render=True, index_map=False, with_new=True,
                   u8_scale: float = U8_SCALE):
        return cls(ctx, kf.kf_image, kf.nbr_images, kf.R, kf.t, kf.K, kf.patch, kf.init_id,
                   kf.init_n, is_new=kf.is_new if (with_new and kf.is_new.any()) else None,
                   storage=storage, render=render, index_map=index_map, u8_scale=u8_scale)

    @property
    def grid(self):
        return (self.width // self.patch, self.height // self.patch)

    @property
    def n_surfels(self):
        gw, gh = self.grid
        return gw * gh

    def dequantized_images(self):
        """(kf, nbrs) as float64 numpy arrays of the exact values the kernels
        sample (stored code times scale)."""
        kf = self.kf_img.double().cpu().numpy() * self.scale
        nb = self.nbr_imgs.double().cpu().numpy() * self.scale
        return kf, nb

    def item(self, render: bool = True, init: bool = True) -> sg.sgn_batch_item:
        return sg.sgn_batch_item(
            self.view.c, self.state.c,
            self.is_new.data_ptr() if (init and self.is_new is not None) else None,
            self.inv_depth_out.data_ptr() if (render and self.inv_depth_out is not None) else None,
            self.index_out.data_ptr() if (render and self.index_out is not None) else None)

    def reset_state(self, init_id, init_n, flags=None):
        self.state = sg.SurfelState.from_arrays(init_id, init_n, flags=flags,
                                                device=self.state.inv_depth.device)


def update_plain(ctx: sg.Context, dk: DeviceKeyframe, prm: sg.sgn_params,
                 plan: Optional[sg.sgn_plan] = None, render: bool = True):
    """The plain single-keyframe form: init (if any new surfels), the
    Gauss-Newton iterations (one wavefront per work item), render."""
    if dk.is_new is not None:
        sg.sgn_init_from_neighbours(ctx.handle, dk.view.c, dk.state.c, dk.is_new.data_ptr(), prm)
    sg.sgn_optimize_keyframe(ctx.handle, dk.view.c, dk.state.c, prm, plan)
    if render and dk.inv_depth_out is not None:
        sg.sgn_render_inverse_depth(ctx.handle, dk.view.c, dk.state.c, dk.inv_depth_out.data_ptr(),
                                    dk.index_out.data_ptr() if dk.index_out is not None else 0)


def update_batch(ctx: sg.Context, dks: Sequence[DeviceKeyframe], prm: sg.sgn_params,
                 plan: Optional[sg.sgn_plan] = None, render: bool = True):
    items = sg.batch_array([d.item(render=render) for d in dks])
    sg.sgn_optimize_batch(ctx.handle, items, len(dks), prm, plan)
    return items


def autotune(ctx: sg.Context, items, n: int, prm: sg.sgn_params) -> sg.sgn_plan:
    """sgn_autotune on a batch descriptor array, with the context's workspace
    for the state snapshot."""
    ws = ctx.workspace(sg.sgn_autotune_workspace_bytes(n, items))
    return sg.sgn_autotune(ctx.handle, items, n, prm, ws)


def transfer_batch(ctx: sg.Context, src_grids, srcs, poses, dst_grids, dsts, dst_is_new_ptrs,
                   dst_src_index_ptrs=None):
    """sgn_transfer_surfels_batch with the context's workspace."""
    ws = ctx.workspace(sg.sgn_transfer_workspace_bytes(dst_grids))
    sg.sgn_transfer_surfels_batch(ctx.handle, src_grids, srcs, poses, dst_grids, dsts, dst_is_new_ptrs,
                                  dst_src_index_ptrs, ws)


class DiscKeyframe:
    """Disc surfels (Eq. 4) of one keyframe on the GPU: the images (as in
    DeviceKeyframe), the surfel state and centres with room for `capacity`
    surfels (the first `count` in use), and a rendered inverse-depth and
    surfel-index map."""

    def __init__(self, ctx: sg.Context, kf_image, nbr_images, R, t, K, radius: float, ux, uy,
                 init_id, init_n, flags=None, capacity: Optional[int] = None, storage: str = "f32",
                 u8_scale: float = U8_SCALE):
        dev = torch.device("cuda", ctx.device)
        self.ctx = ctx
        self.img = DeviceKeyframe(ctx, kf_image, nbr_images, R, t, K, 1, np.zeros(1, np.float32),
                                  np.zeros((1, 3), np.float32), storage=storage, render=False,
                                  u8_scale=u8_scale)
        self.K, self.R, self.t = self.img.K, self.img.R, self.img.t
        self.width, self.height = self.img.width, self.img.height
        self.radius = float(radius)
        m = int(np.asarray(ux).size)
        cap = max(m, int(capacity) if capacity else m)
        self.capacity = cap
        self.count = m
        pad = lambda a, v: np.concatenate([np.asarray(a, np.float32).reshape(-1),
                                           np.full(cap - m, v, np.float32)])
        idn = pad(init_id, 0.0)
        nn = np.concatenate([np.asarray(init_n, np.float32).reshape(-1, 3),
                             np.tile(np.float32([0.0, 0.0, -1.0]), (cap - m, 1))])
        fl = np.zeros(cap, np.uint32)
        if flags is not None:
            fl[:m] = np.asarray(flags, np.uint32).reshape(-1)
        self.state = sg.SurfelState.from_arrays(idn, nn, flags=fl, device=dev)
        self.ux = torch.as_tensor(pad(ux, 0.0), device=dev)
        self.uy = torch.as_tensor(pad(uy, 0.0), device=dev)
        self.inv_depth_out = torch.zeros((self.height, self.width), dtype=torch.float32, device=dev)
        self.index_out = torch.full((self.height, self.width), -1, dtype=torch.int32, device=dev)
        self.counts = torch.zeros(2, dtype=torch.int32, device=dev)

    @classmethod
    def from_scene(cls, ctx, kf, discs, capacity=None, storage="f32", u8_scale: float = U8_SCALE):
        return cls(ctx, kf.kf_image, kf.nbr_images, kf.R, kf.t, kf.K, discs.radius, discs.ux,
                   discs.uy, discs.init_id, discs.init_n, capacity=capacity, storage=storage,
                   u8_scale=u8_scale)

    def item(self) -> sg.sgn_disc_item:
        return sg.sgn_disc_item(self.img.view.c, self.state.c, self.ux.data_ptr(), self.uy.data_ptr(),
                                int(self.count), float(self.radius))

    def dequantized_images(self):
        return self.img.dequantized_images()

    def render(self):
        it = self.item()
        ws = self.ctx.workspace(sg.sgn_disc_render_workspace_bytes(1, it))
        sg.sgn_disc_render(self.ctx.handle, it, self.inv_depth_out.data_ptr(), self.index_out.data_ptr(),
                           ws)

    def place(self, alpha: float = 1.0, beta: float = 2.0, spacing: int = 0):
        """Empty-area search and placement from the current index map; waits
        for the device and returns (placed, qualifying)."""
        sp = int(spacing) if spacing else int(np.floor(self.radius * np.sqrt(2.0)))
        it = self.item()
        ws = self.ctx.workspace(sg.sgn_disc_place_workspace_bytes(1, it, sp))
        sg.sgn_disc_place(self.ctx.handle, it, self.index_out.data_ptr(), self.capacity,
                          sg.sgn_disc_place_params(float(alpha), float(beta), sp),
                          self.counts.data_ptr(), ws)
        placed, found = (int(v) for v in self.counts.cpu().tolist())
        self.count += placed
        return placed, found

    def transfer_from(self, src: "DiscKeyframe", R, t, src_index: Optional[torch.Tensor] = None):
        """Eq. 10: replace this keyframe's surfels with src's, moved by the
        pose X_self = R X_src + t (the ones that land in this image, up to
        the capacity); waits for the device and returns (written, landed)."""
        sg.sgn_disc_transfer(self.ctx.handle, src.item(), sg.pose_of(R, t), self.item(), self.capacity,
                             self.counts.data_ptr(), src_index.data_ptr() if src_index is not None else 0)
        written, landed = (int(v) for v in self.counts.cpu().tolist())
        self.count = written
        return written, landed

    def centres(self):
        return (self.ux[:self.count].cpu().numpy(), self.uy[:self.count].cpu().numpy())

    def state_host(self) -> dict:
        h = self.state.to_host()
        return {k: v[:self.count] for k, v in h.items()}


def disc_items(dks: Sequence[DiscKeyframe]):
    """The descriptor array of several disc keyframes (host memory, read by
    each call); refresh it with refresh_counts after a placement."""
    return sg.disc_array([d.item() for d in dks])


def refresh_counts(items, dks: Sequence[DiscKeyframe]):
    for i, d in enumerate(dks):
        items[i].count = int(d.count)


def disc_render(ctx: sg.Context, dks: Sequence[DiscKeyframe], items=None):
    """Depth-buffered render of several keyframes' discs in one pass."""
    items = disc_items(dks) if items is None else items
    ws = ctx.workspace(sg.sgn_disc_render_workspace_bytes(len(dks), items))
    sg.sgn_disc_render_batch(ctx.handle, items, len(dks), [d.inv_depth_out.data_ptr() for d in dks],
                             [d.index_out.data_ptr() for d in dks], ws)
    return items


def disc_place(ctx: sg.Context, dks: Sequence[DiscKeyframe], alpha: float = 1.0, beta: float = 2.0,
               spacing: int = 0, wait: bool = True, items=None):
    """Empty-area search and placement for several keyframes in one batch,
    each from its current index map (the same results as DiscKeyframe.place
    one by one).  With wait, synchronises once and returns the (placed,
    qualifying) pairs, updating each keyframe's count."""
    sp = int(spacing) if spacing else int(np.floor(dks[0].radius * np.sqrt(2.0)))
    items = disc_items(dks) if items is None else items
    ws = ctx.workspace(sg.sgn_disc_place_workspace_bytes(len(dks), items, sp))
    sg.sgn_disc_place_batch(ctx.handle, items, len(dks), [d.index_out.data_ptr() for d in dks],
                            [d.capacity for d in dks], sg.sgn_disc_place_params(float(alpha), float(beta), sp),
                            [d.counts.data_ptr() for d in dks], ws)
    if not wait:
        return None
    counts = torch.stack([d.counts for d in dks]).cpu().tolist()
    out = []
    for d, (placed, found) in zip(dks, counts):
        d.count += int(placed)
        out.append((int(placed), int(found)))
    return out


def disc_update(ctx: sg.Context, dks: Sequence[DiscKeyframe], prm: sg.sgn_params, items=None):
    """Gauss-Newton over the disc surfels of several keyframes in one launch."""
    items = disc_items(dks) if items is None else items
    sg.sgn_disc_optimize(ctx.handle, items, len(dks), prm)
    return items


_STATE_FIELDS = ("inv_depth", "nx", "ny", "nz", "flags", "cost", "nvalid", "last_update")


class StatePool:
    """Moves the surfel state of many keyframes into one allocation (each
    field a contiguous run of it, each keyframe a view into every field), so
    that a snapshot or a restore of a whole batch is one copy."""

    def __init__(self, dks: Sequence[DeviceKeyframe]):
        counts = [d.n_surfels for d in dks]
        total = sum(counts)
        first = dks[0].state
        dev = first.inv_depth.device
        # every field is 4 bytes per surfel: one float32 buffer, the integer
        # fields as int32 views of their runs
        self.buffer = torch.empty(len(_STATE_FIELDS) * total, dtype=torch.float32, device=dev)
        self.total = total
        self.fields = {}
        for k, f in enumerate(_STATE_FIELDS):
            run = self.buffer[k * total:(k + 1) * total]
            dt = getattr(first, f).dtype
            self.fields[f] = run if dt == torch.float32 else run.view(dt)
        off = 0
        for d, m in zip(dks, counts):
            views = {f: t[off:off + m] for f, t in self.fields.items()}
            for f, v in views.items():
                v.copy_(getattr(d.state, f))
            d.state = sg.SurfelState(*[views[f] for f in _STATE_FIELDS])
            off += m

    def snapshot(self):
        return self.buffer.clone()

    def restore(self, snap, fields=("inv_depth", "nx", "ny", "nz", "flags")):
        """Copy the given fields back from a snapshot: the leading run of
        fields (the default: the state the update reads) in one copy."""
        k = len(fields)
        if tuple(fields) == _STATE_FIELDS[:k]:
            self.buffer[:k * self.total].copy_(snap[:k * self.total], non_blocking=True)
            return
        for f in fields:
            i = _STATE_FIELDS.index(f)
            self.buffer[i * self.total:(i + 1) * self.total].copy_(
                snap[i * self.total:(i + 1) * self.total], non_blocking=True)
