"""Serving loop: keyframe-update requests from many camera streams.

Each registered stream keeps its keyframe image, a ring of neighbour frames
and its surfel state resident on the GPU.  A request brings one new
neighbour frame (image + pose) that replaces the oldest one in the ring, then
asks for the Gauss-Newton iterations on the stream's surfels and returns the
surfels and the per-pixel inverse depth.

Scheduling (host side, this module):
  * admission by memory: every admitted request owns a region of the
    response memory (pinned host memory of the pool's size, carved by a
    first-fit allocator) that its depth map and surfels are copied into; a
    request is admitted only when its region fits, otherwise it waits and is
    admitted as soon as completed requests release memory;
  * per-stream order: a stream never has two requests admitted or in
    flight, so each request sees the state left by the previous one, and a
    request that must wait for its stream holds no memory meanwhile (no
    head-of-line blocking of other streams behind it); among the streams
    that are free the oldest request is admitted first;
  * continuous batching: whenever an execution lane is free, every admitted
    request is packed into one batch and launched (one persistent fused
    kernel for the whole batch); batches on different lanes overlap on the
    device;
  * a request whose execution fails is completed with its error and its
    memory released; the rest of its batch is not affected by the scheduler;
  * on completion a request's response is copied out of its region (when
    the server keeps results) and the region released.

The executor does the device work.  HipExecutor uses the C ABI
(sgn_optimize_batch on per-lane contexts and streams); tests substitute a
CPU executor to check the scheduling logic without a GPU.
"""
from __future__ import annotations

import collections
import heapq
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Deque, Dict, List, Optional, Sequence

import numpy as np


@dataclass
class Request:
    stream: int
    arrival: float                       # host clock (time.perf_counter) at arrival
    frame_index: int                     # which prepared frame of the stream this request brings
    rid: int = 0
    admitted: float = 0.0
    launched: float = 0.0
    done: float = 0.0
    nbytes: int = 0
    offset: int = -1                     # response region in the pool (while admitted)
    error: Optional[str] = None
    result: Any = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class MemoryPool:
    """Byte budget of the response memory with first-fit placement: try_take
    returns the offset of a free region of n bytes (aligned to ALIGN) or None
    when none fits; give releases it.  Free neighbours merge."""

    ALIGN = 256

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.used = 0
        self.peak = 0
        self._free = [(0, self.budget)]          # sorted (offset, size)

    def _round(self, n: int) -> int:
        return (int(n) + self.ALIGN - 1) // self.ALIGN * self.ALIGN

    def try_take(self, n: int) -> Optional[int]:
        if n > self.budget:
            raise ValueError(f"request needs {n} bytes, more than the whole pool ({self.budget})")
        need = self._round(n)
        for i, (off, size) in enumerate(self._free):
            if size >= need:
                if size == need:
                    del self._free[i]
                else:
                    self._free[i] = (off + need, size - need)
                self.used += need
                self.peak = max(self.peak, self.used)
                return off
        return None

    def give(self, off: int, n: int):
        need = self._round(n)
        self.used -= need
        assert self.used >= 0
        import bisect
        i = bisect.bisect_left(self._free, (off, 0))
        self._free.insert(i, (off, need))
        # merge with the following and the preceding region
        if i + 1 < len(self._free) and self._free[i][0] + self._free[i][1] == self._free[i + 1][0]:
            self._free[i] = (self._free[i][0], self._free[i][1] + self._free[i + 1][1])
            del self._free[i + 1]
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] == self._free[i][0]:
            self._free[i - 1] = (self._free[i - 1][0], self._free[i - 1][1] + self._free[i][1])
            del self._free[i]


class Executor:
    """Device side of the server.  launch() enqueues one batch on a lane and
    returns a handle; poll() says whether it finished; finish() returns the
    per-request errors (None = success).  attach_memory() hands over the
    pool's size once (an executor allocates its response memory there);
    response() returns a completed request's own copy of its response."""

    lanes = 1

    def attach_memory(self, nbytes: int):
        pass

    def request_bytes(self, req: Request) -> int:
        raise NotImplementedError

    def response(self, req: Request):
        return None

    def launch(self, lane: int, batch: List[Request]) -> Any:
        raise NotImplementedError

    def poll(self, handle) -> bool:
        raise NotImplementedError

    def finish(self, handle) -> List[Optional[str]]:
        raise NotImplementedError


class Server:
    """keep_results: a completed request keeps its own copy of its response
    in Request.result (otherwise the response is dropped on completion)."""

    def __init__(self, executor: Executor, pool_bytes: int, max_batch: int = 32,
                 clock: Callable[[], float] = time.perf_counter, keep_results: bool = False):
        self.ex = executor
        self.pool = MemoryPool(pool_bytes)
        executor.attach_memory(self.pool.budget)
        self.max_batch = max_batch
        self.clock = clock
        self.keep_results = keep_results
        self.waiting: Dict[int, Deque[Request]] = {}            # per stream, not yet admitted
        self.n_waiting = 0
        self.admitted: Deque[Request] = collections.deque()    # admitted, not launched
        self.busy_streams: set = set()                         # admitted or in flight
        self.lanes_free = list(range(executor.lanes))
        self.inflight: List[tuple] = []                        # (handle, lane, batch)
        self.completed: List[Request] = []
        self.batches: List[int] = []
        self._rid = 0

    # -- requests ----------------------------------------------------------
    def submit(self, req: Request):
        self._rid += 1
        req.rid = self._rid
        req.nbytes = self.ex.request_bytes(req)
        if req.nbytes > self.pool.budget:
            raise ValueError(f"request needs {req.nbytes} bytes, more than the whole pool "
                             f"({self.pool.budget})")
        self.waiting.setdefault(req.stream, collections.deque()).append(req)
        self.n_waiting += 1

    def _admit(self):
        # the oldest waiting request of a stream with nothing admitted or in
        # flight, while its response region fits (no overtaking on memory)
        while self.n_waiting:
            head = None
            for s, q in self.waiting.items():
                if q and s not in self.busy_streams and (head is None or q[0].rid < head.rid):
                    head = q[0]
            if head is None:
                return
            off = self.pool.try_take(head.nbytes)
            if off is None:
                return
            self.waiting[head.stream].popleft()
            self.n_waiting -= 1
            head.offset = off
            head.admitted = self.clock()
            self.busy_streams.add(head.stream)
            self.admitted.append(head)

    def _launch(self):
        while self.lanes_free and self.admitted:
            batch = []
            while self.admitted and len(batch) < self.max_batch:
                batch.append(self.admitted.popleft())
            lane = self.lanes_free.pop(0)
            now = self.clock()
            for r in batch:
                r.launched = now
            try:
                h = self.ex.launch(lane, batch)
            except Exception as e:            # nothing was enqueued for this batch
                self.lanes_free.append(lane)
                self._complete(batch, [f"launch failed: {e}"] * len(batch))
                continue
            self.inflight.append((h, lane, batch))
            self.batches.append(len(batch))

    def _complete(self, batch, errors):
        now = self.clock()
        for r, err in zip(batch, errors):
            r.done = now
            r.error = err
            if err is None and self.keep_results:
                r.result = self.ex.response(r)
            self.pool.give(r.offset, r.nbytes)
            self.busy_streams.discard(r.stream)
            self.completed.append(r)

    def _reap(self):
        still = []
        for h, lane, batch in self.inflight:
            if self.ex.poll(h):
                try:
                    errors = self.ex.finish(h)
                except Exception as e:
                    errors = [f"execution failed: {e}"] * len(batch)
                self._complete(batch, errors)
                self.lanes_free.append(lane)
            else:
                still.append((h, lane, batch))
        self.inflight = still

    def tick(self):
        """One scheduler pass: reap finished batches, admit, launch."""
        self._reap()
        self._admit()
        self._launch()

    def idle(self) -> bool:
        return not (self.n_waiting or self.admitted or self.inflight)

    def drain(self, timeout: float = 60.0):
        t0 = self.clock()
        while not self.idle():
            self.tick()
            if self.clock() - t0 > timeout:
                raise TimeoutError("server did not drain")


def poisson_arrivals(rate: float, duration: float, n_streams: int, seed: int, frames_per_stream: int):
    """(time, stream, frame_index) for Poisson arrivals at `rate` per second
    over `duration` seconds, the stream picked uniformly."""
    rng = np.random.default_rng(seed)
    t = 0.0
    counters = [0] * n_streams
    out = []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        s = int(rng.integers(0, n_streams))
        out.append((t, s, counters[s] % frames_per_stream))
        counters[s] += 1
    return out


def run_trace(server: Server, trace, warmup: float = 0.0, idle_sleep: float = 2e-5):
    """Replay (t, stream, frame) arrivals in real time through the server.
    Returns the completed requests that arrived after `warmup` seconds."""
    t0 = server.clock()
    i = 0
    while i < len(trace) or not server.idle():
        now = server.clock() - t0
        while i < len(trace) and trace[i][0] <= now:
            t, s, fi = trace[i]
            server.submit(Request(stream=s, arrival=t0 + t, frame_index=fi))
            i += 1
        server.tick()
        if server.idle() and i < len(trace):
            wait = trace[i][0] - (server.clock() - t0)
            if wait > 0:
                time.sleep(min(wait, 1e-3))
        elif idle_sleep:
            time.sleep(idle_sleep)
    return [r for r in server.completed if r.arrival - t0 >= warmup]


def latency_stats(reqs: Sequence[Request]) -> Dict[str, float]:
    ok = [r for r in reqs if r.error is None]
    if not ok:
        return {"count": 0}
    lat = np.array([r.latency for r in ok]) * 1e3
    t_first = min(r.arrival for r in ok)
    t_last = max(r.done for r in ok)
    return {"count": len(ok), "errors": len(reqs) - len(ok),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
            "throughput_rps": len(ok) / max(t_last - t_first, 1e-9)}


# --------------------------------------------------------------------------
# GPU executor over the C ABI
# --------------------------------------------------------------------------

class CameraStream:
    """Resident device state of one camera stream."""

    def __init__(self, ctx, kf, extra_frames, storage: str = "f16"):
        import torch

        from . import engine
        self.dk = engine.DeviceKeyframe.from_scene(ctx, kf, storage=storage, render=True)
        self.n_nbr = self.dk.n_nbr
        self.oldest = 0
        self.first = True
        self.R = np.array(self.dk.R)
        self.t = np.array(self.dk.t)
        # prepared request frames (stored in the image dtype) and their poses
        self.frames = extra_frames["images"]          # device tensor (E, H, W) storage dtype
        self.frame_R = extra_frames["R"]
        self.frame_t = extra_frames["t"]

    @property
    def response_bytes(self) -> int:
        """A response: the inverse-depth map (H x W float32) and the surfels
        (8 x n float32 rows: id, nx, ny, nz, flags, cost, nvalid,
        last_update, the integer fields bit-cast)."""
        return self.dk.width * self.dk.height * 4 + self.dk.n_surfels * 8 * 4

    def response_views(self, slab, offset: int):
        """(depth, state) views of a response region of the pinned slab."""
        import torch
        H, W, n = self.dk.height, self.dk.width, self.dk.n_surfels
        d = slab[offset:offset + H * W * 4].view(torch.float32).view(H, W)
        st = slab[offset + H * W * 4:offset + H * W * 4 + 8 * n * 4].view(torch.float32).view(8, n)
        return d, st

    # checkpoint / resume
    def snapshot(self) -> Dict[str, np.ndarray]:
        """Host copy of everything the stream's next requests depend on: the
        surfel state (every field), the keyframe image and the neighbour-frame
        ring as stored (f32/f16/u8), the ring's poses, which slot is the
        oldest and whether the next request still initialises new surfels.
        Take it with no request of the stream in flight."""
        import torch
        torch.cuda.synchronize()
        st = self.dk.state
        snap = {f"state_{f}": getattr(st, f).cpu().numpy() for f in STATE_FIELDS}
        snap["kf_image"] = self.dk.kf_img.cpu().numpy()
        snap["nbr_images"] = self.dk.nbr_imgs.cpu().numpy()
        snap["R"] = self.R.copy()
        snap["t"] = self.t.copy()
        snap["oldest"] = np.array(self.oldest, np.int64)
        snap["first"] = np.array(self.first, np.bool_)
        return snap

    def restore(self, snap: Dict[str, np.ndarray]) -> None:
        """Load a snapshot taken from a stream of the same shape (image size,
        tile size, neighbour count, storage); raises ValueError otherwise and
        then changes nothing."""
        import torch
        st = self.dk.state
        targets = [(f"state_{f}", getattr(st, f)) for f in STATE_FIELDS]
        targets += [("kf_image", self.dk.kf_img), ("nbr_images", self.dk.nbr_imgs)]
        for key, dst in targets:
            if key not in snap:
                raise ValueError(f"snapshot lacks {key}")
            src = snap[key]
            if tuple(src.shape) != tuple(dst.shape) or src.dtype != torch.empty(0, dtype=dst.dtype).numpy().dtype:
                raise ValueError(f"snapshot {key}: {src.dtype}{tuple(src.shape)} does not fit "
                                 f"{dst.dtype}{tuple(dst.shape)}")
        if snap["R"].shape != self.R.shape or snap["t"].shape != self.t.shape:
            raise ValueError("snapshot poses do not fit the neighbour ring")
        torch.cuda.synchronize()
        for key, dst in targets:
            dst.copy_(torch.from_numpy(np.ascontiguousarray(snap[key])))
        self.R[...] = snap["R"]
        self.t[...] = snap["t"]
        self.oldest = int(snap["oldest"])
        self.first = bool(snap["first"])
        torch.cuda.synchronize()


STATE_FIELDS = ("inv_depth", "nx", "ny", "nz", "flags", "cost", "nvalid", "last_update")


def save_snapshot(path, snap: Dict[str, np.ndarray]) -> None:
    """Write a stream snapshot as an .npz archive (plain arrays, no pickles)."""
    np.savez(path, **snap)


def load_snapshot(path) -> Dict[str, np.ndarray]:
    """Read a stream snapshot written by save_snapshot."""
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def respond(cs: CameraStream, slab, req: Request, torch):
    """Enqueue the copies of a stream's depth map and surfel state into the
    request's response region on the current stream."""
    dk = cs.dk
    depth, state = cs.response_views(slab, req.offset)
    depth.copy_(dk.inv_depth_out, non_blocking=True)
    for k, src in enumerate((dk.state.inv_depth, dk.state.nx, dk.state.ny, dk.state.nz,
                             dk.state.flags.view(torch.float32), dk.state.cost,
                             dk.state.nvalid.view(torch.float32), dk.state.last_update.view(torch.float32))):
        state[k].copy_(src, non_blocking=True)


class HipExecutor(Executor):
    """Runs batches through sgn_optimize_batch on `lanes` contexts, each on
    its own torch stream (default priority)."""

    def __init__(self, streams: List[CameraStream], lanes: int = 2, iters: int = 15,
                 plan=None, pixels_per_lane: int = 4):
        import torch

        from . import surfgn as sg
        self.sg = sg
        self.torch = torch
        self.streams = streams
        self.lanes = lanes
        self.tstreams = [torch.cuda.Stream() for _ in range(lanes)]
        self.ctxs = [sg.Context(0, stream=s) for s in self.tstreams]
        self.params = sg.params(iters=iters)
        self.plan = plan
        # every plan here gives a 4x4 surfel the same lanes (16 lanes of one
        # pixel, or 4 lanes of four pixels), so a request's result is the
        # same, bitwise, alone and in any mix
        if pixels_per_lane == 4:
            self.small_plan = sg.plan(4, 4, 1, 0, 0, 1, groups=1)
            self.single_plan = sg.plan(4, 4, 0, 0, 0, 0, groups=1)
            # one wavefront per work item, the items split into one share
            # per XCD (batches of eight keyframes or more)
            self.large_plan = sg.plan(4, 4, 0, 0, 0, 1, groups=1)
        elif pixels_per_lane == 1:
            self.small_plan = sg.plan(2, 2, 1, 0, 0, 1, groups=1)
            self.single_plan = sg.plan(2, 2, 0, 0, 0, 0, groups=1)
            self.large_plan = sg.plan(2, 2, 1, 0, 0, 1, groups=4)
        else:
            raise ValueError("pixels_per_lane is 1 or 4")
        self.small_batch_surfels = 200_000
        self.slab = None

    def attach_memory(self, nbytes: int):
        """The response memory: one pinned host allocation of the pool's size."""
        self.slab = self.torch.empty(int(nbytes), dtype=self.torch.uint8, pin_memory=True)

    def request_bytes(self, req: Request) -> int:
        return self.streams[req.stream].response_bytes

    def response(self, req: Request):
        """The request's own copy of its response: (depth (H, W), surfels (8, n))."""
        d, st = self.streams[req.stream].response_views(self.slab, req.offset)
        return d.numpy().copy(), st.numpy().copy()

    def launch(self, lane: int, batch: List[Request]):
        torch = self.torch
        ts = self.tstreams[lane]
        items = []
        outs = []
        with torch.cuda.stream(ts):
            for r in batch:
                cs = self.streams[r.stream]
                dk = cs.dk
                slot = cs.oldest
                # the new frame replaces the oldest neighbour (device copy on this lane)
                dk.nbr_imgs[slot].copy_(cs.frames[r.frame_index], non_blocking=True)
                cs.R[slot] = cs.frame_R[r.frame_index]
                cs.t[slot] = cs.frame_t[r.frame_index]
                cs.oldest = (cs.oldest + 1) % cs.n_nbr
                view = self.sg.KeyframeView(dk.kf_img, [dk.nbr_imgs[i] for i in range(dk.n_nbr)],
                                            cs.R, cs.t, dk.K, dk.patch, dk.scale)
                it = self.sg.sgn_batch_item(view.c, dk.state.c,
                                            dk.is_new.data_ptr() if (cs.first and dk.is_new is not None) else None,
                                            dk.inv_depth_out.data_ptr(), None)
                cs.first = False
                items.append(it)
                outs.append(view)
            arr = None
            ctx = self.ctxs[lane].handle
            if len(items) == 1:
                # a lone request: the single-keyframe calls launch directly and
                # skip the batch table (same results, bitwise)
                it, view = items[0], outs[0]
                dk = self.streams[batch[0].stream].dk
                if it.is_new:
                    self.sg.sgn_init_from_neighbours(ctx, view.c, dk.state.c, it.is_new, self.params)
                self.sg.sgn_optimize_keyframe(ctx, view.c, dk.state.c, self.params, self.single_plan)
                self.sg.sgn_render_inverse_depth(ctx, view.c, dk.state.c, dk.inv_depth_out.data_ptr())
            else:
                plan = self.plan
                if plan is None:
                    # a small batch cannot fill the device with four groups per
                    # work item: use one group per wavefront there
                    total = sum(self.streams[r.stream].dk.n_surfels for r in batch)
                    plan = self.small_plan if total < self.small_batch_surfels else self.large_plan
                arr = self.sg.batch_array(items)
                self.sg.sgn_optimize_batch(ctx, arr, len(items), self.params, plan)
            # responses: depth map and surfels copied into each request's region
            for r in batch:
                respond(self.streams[r.stream], self.slab, r, torch)
            ev = torch.cuda.Event()
            ev.record(ts)
        return (ev, batch, outs, arr)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def finish(self, handle):
        ev, batch, _, _ = handle
        ev.synchronize()
        return [None] * len(batch)


class PlainExecutor(HipExecutor):
    """The plain form: one request at a time with the single-keyframe calls
    (init, non-persistent Gauss-Newton launch, render) on one lane."""

    def __init__(self, streams, iters: int = 15, pixels_per_lane: int = 4):
        super().__init__(streams, lanes=1, iters=iters, pixels_per_lane=pixels_per_lane)
        # the single-keyframe plan: one group per wavefront, one wavefront per item
        self.plain_plan = self.single_plan

    def launch(self, lane: int, batch: List[Request]):
        assert len(batch) == 1
        torch = self.torch
        ts = self.tstreams[0]
        r = batch[0]
        cs = self.streams[r.stream]
        dk = cs.dk
        ctx = self.ctxs[0]
        with torch.cuda.stream(ts):
            slot = cs.oldest
            dk.nbr_imgs[slot].copy_(cs.frames[r.frame_index], non_blocking=True)
            cs.R[slot] = cs.frame_R[r.frame_index]
            cs.t[slot] = cs.frame_t[r.frame_index]
            cs.oldest = (cs.oldest + 1) % cs.n_nbr
            view = self.sg.KeyframeView(dk.kf_img, [dk.nbr_imgs[i] for i in range(dk.n_nbr)],
                                        cs.R, cs.t, dk.K, dk.patch, dk.scale)
            if cs.first and dk.is_new is not None:
                self.sg.sgn_init_from_neighbours(ctx.handle, view.c, dk.state.c, dk.is_new.data_ptr(),
                                                 self.params)
            cs.first = False
            self.sg.sgn_optimize_keyframe(ctx.handle, view.c, dk.state.c, self.params,
                                          self.plain_plan)
            self.sg.sgn_render_inverse_depth(ctx.handle, view.c, dk.state.c, dk.inv_depth_out.data_ptr())
            respond(cs, self.slab, r, torch)
            ev = torch.cuda.Event()
            ev.record(ts)
        return (ev, batch, [view], None)


def make_streams(ctx, specs, extra: int = 4, storage: str = "f16", device="cuda"):
    """Camera streams from scene specs: the spec's neighbours fill the ring,
    `extra` more rendered views become the frames requests bring."""
    import dataclasses

    import torch

    from scenegen import make_keyframe
    out = []
    for sp in specs:
        big = make_keyframe(dataclasses.replace(sp, n_nbr=sp.n_nbr + extra), device=device)
        base = dataclasses.replace(big, nbr_images=big.nbr_images[:sp.n_nbr], R=big.R[:sp.n_nbr],
                                   t=big.t[:sp.n_nbr])
        cs = CameraStream(ctx, base, {"images": None, "R": big.R[sp.n_nbr:], "t": big.t[sp.n_nbr:]},
                          storage=storage)
        # request frames in the stream's storage dtype
        ex = big.nbr_images[sp.n_nbr:]
        if storage == "f32":
            cs.frames = ex.contiguous()
        else:
            from . import surfgn as sg
            from .engine import STORAGE, U8_SCALE
            tdt = torch.float16 if storage == "f16" else torch.uint8
            fr = torch.empty(ex.shape, dtype=tdt, device=ex.device)
            for i in range(ex.shape[0]):
                sg.sgn_quantize(ctx.handle, ex[i].data_ptr(), ex[i].stride(0),
                                sg.image_of(fr[i], 1.0 if storage == "f16" else U8_SCALE))
            cs.frames = fr
        out.append(cs)
    torch.cuda.synchronize()   # uploads and quantisation are done before any lane uses them
    return out


def serving_benchmark(n_streams: int = 32, rate: float = 200.0, duration: float = 6.0,
                      warmup: float = 1.0, storage: str = "f16", lanes: int = 2,
                      pool_bytes: int = 256 << 20, iters: int = 15, seed: int = 599,
                      specs=None, log=print, sweep=(), sweep_duration: float = 2.0,
                      sweep_warmup: float = 0.25, pixels_per_lane: int = 4):
    """Served (continuous batching) and plain (FIFO, one request at a time,
    single-keyframe calls) runs of the same Poisson trace at `rate`, then, on
    the same resident streams, shorter traces at each rate of `sweep`.
    Returns the latency / throughput statistics of both modes, the sweep's
    under "sweep" keyed by rate."""
    import torch

    from . import surfgn as sg
    from scenegen import stream_specs
    specs = specs if specs is not None else stream_specs(n_streams)
    extra = 4
    traces = [(rate, duration, warmup)] + [(r, sweep_duration, sweep_warmup) for r in sweep]
    out = {"trace": {"streams": len(specs), "rate_rps": rate, "seconds": duration,
                     "warmup_s": warmup, "iterations": iters, "storage": storage,
                     "pool_mb": pool_bytes >> 20, "lanes": lanes,
                     "requests": len(poisson_arrivals(rate, duration, len(specs), seed, extra))}}
    if sweep:
        out["sweep"] = {str(int(r) if float(r).is_integer() else r): {} for r in sweep}
    for mode in ("served", "plain"):
        ctx = sg.Context(0)
        streams = make_streams(ctx, specs, extra=extra, storage=storage)
        torch.cuda.synchronize()
        ex = HipExecutor(streams, lanes=lanes, iters=iters, pixels_per_lane=pixels_per_lane) \
            if mode == "served" else PlainExecutor(streams, iters=iters, pixels_per_lane=pixels_per_lane)
        srv = Server(ex, pool_bytes=pool_bytes, max_batch=32 if mode == "served" else 1)
        # warm the kernels and graphs on a short burst outside the measured trace
        for s in range(min(4, len(streams))):
            srv.submit(Request(stream=s, arrival=srv.clock(), frame_index=0))
        srv.drain()
        for k, (r_rate, r_dur, r_warm) in enumerate(traces):
            srv.completed.clear()
            srv.batches.clear()
            srv.pool.peak = 0
            trace = poisson_arrivals(r_rate, r_dur, len(specs), seed + k, extra)
            done = run_trace(srv, trace, warmup=r_warm)
            st = latency_stats(done)
            st["offered_rps"] = r_rate
            sf = sum(streams[r.stream].dk.n_surfels * streams[r.stream].dk.n_nbr for r in done
                     if r.error is None) * iters
            span = max(r.done for r in done) - min(r.arrival for r in done) if done else 1.0
            st["surfel_frame_updates_per_s"] = sf / span
            st["mean_batch"] = float(np.mean(srv.batches)) if srv.batches else 0.0
            st["pool_peak_mb"] = srv.pool.peak / 2 ** 20
            if k == 0:
                out[mode] = st
            else:
                out["sweep"][str(int(r_rate) if float(r_rate).is_integer() else r_rate)][mode] = st
            log(f"{mode} at {r_rate:g} req/s: {st}")
        for c in getattr(ex, "ctxs", []):
            c.close()
        ctx.close()
        del streams, ex, srv
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return out
