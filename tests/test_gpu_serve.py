"""Serving on the GPU: served responses against the oracle over consecutive
requests (carried state, 1920x1080 included), a request's result is the same
alone and in the mix (bitwise, same plan), responses carry the device state,
every request keeps its own response, and a short trace completes with
admission binding."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from scenegen import stream_specs

pytestmark = pytest.mark.gpu


def _specs():
    # six streams of the serving workload, reduced to 320x240 / 640x480 for speed
    out = []
    for i, sp in enumerate(stream_specs(6)):
        W, H = ((320, 240), (640, 480))[i % 2]
        out.append(dataclasses.replace(sp, width=W, height=H))
    return out


def test_alone_equals_mix():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01997_amd import serve
    from paper_1910_01997_amd import surfgn as sg
    specs = _specs()
    results = {}
    for mode in ("mix", "alone"):
        ctx = sg.Context(0)
        streams = serve.make_streams(ctx, specs, extra=2)
        ex = serve.HipExecutor(streams, lanes=2, iters=8)
        srv = serve.Server(ex, pool_bytes=1 << 30, max_batch=32 if mode == "mix" else 1, keep_results=True)
        for s in range(len(specs)):
            srv.submit(serve.Request(stream=s, arrival=srv.clock(), frame_index=1))
            if mode == "alone":
                srv.drain()
        srv.drain()
        assert all(r.error is None for r in srv.completed)
        if mode == "mix":
            assert max(srv.batches) > 1
        else:
            assert max(srv.batches) == 1
        results[mode] = {r.stream: r.result for r in srv.completed}
        # the response holds the device state
        for r in srv.completed:
            dk = streams[r.stream].dk
            assert np.array_equal(r.result[1][0], dk.state.inv_depth.cpu().numpy())
        for c in ex.ctxs:
            c.close()
        ctx.close()
    for s in range(len(specs)):
        assert np.array_equal(results["mix"][s][0], results["alone"][s][0]), f"depth of stream {s}"
        assert np.array_equal(results["mix"][s][1], results["alone"][s][1]), f"surfels of stream {s}"


def test_short_trace_with_binding_admission():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01997_amd import serve
    specs = _specs()
    res = serve.serving_benchmark(specs=specs, rate=300.0, duration=1.5, warmup=0.2,
                                  pool_bytes=6 << 20, iters=8)
    for mode in ("served", "plain"):
        st = res[mode]
        assert st["count"] > 50 and st["errors"] == 0
        assert st["pool_peak_mb"] <= 6.0 + 1e-9
        assert st["p99_ms"] >= st["p50_ms"] > 0


def test_snapshot_resume_equals_uninterrupted(tmp_path):
    """Checkpoint / resume: a stream snapshot written to .npz after its first
    request and loaded into freshly built streams gives, for the next
    requests, bitwise the responses of the uninterrupted run."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01997_amd import serve
    from paper_1910_01997_amd import surfgn as sg
    specs = _specs()[:2]

    def run(streams, frames):
        ex = serve.HipExecutor(streams, lanes=1, iters=6)
        srv = serve.Server(ex, pool_bytes=1 << 30, max_batch=1, keep_results=True)
        out = {}
        for f in frames:
            for s in range(len(streams)):
                srv.submit(serve.Request(stream=s, arrival=srv.clock(), frame_index=f))
                srv.drain()
        assert all(r.error is None for r in srv.completed)
        for r in srv.completed:
            out[(r.stream, r.frame_index)] = r.result
        for c in ex.ctxs:
            c.close()
        return out

    print("case snapshot after one request, resume two more", flush=True)
    ctx = sg.Context(0)
    streams = serve.make_streams(ctx, specs, extra=3)
    run(streams, [0])
    paths = []
    for s, cs in enumerate(streams):
        paths.append(tmp_path / f"stream{s}.npz")
        serve.save_snapshot(paths[-1], cs.snapshot())
    uninterrupted = run(streams, [1, 2])
    ctx.close()

    ctx2 = sg.Context(0)
    fresh = serve.make_streams(ctx2, specs, extra=3)
    for cs, p in zip(fresh, paths):
        cs.restore(serve.load_snapshot(p))
    resumed = run(fresh, [1, 2])
    assert uninterrupted.keys() == resumed.keys()
    for k in uninterrupted:
        assert np.array_equal(uninterrupted[k][0], resumed[k][0]), f"depth {k}"
        assert np.array_equal(uninterrupted[k][1], resumed[k][1]), f"surfels {k}"
    # a snapshot of another shape is refused and changes nothing
    before = fresh[0].snapshot()
    with pytest.raises(ValueError):
        fresh[0].restore(serve.load_snapshot(paths[1]))
    after = fresh[0].snapshot()
    assert all(np.array_equal(before[k], after[k]) for k in before)
    ctx2.close()


class _RingKeyframe:
    """What one served request saw, on the host: the keyframe image, the
    neighbour ring after the request's frame replaced the oldest one, the
    ring's poses, intrinsics and tile edge (the attributes the parity helpers
    read)."""

    def __init__(self, K, patch, width, height, kf, nbr, R, t):
        self.K, self.patch, self.width, self.height = K, patch, width, height
        self.R, self.t = np.array(R), np.array(t)
        self._kf, self._nb = kf, nbr

    @property
    def grid(self):
        return (self.width // self.patch, self.height // self.patch)

    def dequantized_images(self):
        return self._kf, self._nb


def test_served_responses_match_the_oracle_across_requests():
    """Three consecutive requests on each of three streams of the serving
    workload (1920x1080 with 5 neighbours, 320x240 with 5 and with 9), served
    together by continuous batching.  Every response (surfels and depth map)
    is compared with the oracle run on the ring images and poses that request
    saw, from the state the previous response carried (the first request from
    the stream's initial state, its new surfels initialised from neighbours)."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import oracle
    from paper_1910_01997_amd import serve
    from paper_1910_01997_amd import surfgn as sg
    from tests.parity import assert_parity, assert_render, check_parity
    specs = [stream_specs(32)[i] for i in (20, 12, 5)]
    assert (specs[0].width, specs[0].height) == (1920, 1080)
    print("case serving parity: streams 1920x1080 N5, 320x240 N5, 320x240 N9, 3 requests each", flush=True)
    ctx = sg.Context(0)
    streams = serve.make_streams(ctx, specs, extra=3)
    snaps = [cs.snapshot() for cs in streams]
    frames = [cs.frames.double().cpu().numpy() * cs.dk.scale for cs in streams]
    ex = serve.HipExecutor(streams, lanes=2, iters=15)
    srv = serve.Server(ex, pool_bytes=1 << 30, max_batch=32, keep_results=True)
    for f in range(3):
        for s in range(len(streams)):
            srv.submit(serve.Request(stream=s, arrival=srv.clock(), frame_index=f))
    srv.drain()
    assert all(r.error is None for r in srv.completed)
    assert max(srv.batches) > 1                      # requests of several streams ran together
    resp = {(r.stream, r.frame_index): r.result for r in srv.completed}
    for c in ex.ctxs:
        c.close()
    prm = oracle.OracleParams(iters=15)
    for s, cs in enumerate(streams):
        dk, snap = cs.dk, snaps[s]
        n = dk.n_surfels
        kf = snap["kf_image"].astype(np.float64) * dk.scale
        ring = snap["nbr_images"].astype(np.float64) * dk.scale
        R, t = snap["R"].copy(), snap["t"].copy()
        st_id = snap["state_inv_depth"]
        st_n = np.stack([snap["state_nx"], snap["state_ny"], snap["state_nz"]], 1)
        st_flags = snap["state_flags"].astype(np.uint32)
        is_new = dk.is_new.cpu().numpy() if dk.is_new is not None else None
        for f in range(3):
            slot = f % dk.n_nbr
            ring[slot] = frames[s][f]
            R[slot], t[slot] = cs.frame_R[f], cs.frame_t[f]
            hk = _RingKeyframe(dk.K, dk.patch, dk.width, dk.height, kf, ring.copy(), R, t)
            depth, state = resp[(s, f)]
            dev = {"inv_depth": state[0].copy(), "n": np.ascontiguousarray(state[1:4].T),
                   "flags": state[4].view(np.uint32).copy(), "cost": state[5].copy(),
                   "nvalid": state[6].view(np.int32).astype(np.int64)}
            label = f"served stream {s} {dk.width}x{dk.height} N={dk.n_nbr} request {f}"
            res = check_parity(hk, dev, st_id, st_n, is_new if f == 0 else None, prm, label=label,
                               init_flags=st_flags)
            assert_parity(res, label=label, max_unstable=SERVE_MAX_UNSTABLE[s])
            assert_render(hk, dev, depth)
            # the next request starts from this response's state
            st_id, st_n, st_flags = dev["inv_depth"], dev["n"], dev["flags"]
        assert dev["inv_depth"].size == n
    ctx.close()


# the probe's unstable fraction on the three streams (measured over the three
# requests: 0.072-0.145, 0.046-0.113, 0.034-0.104)
SERVE_MAX_UNSTABLE = (0.17, 0.14, 0.13)
